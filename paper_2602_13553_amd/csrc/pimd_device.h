// Device helpers shared by the step kernels of libpimd.so (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include "pimd_internal.h"

namespace pimd {

// --------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) and Box-Muller.
// --------------------------------------------------------------------------
// Each round takes two 32 x 32 -> 64-bit products (one v_mad_u64_u32 each);
// the key is wave-uniform, so its Weyl bumps stay in scalar registers.
__device__ __forceinline__ void philox4x32_10(unsigned c[4], unsigned k0, unsigned k1)
{
    const unsigned M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const unsigned W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const unsigned long long p0 = (unsigned long long)M0 * c[0];
        const unsigned long long p1 = (unsigned long long)M1 * c[2];
        const unsigned n0 = (unsigned)(p1 >> 32) ^ c[1] ^ k0;
        const unsigned n2 = (unsigned)(p0 >> 32) ^ c[3] ^ k1;
        c[0] = n0; c[1] = (unsigned)p1; c[2] = n2; c[3] = (unsigned)p0;
        k0 += W0; k1 += W1;
    }
}

// The uniform of a word w: n = w + 1 in [1, 2^32], u = n 2^-32 on (0, 1].

// -2 ln u for u = n 2^-32.  With n = 2^e m, m in [sqrt(1/2), sqrt(2)):
// ln u = (e - 32) ln 2 + 2 atanh(s), s = (m - 1)/(m + 1), |s| <= 0.1716, and
// atanh(s) = s (1 + s^2/3 + s^4/5 + ...) summed to s^22 (next term < 2^-60).
__device__ __forceinline__ double neg2log_u(unsigned w)
{
    const double n = (double)w + 1.0;                          // exact
    int e = __builtin_amdgcn_frexp_exp(n);                     // n = 2^e * m0, m0 in [0.5, 1)
    double m = __builtin_amdgcn_frexp_mant(n);
    if (m < 0.70710678118654752440) { m *= 2.0; e -= 1; }      // m in [sqrt(1/2), sqrt(2))
    const double num = m - 1.0, den = m + 1.0;
    double r = __builtin_amdgcn_rcp(den);                      // two Newton steps
    r = fma(fma(-den, r, 1.0), r, r);
    r = fma(fma(-den, r, 1.0), r, r);
    double s = num * r;
    s = fma(fma(-den, s, num), r, s);                          // residual correction
    const double s2 = s * s;
    double p = 1.0 / 23.0;
    p = fma(p, s2, 1.0 / 21.0);
    p = fma(p, s2, 1.0 / 19.0);
    p = fma(p, s2, 1.0 / 17.0);
    p = fma(p, s2, 1.0 / 15.0);
    p = fma(p, s2, 1.0 / 13.0);
    p = fma(p, s2, 1.0 / 11.0);
    p = fma(p, s2, 1.0 / 9.0);
    p = fma(p, s2, 1.0 / 7.0);
    p = fma(p, s2, 1.0 / 5.0);
    p = fma(p, s2, 1.0 / 3.0);
    const double lnm = 2.0 * fma(s * s2, p, s);
    // ln 2 = LN2_HI + LN2_LO, LN2_HI = ln 2 truncated to 40 fraction bits (so
    // that k LN2_HI is exact for |k| < 2^12)
    const double LN2_HI = 0x1.62e42fefa2p-1, LN2_LO = 0x1.9ef35793c7673p-41;
    const double k = (double)(e - 32);
    const double lnu = fma(k, LN2_HI, fma(k, LN2_LO, lnm));
    return -2.0 * lnu;
}

// sin and cos of 2 pi u for u = n 2^-32.  The octant q = floor(8u) and the
// offset inside it come exactly from the integer n; the angle t in [0, pi/4]
// (measured from the nearer octant edge) goes through Taylor series to t^19
// and t^20 (truncation < 2^-64), then q maps (sin t, cos t) back.
__device__ __forceinline__ void sincos_2pi_u(unsigned w, double &sn, double &cs)
{
    const unsigned long long n = (unsigned long long)w + 1ULL;  // [1, 2^32]
    const unsigned q = (unsigned)(n >> 29);                     // 0..8
    const unsigned rem = (unsigned)n & ((1u << 29) - 1u);
    const bool odd = (q & 1u) != 0u;
    const unsigned tq = odd ? (1u << 29) - rem : rem;
    const double t = (double)tq * (0.78539816339744830962 * 0x1p-29);
    const double t2 = t * t;
    double ps = -1.0 / 121645100408832000.0;                   // -1/19!
    ps = fma(ps, t2, 1.0 / 355687428096000.0);
    ps = fma(ps, t2, -1.0 / 1307674368000.0);
    ps = fma(ps, t2, 1.0 / 6227020800.0);
    ps = fma(ps, t2, -1.0 / 39916800.0);
    ps = fma(ps, t2, 1.0 / 362880.0);
    ps = fma(ps, t2, -1.0 / 5040.0);
    ps = fma(ps, t2, 1.0 / 120.0);
    ps = fma(ps, t2, -1.0 / 6.0);
    const double S = fma(t * t2, ps, t);
    double pc = 1.0 / 2432902008176640000.0;                    // 1/20!
    pc = fma(pc, t2, -1.0 / 6402373705728000.0);
    pc = fma(pc, t2, 1.0 / 20922789888000.0);
    pc = fma(pc, t2, -1.0 / 87178291200.0);
    pc = fma(pc, t2, 1.0 / 479001600.0);
    pc = fma(pc, t2, -1.0 / 3628800.0);
    pc = fma(pc, t2, 1.0 / 40320.0);
    pc = fma(pc, t2, -1.0 / 720.0);
    pc = fma(pc, t2, 1.0 / 24.0);
    pc = fma(pc, t2, -0.5);
    const double C = fma(t2, pc, 1.0);
    // angle = p pi/2 + (odd ? pi/2 - t : t), p = (q >> 1) & 3
    const double bs = odd ? C : S, bc = odd ? S : C;
    const unsigned p = (q >> 1) & 3u;
    sn = (p == 0u) ? bs : (p == 1u) ? bc : (p == 2u) ? -bs : -bc;
    cs = (p == 0u) ? bc : (p == 1u) ? -bs : (p == 2u) ? -bc : bs;
}

// The barostat's own noise takes this index in place of an atom's.
constexpr unsigned kBaroNoiseIndex = 0xFFFFFFFFu;

// Three N(0,1) deviates for atom i, mode k, step s and O step q of the step
// (0, or 1 for OBABO's second): counter (i, k, s mod 2^32, s / 2^32 + q 2^31),
// key (seed mod 2^32, seed / 2^32); Box-Muller (z0, z1) from (u0, u1), z2
// from (u2, u3).
__device__ __forceinline__ void gauss3(unsigned long long seed, unsigned i, unsigned k,
                                       unsigned long long s, double z[3], unsigned q = 0u)
{
    unsigned c[4] = {i, k, (unsigned)s, (unsigned)(s >> 32) | (q << 31)};
    philox4x32_10(c, (unsigned)seed, (unsigned)(seed >> 32));
    const double r0 = sqrt(neg2log_u(c[0]));
    const double r2 = sqrt(neg2log_u(c[2]));
    double s1, c1, s3, c3;
    sincos_2pi_u(c[1], s1, c1);
    sincos_2pi_u(c[3], s3, c3);
    z[0] = r0 * c1;
    z[1] = r0 * s1;
    z[2] = r2 * c3;
}

// --------------------------------------------------------------------------
// Block reductions (fixed order).
// --------------------------------------------------------------------------
// Wave butterflies, then the kBlock/64 wave results in index order: the
// same order on every call, two barriers per reduction.
template <int NV>
__device__ inline void block_sum(double (&v)[NV], double *red /* >= NV * kBlock/64 */)
{
    constexpr int NW = kBlock / 64;
    const int t = threadIdx.x, w = t >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double x = v[q];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
        v[q] = x;
    }
    if ((t & 63) == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) red[q * NW + w] = v[q];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double x = red[q * NW];
#pragma unroll
        for (int u = 1; u < NW; ++u) x += red[q * NW + u];
        v[q] = x;
    }
    __syncthreads();
}

// Cell of an active atom's centroid c in the periodic cell grid, stored in
// cinfo with the integer box index of the unwrapped centroid (the list build
// forms image shifts from integers alone).  A plain store per atom: the cell
// lists themselves are built by k_finalize, and only at a rebuild.
// Non-finite centroids land in a clamped (valid) cell; the non-finite flag of
// the step catches them.  Every atom's (cell, box index) pair places it within
// rounding of its centroid, which the list build's stencil margin absorbs.
// box, icw: the box lengths and cells per unit length to bin in.
__device__ inline int cell_of_in(const FusedArgs &a, int ia, const double c[3], const double *box,
                                 const double *icw)
{
    int cc[3], nb[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double L = box[d];
        const double fl = floor(c[d] / L);
        const double w = c[d] - L * fl;
        // w may round to L itself: the centroid then lies at the top of box fl
        int q = (w < L) ? (w >= 0.0 ? (int)(w * icw[d]) : 0) : a.nc[d] - 1;
        q = q < 0 ? 0 : (q >= a.nc[d] ? a.nc[d] - 1 : q);
        cc[d] = q;
        nb[d] = (fl > -1e6 && fl < 1e6) ? (int)fl : 0;
    }
    const int cell = (cc[2] * a.nc[1] + cc[1]) * a.nc[0] + cc[0];
    a.cinfo[ia] = make_int4(cell, nb[0], nb[1], nb[2]);
    return cell;
}

__device__ inline int cell_of(const FusedArgs &a, int ia, const double c[3])
{
    return cell_of_in(a, ia, c, a.box, a.icw);
}
// At a rebuild, builds the centroid cell lists from the cells recorded by
// the step pass, each cell's atoms in increasing index order, without a sort:
// wave w takes the contiguous atom range [w*na/4, (w+1)*na/4) in chunks of 64
// in index order.  A first pass counts, per wave, the atoms of each cell; the
// place of wave w's atoms in cell q starts after the atoms of waves < w.  The
// second pass places each atom at its wave's running offset in its cell plus
// its rank among the lower lanes of its chunk that share the cell (groups of
// equal cells from one ballot per cell-index bit), and writes its entry with
// its centroid and box indices.  Decides whether the cells can serve this
// rebuild: no cell over capacity, and a stencil of 2R+1 cells per dim that
// does not wrap onto itself.  One block; no atomics.
// lanes of the wave whose value of q equals this lane's (ok lanes only)
__device__ __forceinline__ unsigned long long same_cell_lanes(bool ok, int q, int nbits)
{
    unsigned long long same = __ballot(ok);
    for (int b = 0; b < nbits; ++b) {
        const bool bit = ((q >> b) & 1) != 0;
        const unsigned long long m = __ballot(ok && bit);
        same &= bit ? m : ~m;
    }
    return same;
}

// icw: cells per unit length of the box the centroids were binned in.
__device__ inline void cells_finalize(const FusedArgs &a, const double *icw, double rlist,
                                      int *scnt /* [4][ncell] */, int *sflag)
{
    static_assert(kBlock == 256, "four waves split the atoms");
    const int t = threadIdx.x, w = t >> 6, lane = t & 63;
    const int ncell = a.ncell, cap = a.cell_cap, na = a.n_active;
    Ctl *c = a.ctl;
    for (int q = t; q < 4 * ncell; q += kBlock) scnt[q] = 0;
    if (t == 0) sflag[0] = 0;
    int nbits = 0;
    while ((1 << nbits) < ncell) ++nbits;
    const int per = (na + 3) / 4;
    const int lo = min(na, w * per), hi = min(na, lo + per);
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int *mine = scnt + w * ncell;
    __syncthreads();
    // pass 1: per-wave counts (the lowest lane of each equal-cell group adds
    // the group's size; the groups of one chunk have distinct cells)
    constexpr int U = 16;
    for (int i0 = lo; i0 < hi; i0 += 64 * U) {
        int qv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u * 64 + lane;
            qv[u] = i < hi ? a.cinfo[i].x : -1;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (i0 + u * 64 >= hi) break;                    // uniform over the wave
            const bool ok = qv[u] >= 0;
            const unsigned long long same = same_cell_lanes(ok, qv[u], nbits);
            if (ok && (same & below) == 0) mine[qv[u]] += __popcll(same);
        }
    }
    __syncthreads();
    // offsets of each wave in each cell, totals, capacity
    for (int q = t; q < ncell; q += kBlock) {
        int o = 0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int v = scnt[u * ncell + q];
            scnt[u * ncell + q] = o;
            o += v;
        }
        a.cell_scnt[q] = o;
        if (o > cap) sflag[0] = 1;
    }
    __syncthreads();
    bool ok_all = sflag[0] == 0;
    int R[3] = {0, 0, 0};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        // a relative margin covers centroids placed within rounding of a cell face
        const double rr = rlist * icw[d] * (1.0 + 1e-12);
        if (rr > 0.0 && rr <= 0.5 * (double)(a.nc[d] - 1))
            R[d] = (int)ceil(rr);
        else
            ok_all = false;
        if (2 * R[d] + 1 > a.nc[d]) ok_all = false;
    }
    if (ok_all) {
        // pass 2: placement in index order, entries written directly
        constexpr int V = 8;
        for (int i0 = lo; i0 < hi; i0 += 64 * V) {
            int4 ci[V];
            double cx[V], cy[V], cz[V];
#pragma unroll
            for (int u = 0; u < V; ++u) {
                const int i = i0 + u * 64 + lane;
                const int ii = i < hi ? i : lo;
                ci[u] = i < hi ? a.cinfo[ii] : make_int4(-1, 0, 0, 0);
                cx[u] = a.cent[ii * 3]; cy[u] = a.cent[ii * 3 + 1]; cz[u] = a.cent[ii * 3 + 2];
            }
#pragma unroll
            for (int u = 0; u < V; ++u) {
                if (i0 + u * 64 >= hi) break;                // uniform over the wave
                const int q = ci[u].x;
                const bool ok = q >= 0;
                const unsigned long long same = same_cell_lanes(ok, q, nbits);
                if (ok) {
                    const int slot = mine[q] + __popcll(same & below);
                    CellEntry ce;
                    ce.c[0] = cx[u]; ce.c[1] = cy[u]; ce.c[2] = cz[u];
                    ce.j = i0 + u * 64 + lane;
                    ce.nb[0] = ci[u].y; ce.nb[1] = ci[u].z; ce.nb[2] = ci[u].w;
                    ce.pad = 0;
                    a.cell_ent[(size_t)q * cap + slot] = ce;
                }
                // every lane has read its offset before the group's leader moves it
                if (ok && (same & below) == 0) mine[q] += __popcll(same);
            }
        }
    }
    if (t == 0) {
        c->cell_ok = ok_all ? 1 : 0;
        c->cell_R[0] = R[0];
        c->cell_R[1] = R[1];
        c->cell_R[2] = R[2];
    }
}


// Sums of NS values and maxima of NM values in one exchange (one barrier).
// The caller passes a barrier before red is written again.
template <int NS, int NM>
__device__ inline void block_sum_max(double (&sv)[NS], double (&mv)[NM],
                                     double *red /* >= (NS + NM) * kBlock/64 */)
{
    constexpr int NW = kBlock / 64;
    const int t = threadIdx.x, w = t >> 6;
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        double x = sv[q];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
        sv[q] = x;
    }
#pragma unroll
    for (int q = 0; q < NM; ++q) {
        double x = mv[q];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o));
        mv[q] = x;
    }
    if ((t & 63) == 0) {
#pragma unroll
        for (int q = 0; q < NS; ++q) red[q * NW + w] = sv[q];
#pragma unroll
        for (int q = 0; q < NM; ++q) red[(NS + q) * NW + w] = mv[q];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        double x = red[q * NW];
#pragma unroll
        for (int u = 1; u < NW; ++u) x += red[q * NW + u];
        sv[q] = x;
    }
#pragma unroll
    for (int q = 0; q < NM; ++q) {
        double x = red[(NS + q) * NW];
#pragma unroll
        for (int u = 1; u < NW; ++u) x = fmax(x, red[(NS + q) * NW + u]);
        mv[q] = x;
    }
}

template <int NV>
__device__ inline void block_maxv(double (&v)[NV], double *red /* >= NV * kBlock/64 */)
{
    constexpr int NW = kBlock / 64;
    const int t = threadIdx.x, w = t >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double x = v[q];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o));
        v[q] = x;
    }
    if ((t & 63) == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) red[q * NW + w] = v[q];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double x = red[q * NW];
#pragma unroll
        for (int u = 1; u < NW; ++u) x = fmax(x, red[q * NW + u]);
        v[q] = x;
    }
    __syncthreads();
}

__device__ inline double block_max(double v, double *red)
{
    constexpr int NW = kBlock / 64;
    const int t = threadIdx.x, w = t >> 6;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    if ((t & 63) == 0) red[w] = v;
    __syncthreads();
    v = red[0];
#pragma unroll
    for (int u = 1; u < NW; ++u) v = fmax(v, red[u]);
    __syncthreads();
    return v;
}

}  // namespace pimd
