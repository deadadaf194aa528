// Bosonic exchange springs (the bosonic fix of Sec. III.C; the recursion of
// Hirshberg et al. 2019, evaluated in O(N^2) like Feldman and Hirshberg's
// algorithm, both cited by the paper).
//
// N identical particles of P beads.  The springs inside each particle's ring
// (bead j to j+1, j < P-1) are those of distinguishable particles; the link
// from bead P-1 of particle l to bead 0 of particle l' is summed over exchange
// cycles by the recursion over the cycle that holds the last particle,
//   exp(-beta_n V[n]) = (1/n) sum_{k=1..n} exp(-beta_n (E[n,k] + V[n-k])),
// E[n,k] the single ring through particles n-k..n-1 (0-based), V[0] = 0.
//
// Every term of V[n] holds the inner-ring energies of all of particles
// 0..n-1 once, so V[n] = sum_{l<n} eint[l] + V'[n], with V' the same
// recursion over the links alone (E'[n,k]: chain links n-k..n-2 plus the
// closing link n-1 -> n-k).  The kernels run V' and add the inner energies
// at the end, so no ring weight sees them.  The chain sums are differences of
// double-double prefix sums and V' is carried in double-double, so each
// weight's exponent E' + V'[n-k] - V'[n] is formed to the rounding of its
// own size, not of V_B's.
//
//   k_boson_inner : inner-ring spring forces (sets f) and energies, one
//                   thread per particle
//   k_boson_seq   : one block: prefix sums, the forward recursion (V', the
//                   ring weights w[n,k] into scratch, the weighted energy EV'
//                   of the primitive estimator) and its adjoint (adj[n] =
//                   dV'[N]/dV'[n]); sequential in n, parallel in k
//   k_boson_rows  : one block per n: q[n,k] = adj[n] w[n,k] (the probability
//                   of ring (n,k)'s closing link), and its suffix sums over k
//   k_boson_links : one wave per particle: the chain links' probabilities
//                   (sums of those suffix sums) and the link forces on the
//                   particle's first and last beads
#include "../../include/pimd.h"
#include "pimd_internal.h"
#include "pimd_device.h"

#include <cmath>
#include <mutex>

namespace pimd {

// The allocation-free entry point's scratch (pimd_boson_spring_noalloc): one
// copy per device, 2.1 MB, held until the process ends.  Host code reaches it
// only through the per-device address from hipGetSymbolAddress (in host code
// the array's name is a host-side stand-in, not a device address).
constexpr int kBosonNoAllocMaxN = 512;
static __device__ __align__(256) double scratch[boson_scr_doubles(kBosonNoAllocMaxN)];

namespace {

constexpr int kSeq = 256;   // threads of the sequential kernel
constexpr int kSeqU = (kBosonMaxN + kSeq - 1) / kSeq;   // k per thread and stage

__device__ __forceinline__ size_t tri_row(int n) { return (size_t)n * (size_t)(n - 1) / 2; }

__device__ __forceinline__ size_t bidx(const BosonArgs &a, int j, int l, int d)
{
    return a.layout ? ((size_t)l * 3 + d) * a.P + j : ((size_t)j * a.N + l) * 3 + d;
}

// a - b under the minimum image in each periodic dimension
__device__ __forceinline__ double mic(double a, double b, double L)
{
    const double u = a - b;
    return L > 0.0 ? u - L * rint(u / L) : u;
}

// --- double-double arithmetic (error-free sums; no products involved) ---
struct DD {
    double hi, lo;
};

__device__ __forceinline__ DD two_sum(double a, double b)
{
    const double s = a + b;
    const double bb = s - a;
    return {s, (a - (s - bb)) + (b - bb)};
}

__device__ __forceinline__ DD dd_add(DD a, DD b)
{
    const DD s = two_sum(a.hi, b.hi);
    const double lo = s.lo + (a.lo + b.lo);
    const double hi = s.hi + lo;
    return {hi, lo - (hi - s.hi)};
}

__device__ __forceinline__ DD dd_add1(DD a, double b)
{
    const DD s = two_sum(a.hi, b);
    const double lo = s.lo + a.lo;
    const double hi = s.hi + lo;
    return {hi, lo - (hi - s.hi)};
}

// a - b, rounded once (to the rounding of the difference's own size)
__device__ __forceinline__ double dd_diff(DD a, DD b)
{
    const DD s = two_sum(a.hi, -b.hi);
    return s.hi + (s.lo + (a.lo - b.lo));
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ double wave_min(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
    return v;
}

// Block reductions of the sequential kernel (kSeq threads); every thread gets
// the result.  The waves' values are combined in wave order.
__device__ __forceinline__ double seq_min(double v, double *red)
{
    constexpr int NW = kSeq / 64;
    v = wave_min(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = red[0];
#pragma unroll
    for (int u = 1; u < NW; ++u) r = fmin(r, red[u]);
    __syncthreads();
    return r;
}

__device__ __forceinline__ void seq_sum2(double &a, double &b, double *red)
{
    constexpr int NW = kSeq / 64;
    a = wave_sum(a);
    b = wave_sum(b);
    if ((threadIdx.x & 63) == 0) {
        red[threadIdx.x >> 6] = a;
        red[NW + (threadIdx.x >> 6)] = b;
    }
    __syncthreads();
    double ra = red[0], rb = red[NW];
#pragma unroll
    for (int u = 1; u < NW; ++u) {
        ra += red[u];
        rb += red[NW + u];
    }
    __syncthreads();
    a = ra;
    b = rb;
}

// Inner-ring springs: forces on every bead (overwrites f) and each particle's
// inner spring energy eint[l] = kspring sum_j |x_{j+1} - x_j|^2.
__global__ __launch_bounds__(kBlock) void k_boson_inner(BosonArgs a)
{
    const int l = blockIdx.x * kBlock + threadIdx.x;
    if (l >= a.N) return;
    const int P = a.P;
    const double k2 = 2.0 * a.ks;
    double e = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        double prev = 0.0, cur = a.x[bidx(a, 0, l, d)];
        for (int j = 0; j < P; ++j) {
            const double next = (j + 1 < P) ? a.x[bidx(a, j + 1, l, d)] : 0.0;
            double g = 0.0;
            if (j + 1 < P) {
                const double u = next - cur;
                g += k2 * u;
                e += u * u;
            }
            if (j > 0) g -= k2 * (cur - prev);
            a.f[bidx(a, j, l, d)] = g;
            prev = cur;
            cur = next;
        }
    }
    a.scr[boson_scr_eint(a.N) + l] = a.ks * e;
}

struct SeqLds {
    double e0[kBosonMaxN * 3];      // bead 0 of each particle
    double el[kBosonMaxN * 3];      // bead P-1
    double chi[kBosonMaxN + 1];     // prefix sums of the chain links l -> l+1 (double-double)
    double clo[kBosonMaxN + 1];
    double vhi[kBosonMaxN + 1];     // V' (double-double)
    double vlo[kBosonMaxN + 1];
    double ev[kBosonMaxN + 1];      // EV'
    double adj[kBosonMaxN + 1];     // dV'[N]/dV'[n]; first the scan of chunk totals
    double red[16];
};

__device__ __forceinline__ double link_e(const SeqLds &s, const BosonArgs &a, int l, int l2)
{
    double e = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double u = mic(s.e0[l2 * 3 + d], s.el[l * 3 + d], a.box[d]);
        e += u * u;
    }
    return a.ks * e;
}

__global__ __launch_bounds__(kSeq) void k_boson_seq(BosonArgs a)
{
    __shared__ SeqLds s;
    const int t = threadIdx.x, N = a.N;
    double *w = a.scr;                               // ring weights w[n,k]
    for (int e = t; e < N * 3; e += kSeq) {
        const int l = e / 3, d = e - l * 3;
        s.e0[e] = a.x[bidx(a, 0, l, d)];
        s.el[e] = a.x[bidx(a, a.P - 1, l, d)];
    }
    // the inner energies' sum, thread-strided, then in wave order
    double esum = 0.0;
    for (int l = t; l < N; l += kSeq) esum += a.scr[boson_scr_eint(N) + l];
    {
        double dummy = 0.0;
        seq_sum2(esum, dummy, s.red);   // (its barrier also publishes e0, el)
    }
    // Prefix sums ch[m] = sum_{l<m} link(l, l+1), m = 0..N-1, in
    // double-double: each thread sums a contiguous chunk, the chunk totals
    // are scanned (Hillis-Steele), then each chunk is written out.
    const int nl = N - 1;                            // chain links
    const int C = (nl + kSeq - 1) / kSeq;
    const int l0 = t * C, l1 = min(l0 + C, nl);
    DD tot = {0.0, 0.0};
    for (int l = l0; l < l1; ++l) tot = dd_add1(tot, link_e(s, a, l, l + 1));
    s.adj[t] = tot.hi;
    s.ev[t] = tot.lo;
    __syncthreads();
    for (int off = 1; off < kSeq; off <<= 1) {
        DD add = {0.0, 0.0};
        if (t >= off) add = {s.adj[t - off], s.ev[t - off]};
        __syncthreads();
        if (t >= off) {
            const DD v = dd_add({s.adj[t], s.ev[t]}, add);
            s.adj[t] = v.hi;
            s.ev[t] = v.lo;
        }
        __syncthreads();
    }
    DD run = {0.0, 0.0};
    if (t > 0) run = {s.adj[t - 1], s.ev[t - 1]};
    __syncthreads();   // the scan's slots are read before s.ev is reused
    if (t == 0) {
        s.chi[0] = 0.0;
        s.clo[0] = 0.0;
    }
    for (int l = l0; l < l1; ++l) {
        run = dd_add1(run, link_e(s, a, l, l + 1));
        s.chi[l + 1] = run.hi;
        s.clo[l + 1] = run.lo;
    }
    if (t == 0) {
        s.vhi[0] = 0.0;
        s.vlo[0] = 0.0;
        s.ev[0] = 0.0;
    }
    __syncthreads();

    // Forward: V'[n] = V'[n-1] + delta_n, delta_n a soft minimum of
    // b_k = E'[n,k] + V'[n-k] - V'[n-1] (all small), stabilized by the
    // minimum; w[n,k] = exp(-beta_n (b_k - delta_n)) / n.  Thread t takes
    // k = 1 + t + u kSeq.  V'[n-1] is in every thread's registers; V'[m] for
    // m < n-1 was written by thread 0 before at least one barrier.
    DD vprev = {0.0, 0.0};
    const double bn = a.bn;
    for (int n = 1; n <= N; ++n) {
        const DD chn = {s.chi[n - 1], s.clo[n - 1]};
        double b[kSeqU], E[kSeqU];
        double mloc = INFINITY;
#pragma unroll
        for (int u = 0; u < kSeqU; ++u) {
            const int k = 1 + t + u * kSeq;
            b[u] = INFINITY;
            E[u] = 0.0;
            if (k <= n) {
                const int j = n - k;
                const double c = dd_diff(chn, {s.chi[j], s.clo[j]});
                E[u] = c + link_e(s, a, n - 1, j);
                const double dv = (k == 1) ? 0.0 : dd_diff({s.vhi[j], s.vlo[j]}, vprev);
                b[u] = E[u] + dv;
                mloc = fmin(mloc, b[u]);
            }
        }
        const double m = seq_min(mloc, s.red);
        double sw = 0.0, st = 0.0;
        double ex[kSeqU];
#pragma unroll
        for (int u = 0; u < kSeqU; ++u) {
            const int k = 1 + t + u * kSeq;
            ex[u] = 0.0;
            if (k <= n) {
                ex[u] = exp(-bn * (b[u] - m));
                sw += ex[u];
                st += ex[u] * (E[u] + s.ev[n - k]);
            }
        }
        seq_sum2(sw, st, s.red);
        const double delta = m - log(sw / (double)n) / bn;
        vprev = dd_add1(vprev, delta);
        const double isw = 1.0 / sw;
#pragma unroll
        for (int u = 0; u < kSeqU; ++u) {
            const int k = 1 + t + u * kSeq;
            if (k <= n) w[tri_row(n) + (k - 1)] = ex[u] * isw;
        }
        if (t == 0) {
            s.vhi[n] = vprev.hi;
            s.vlo[n] = vprev.lo;
            s.ev[n] = st * isw;
        }
    }
    // Adjoints: adj[N] = 1, adj[n-k] += adj[n] w[n,k] for n = N..1 (the
    // targets of one n are distinct); a barrier per n makes adj[n] final.
    for (int e = t; e <= N; e += kSeq) s.adj[e] = (e == N) ? 1.0 : 0.0;
    for (int n = N; n >= 1; --n) {
        double wr[kSeqU];
#pragma unroll
        for (int u = 0; u < kSeqU; ++u) {
            const int k = 1 + t + u * kSeq;
            wr[u] = (k <= n) ? w[tri_row(n) + (k - 1)] : 0.0;
        }
        __syncthreads();
        const double an = s.adj[n];
#pragma unroll
        for (int u = 0; u < kSeqU; ++u) {
            const int k = 1 + t + u * kSeq;
            if (k <= n) s.adj[n - k] += an * wr[u];
        }
    }
    __syncthreads();
    for (int e = t; e <= N; e += kSeq) a.scr[boson_scr_adj(N) + e] = s.adj[e];
    if (t == 0) {
        const DD vb = dd_add1({s.vhi[N], s.vlo[N]}, esum);
        a.res[0] = vb.hi + vb.lo;
        a.res[1] = esum + s.ev[N];
    }
}

// Row n = blockIdx.x + 1: q[n,k] = adj[n] w[n,k], the probability of ring
// (n,k)'s closing link n-1 -> n-k; T[n,k] = sum_{k' >= k} q[n,k'] (each
// thread a contiguous chunk of k, then a scan of the chunk totals from the
// right).  With prob, row n-1 of it gets the closing links and zeros (its
// chain entry n is written by k_boson_links).
__global__ __launch_bounds__(kBlock) void k_boson_rows(BosonArgs a)
{
    __shared__ double tot[kBlock];
    const int n = blockIdx.x + 1, t = threadIdx.x, N = a.N;
    const double an = a.scr[boson_scr_adj(N) + n];
    const double *w = a.scr + tri_row(n);
    double *T = a.scr + boson_scr_tri(N) + tri_row(n);
    constexpr int CU = (kBosonMaxN + kBlock - 1) / kBlock;
    const int C = (n + kBlock - 1) / kBlock;
    const int k0 = 1 + t * C;
    double q[CU];
    double acc = 0.0;
#pragma unroll
    for (int u = CU - 1; u >= 0; --u) {
        const int k = k0 + u;
        q[u] = 0.0;
        if (u < C && k <= n) {
            q[u] = an * w[k - 1];
            acc += q[u];
        }
    }
    tot[t] = acc;
    __syncthreads();
    // suffix scan of the chunk totals: tot[t] = sum over threads >= t
    for (int off = 1; off < kBlock; off <<= 1) {
        const double add = (t + off < kBlock) ? tot[t + off] : 0.0;
        __syncthreads();
        tot[t] += add;
        __syncthreads();
    }
    double run = (t + 1 < kBlock) ? tot[t + 1] : 0.0;
#pragma unroll
    for (int u = CU - 1; u >= 0; --u) {
        const int k = k0 + u;
        if (u < C && k <= n) {
            run += q[u];
            T[k - 1] = run;
        }
    }
    if (a.prob) {
        double *row = a.prob + (size_t)(n - 1) * N;
#pragma unroll
        for (int u = 0; u < CU; ++u) {
            const int k = k0 + u;
            if (u < C && k <= n) row[n - k] = q[u];
        }
        for (int j = n + t; j < N; j += kBlock) row[j] = 0.0;
    }
}

// One wave per particle l: the chain links' probabilities
//   chain[l] = sum_{n=l+2..N} T[n, n-l]   (the rings in which l -> l+1 is a link)
// and the link forces on its last bead (links l -> l', l' <= l+1) and its
// first bead (links l'' -> l, l'' >= l-1).
__global__ __launch_bounds__(kBlock) void k_boson_links(BosonArgs a)
{
    const int lane = threadIdx.x & 63;
    const int l = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    const int N = a.N;
    if (l >= N) return;
    const double *w = a.scr;
    const double *T = a.scr + boson_scr_tri(N);
    const double *adj = a.scr + boson_scr_adj(N);
    auto X = [&](int j, int p, int d) { return a.x[bidx(a, j, p, d)]; };
    double cl = 0.0, cm = 0.0;
    for (int n = l + 2 + lane; n <= N; n += 64) cl += T[tri_row(n) + (n - l) - 1];
    if (l >= 1)
        for (int n = l + 1 + lane; n <= N; n += 64) cm += T[tri_row(n) + (n - l + 1) - 1];
    cl = wave_sum(cl);
    cm = wave_sum(cm);
    const double k2 = 2.0 * a.ks;
    const int Pl = a.P - 1;
    double el[3], e0[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        el[d] = X(Pl, l, d);
        e0[d] = X(0, l, d);
    }
    // last bead: closing links l -> l' (ring (l+1, l+1-l')), then the chain
    double g[3] = {0.0, 0.0, 0.0};
    const double an = adj[l + 1];
    for (int lp = lane; lp <= l; lp += 64) {
        const double q = an * w[tri_row(l + 1) + (l - lp)];
#pragma unroll
        for (int d = 0; d < 3; ++d) g[d] += k2 * q * mic(X(0, lp, d), el[d], a.box[d]);
    }
    // first bead: closing links m -> l (ring (m+1, m+1-l)), m = l..N-1
    double h[3] = {0.0, 0.0, 0.0};
    for (int m = l + lane; m < N; m += 64) {
        const double q = adj[m + 1] * w[tri_row(m + 1) + (m - l)];
#pragma unroll
        for (int d = 0; d < 3; ++d) h[d] -= k2 * q * mic(e0[d], X(Pl, m, d), a.box[d]);
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        g[d] = wave_sum(g[d]);
        h[d] = wave_sum(h[d]);
    }
    if (lane == 0) {
        if (l + 1 < N) {
#pragma unroll
            for (int d = 0; d < 3; ++d) g[d] += k2 * cl * mic(X(0, l + 1, d), el[d], a.box[d]);
            if (a.prob) a.prob[(size_t)l * N + l + 1] = cl;
        }
        if (l >= 1) {
#pragma unroll
            for (int d = 0; d < 3; ++d) h[d] -= k2 * cm * mic(e0[d], X(Pl, l - 1, d), a.box[d]);
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            a.f[bidx(a, Pl, l, d)] += g[d];
            a.f[bidx(a, 0, l, d)] += h[d];
        }
    }
}

// ---------------------------------------------------------------------------
// The bosonic fix's step in a context (Sec. III.C: Cartesian coordinates,
// since the normal modes change under exchange; the thermostat of Eq. D3 on
// every bead with one damping time).  Thread = (atom, bead), A = kBlock/P
// atoms per block, tiles strided over the grid.  The forces are the array f
// (the potential's: force pass, trap kernel or caller) plus fs (the springs
// inside the rings and the exchange links).  Modes as the distinguishable
// pass: STEP (the pending closing kick, and OBABO's last O, then the
// estimators' sums at that synchronized state, then the opening of the new
// step: BAOAB B A O A, OBABO O B A A), CLOSE, EST, PREP (centroids only).
// The partials are those of the distinguishable pass: PF_EKIN (Cartesian
// kinetic energy), PF_VIR (sum of r . F over the potential's forces, for
// K_VR), the excursion and displacement maxima for the neighbor lists, and
// the non-finite flag.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_bpass(FusedArgs a)
{
    __shared__ double sX[3 * kBlock];    // [A][3][P] positions of the tile
    __shared__ double sC[3 * kBlock];    // [A][3] centroids
    __shared__ double red[64];
    const int P = a.P, N = a.N;
    const int A = kBlock / P;
    const int t = threadIdx.x, la = t / P, k = t - la * P;
    const bool lane_ok = la < A;
    const int mode = a.mode;
    const long long budget = a.ctl->budget;
    const unsigned long long step = a.ctl->step;
    const int synced = a.ctl->synced;
    const bool spent = (mode == FUSED_STEP && budget == 0);
    const bool closing = (mode == FUSED_STEP || mode == FUSED_CLOSE) && !synced;
    const bool est_now = closing || mode == FUSED_EST;
    const bool moves = (mode == FUSED_STEP || mode == FUSED_PREP);
    const double c1 = a.modes[MD_C1], c2 = a.modes[MD_C2];
    const double h = a.hdt;
    double acc_ekin = 0.0, acc_vir = 0.0, acc_emax = 0.0, acc_dmax = 0.0, acc_bad = 0.0;
    const int ntiles = (N + A - 1) / A;
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int i = tile * A + la;
        const bool act = lane_ok && i < N;
        double x[3] = {0.0, 0.0, 0.0}, v[3] = {0.0, 0.0, 0.0}, fp[3] = {0.0, 0.0, 0.0};
        double ft[3] = {0.0, 0.0, 0.0};
        double hm = 0.0, im = 0.0, sg = 0.0, active = 0.0, cref[3] = {0.0, 0.0, 0.0};
        unsigned oi = 0;
        const size_t b = (size_t)i * 3 * P + k;
        if (act) {
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                x[d] = a.x[b + d * P];
                v[d] = a.v[b + d * P];
                if (mode != FUSED_PREP) {
                    fp[d] = a.f[b + d * P];
                    ft[d] = fp[d] + a.fs[b + d * P];
                }
            }
            hm = a.atoms[i * 4 + AT_HALF_M];
            im = a.atoms[i * 4 + AT_INV_M];
            sg = a.atoms[i * 4 + AT_SIGMA];
            active = a.atoms[i * 4 + AT_ACTIVE];
            oi = (unsigned)a.orig[i];
            if (k == 0 && moves) {
                cref[0] = a.cref[i * 3]; cref[1] = a.cref[i * 3 + 1]; cref[2] = a.cref[i * 3 + 2];
            }
        }
        if (spent) return;
        if (act) {
            // PILE on this bead's velocity over one O step, noise of step s_
            // and O step q_ of that step, counter (atom, bead, s_, q_)
            auto o_step = [&](unsigned long long s_, unsigned long long q_) {
                double z[3];
                gauss3(a.seed, oi, (unsigned)k, s_, z, (unsigned)q_);
#pragma unroll
                for (int d = 0; d < 3; ++d) v[d] = c1 * v[d] + c2 * sg * z[d];
            };
            if (closing) {
#pragma unroll
                for (int d = 0; d < 3; ++d) v[d] += h * ft[d] * im;
                if (a.obabo && a.nvt) o_step(step - 1, 1);
            }
            if (est_now) {
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    acc_ekin += hm * v[d] * v[d];
                    acc_vir += x[d] * fp[d];
                }
            }
            if (mode == FUSED_STEP) {
                if (a.obabo) {
                    if (a.nvt) o_step(step, 0);
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        v[d] += h * ft[d] * im;
                        x[d] += h * v[d];
                        x[d] += h * v[d];
                    }
                } else {
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        v[d] += h * ft[d] * im;
                        x[d] += h * v[d];
                    }
                    if (a.nvt) o_step(step, 0);
#pragma unroll
                    for (int d = 0; d < 3; ++d) x[d] += h * v[d];
                }
#pragma unroll
                for (int d = 0; d < 3; ++d) a.x[b + d * P] = x[d];
            }
            if (mode == FUSED_STEP || mode == FUSED_CLOSE) {
#pragma unroll
                for (int d = 0; d < 3; ++d) a.v[b + d * P] = v[d];
            }
#pragma unroll
            for (int d = 0; d < 3; ++d)
                if (!isfinite(x[d]) || !isfinite(v[d])) acc_bad = 1.0;
        }
        if (moves) {
            // centroids, the beads' excursions and the centroids' displacement
            // since the last list build (the rebuild criterion), cells
            __syncthreads();   // the previous tile's reads of sX and sC are done
            if (act) {
#pragma unroll
                for (int d = 0; d < 3; ++d) sX[(la * 3 + d) * P + k] = x[d];
            }
            __syncthreads();
            if (act && k == 0) {
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    double c = 0.0;
                    for (int j = 0; j < P; ++j) c += sX[(la * 3 + d) * P + j];
                    sC[la * 3 + d] = c / (double)P;
                }
            }
            __syncthreads();
            if (act) {
                double e2 = 0.0, c[3];
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    c[d] = sC[la * 3 + d];
                    const double u = x[d] - c[d];
                    e2 += u * u;
                }
                if (active != 0.0) acc_emax = fmax(acc_emax, e2);
                if (k == 0) {
                    double d2 = 0.0;
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        a.cent[i * 3 + d] = c[d];
                        const double u = c[d] - cref[d];
                        d2 += u * u;
                    }
                    if (active != 0.0) acc_dmax = fmax(acc_dmax, d2);
                    if (a.ncell > 0 && i < a.n_active) (void)cell_of(a, i, c);
                }
            }
        }
    }
    if (spent) return;
    double s2[2] = {acc_ekin, acc_vir};
    double m3[3] = {acc_emax, acc_dmax, acc_bad};
    block_sum_max<2, 3>(s2, m3, red);
    if (t == 0) {
        double *pp = a.partials + (size_t)blockIdx.x * PF_COUNT;
        for (int q = 0; q < PF_COUNT; ++q) pp[q] = 0.0;
        pp[PF_EKIN] = s2[0];
        pp[PF_VIR] = s2[1];
        pp[PF_EMAX] = m3[0];
        pp[PF_DMAX] = m3[1];
        pp[PF_NONFINITE] = m3[2];
    }
}

// Harmonic trap on Cartesian beads: f = -m mvv2e omega^2 x for every bead,
// and per block the energy sum 1/2 m mvv2e omega^2 |x|^2 (fpartials, with a
// zero virial).  Thread = (atom, bead) as in the step pass.
__global__ __launch_bounds__(kBlock) void k_btrap(FusedArgs a, double *f, double *fpartials)
{
    __shared__ double red[64];
    const int P = a.P, A = kBlock / P;
    const int t = threadIdx.x, la = t / P, k = t - la * P;
    const int i = blockIdx.x * A + la;
    double e = 0.0;
    if (!a.ctl->ran) return;   // the system took no step (uniform per block)
    if (la < A && i < a.N) {
        const double kk = 2.0 * a.atoms[i * 4 + AT_HALF_M] * a.omega2;
        const size_t b = (size_t)i * 3 * P + k;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double xv = a.x[b + d * P];
            f[b + d * P] = -kk * xv;
            e += 0.5 * kk * xv * xv;
        }
    }
    double e1[1] = {e};
    block_sum<1>(e1, red);
    if (t == 0) reinterpret_cast<double2 *>(fpartials)[blockIdx.x] = make_double2(e1[0], 0.0);
}

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// The current device's address of scratch, looked up at its first use.
hipError_t device_scratch(double **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = static_cast<double *>(p);
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

int boson_args(const double *x, int32_t N, int32_t P, double kspring, double beta_n,
               const double *box, double *f, double *prob, double *out, int max_n, BosonArgs &a)
{
    if (!x || !f || !out) return report_error(PIMD_ERR_ARG, "x, f and out must be non-NULL");
    if (N < 1 || P < 1) return report_error(PIMD_ERR_ARG, "N and P must be >= 1");
    if (!(kspring >= 0.0) || !std::isfinite(kspring) || !(beta_n > 0.0) || !std::isfinite(beta_n))
        return report_error(PIMD_ERR_ARG, "kspring >= 0 and beta_n > 0 must be finite");
    if (box)
        for (int d = 0; d < 3; ++d)
            if (!(box[d] >= 0.0) || !std::isfinite(box[d]))
                return report_error(PIMD_ERR_ARG, "box lengths must be finite and >= 0");
    if (N > max_n)
        return report_error(PIMD_ERR_UNSUPPORTED, max_n == kBosonNoAllocMaxN
                                                      ? "N > 512 (the allocation-free scratch's limit)"
                                                      : "N > 1024");
    if (P > kMaxBeads) return report_error(PIMD_ERR_UNSUPPORTED, "P > 128");
    a = BosonArgs{};
    a.x = x;
    a.N = N;
    a.P = P;
    a.layout = 0;
    a.ks = kspring;
    a.bn = beta_n;
    for (int d = 0; d < 3; ++d) a.box[d] = box ? box[d] : 0.0;
    a.f = f;
    a.prob = prob;
    a.res = out;
    return PIMD_OK;
}

}  // namespace

int boson_pass_grid(int N, int P)
{
    const int A = kBlock / P;
    const int ntiles = (N + A - 1) / A;
    return ntiles < 2048 ? ntiles : 2048;
}

void launch_boson_pass(const FusedArgs &a, int grid, hipStream_t st)
{
    hipLaunchKernelGGL(k_bpass, dim3(grid), dim3(kBlock), 0, st, a);
}

int boson_trap_grid(int N, int P)
{
    const int A = kBlock / P;
    return (N + A - 1) / A;
}

void launch_boson_trap(const FusedArgs &a, double *f, double *fpartials, hipStream_t st)
{
    hipLaunchKernelGGL(k_btrap, dim3(boson_trap_grid(a.N, a.P)), dim3(kBlock), 0, st, a, f,
                       fpartials);
}

void launch_boson_springs(const BosonArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL(k_boson_inner, dim3((a.N + kBlock - 1) / kBlock), dim3(kBlock), 0, st, a);
    hipLaunchKernelGGL(k_boson_seq, dim3(1), dim3(kSeq), 0, st, a);
    hipLaunchKernelGGL(k_boson_rows, dim3(a.N), dim3(kBlock), 0, st, a);
    hipLaunchKernelGGL(k_boson_links, dim3((a.N + kBlock / 64 - 1) / (kBlock / 64)), dim3(kBlock), 0,
                       st, a);
}

}  // namespace pimd

using namespace pimd;

extern "C" {

int pimd_boson_spring(const double *x, int32_t N, int32_t P, double kspring, double beta_n,
                      const double *box, double *f, double *prob, double *out, void *stream)
{
    BosonArgs a;
    int rc = boson_args(x, N, P, kspring, beta_n, box, f, prob, out, kBosonMaxN, a);
    if (rc != PIMD_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipMalloc((void **)&a.scr, boson_scr_doubles(N) * sizeof(double));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return report_error(PIMD_ERR_OOM, "scratch allocation failed");
    }
    launch_boson_springs(a, st);
    e = hipGetLastError();
    // the scratch is freed once the kernels that read it are done
    const hipError_t es = hipStreamSynchronize(st);
    (void)hipFree(a.scr);
    if (e == hipSuccess) e = es;
    if (e != hipSuccess) return report_error(PIMD_ERR_DEVICE, hipGetErrorString(e));
    return PIMD_OK;
}

int pimd_boson_spring_noalloc(const double *x, int32_t N, int32_t P, double kspring,
                              double beta_n, const double *box, double *f, double *prob,
                              double *out, void *stream)
{
    BosonArgs a;
    int rc = boson_args(x, N, P, kspring, beta_n, box, f, prob, out, kBosonNoAllocMaxN, a);
    if (rc != PIMD_OK) return rc;
    hipError_t e = device_scratch(&a.scr);
    if (e != hipSuccess) return report_error(PIMD_ERR_DEVICE, hipGetErrorString(e));
    // every scratch value the kernels read is written earlier in the same
    // call, so nothing needs clearing
    launch_boson_springs(a, (hipStream_t)stream);
    e = hipGetLastError();
    if (e != hipSuccess) return report_error(PIMD_ERR_DEVICE, hipGetErrorString(e));
    return PIMD_OK;
}

}  // extern "C"
