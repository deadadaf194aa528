// Fused BAOAB step pass with the normal-mode transforms on the FP64 matrix
// cores (v_mfma_f64_16x16x4f64), for P in {16, 32, 64}.
//
// The positions' normal modes are carried from step to step relative to each
// atom's bead 0: y~ = M (x - x_0 1) (App. B, Eq. B1; exact because the
// non-centroid rows of M sum to zero), so a step needs two of the three
// transforms of Sec. IV.A, f~ = M f and the inverse x = x_0 + M^T y~.  At the
// end of the step the reference moves to the new bead 0, which changes only
// the centroid mode, by -sqrt(P) times that bead's offset.
//
// A block works on T = 64/P tiles of 16 atoms at once.  The f and y~ rows of
// those atoms ([atom][d][P], contiguous in memory) are copied into LDS by
// direct global-to-LDS loads, the next block tile's copies in flight while
// the current one is processed (the y~ tile is double-buffered, the f tile
// refilled once its products are formed); v~ and the per-atom values come
// into registers the same way one phase ahead.  Each atom tile is shared by
// P/16 waves, wave w taking mode block (and, in the inverse, bead block)
// w % (P/16).  Per dim d the wave forms
//   f~^T[atom][mode] = sum_bead f^T[atom][bead] M^T[bead][mode]
//   x^T[atom][bead]  = x_0 + sum_mode y~^T[atom][mode] M[mode][bead]
// with the B operands (4 rows x 16 columns of M^T or M) read from a table of
// M's distinct values in LDS (m_index).
//
// Operand layout of the instruction (checked on the device): A[i][k] in lane
// i + 16k, B[k][j] in lane j + 16k, and accumulator register r of lane l
// holds D[4r + l/16][l%16].  With atoms as rows, lane l holds, for one mode
// (column l%16 of the wave's mode block), the four atoms 4r + l/16: the
// per-(atom, mode) work (B, A, O with one Philox call for the three dims, A)
// runs in registers, and v~ and y~ are read and written as 128-byte segments.
//
// LDS bank swizzle.  A 64-bit LDS access of a wave is served in groups of 16
// or 32 lanes.  The operand reads take lane (i, k) -> row i, column c + k;
// the update takes lane (i, k) -> row 4r + k, columns c + i.  Rows are a
// multiple of 32 words long, so unswizzled the operand reads of one group
// would all hit one bank.  The copies permute each row's 16-byte units by
// unit ^ (row mod 16) (mod 8 for P = 16): the 16 rows of a group then read
// 16 distinct units of an aligned 32-word window, and the update's 16
// consecutive columns stay inside one.
//
// Waits.  The barriers between phases wait for LDS operations only
// (lds_barrier); a workgroup fence there would also wait for every global
// load, store and copy in flight, which is what serialized the memory and
// arithmetic phases of an earlier version.  Only the barrier at the top of a
// tile waits for the tile's copies.
#include "pimd_device.h"
#include "pimd_internal.h"

namespace pimd {

typedef double d4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int kWaves = kBlock / 64;

// Wave priority around the phases whose instructions should win issue
// arbitration: the tile copies (3, so that the next tile's bytes are requested
// as early as possible) and the matrix-core loops (2, so that the long MFMA
// chains start while the other block's waves fill the vector ALUs); 0 for the
// rest.  Measured on the water P = 64 state: 93.0 -> 89.8 us per launch.
__device__ __forceinline__ void prio(int p)
{
    if (p == 3) __builtin_amdgcn_s_setprio(3);
    else if (p == 2) __builtin_amdgcn_s_setprio(2);
    else __builtin_amdgcn_s_setprio(0);
}

__device__ __forceinline__ d4 mfma4(double a, double b, d4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <int P>
struct Lds {
    static constexpr int NMB = P / 16;            // mode blocks = waves per atom tile
    static constexpr int T = kWaves / NMB;        // atom tiles per block
    static constexpr int ROW = 3 * P;             // doubles per atom row of f and y~ ([d][P])
    static constexpr int UNITS = ROW / 2;         // 16-byte units per row
    static constexpr int SWZ = (UNITS % 16 == 0) ? 15 : 7;   // unit swizzle mask
    static constexpr int TILE = 16 * T * ROW;     // a block tile of f or y~ (doubles)
    static constexpr int AW = 13;                 // per-atom row of the atom table
    static constexpr int A_ELEMS = 16 * T * AW;
    static constexpr int MK_ELEMS = 8 * P;        // the per-mode table, shared by the block
    static constexpr int MT_ELEMS = 2 * P + 4;    // the distinct entries of M (m_index)
    static constexpr int NDMA = TILE / 2 / 64 / kWaves;   // 16-byte copies per lane per tile
    static constexpr int bytes = 8 * (3 * TILE + A_ELEMS + MK_ELEMS + MT_ELEMS);
    static_assert(NDMA * 64 * kWaves * 2 == TILE, "tile units split evenly over the waves");
    static_assert(UNITS % (SWZ + 1) == 0, "the swizzle stays inside a row");
    static_assert(2 * bytes <= 160 * 1024, "two blocks per CU");
    static_assert(16 * T <= kBlock, "one thread per atom of the block tile");
};

// In an f or y~ tile, column c of row a is stored at
//   a ROW + ((((c >> 1) ^ (a & SWZ)) << 1) | (c & 1)):
// the row's 16-byte units are permuted by unit ^ (a & SWZ).  With c = d P + j
// (j < P) and SWZ < P/2 that is a ROW + d P + swc(a & SWZ, j): the permutation
// stays inside each dimension's P columns.
template <int P>
__device__ __forceinline__ int swc(int s, int j)
{
    static_assert(Lds<P>::SWZ < P / 2, "the swizzle stays inside a dimension's columns");
    return (((j >> 1) ^ s) << 1) | (j & 1);
}

// The lane index, opaque to the compiler: lane-dependent offsets derived from
// it are formed where they are used instead of being hoisted out of the tile
// loop, where they would hold registers over the whole pass.
__device__ __forceinline__ int opaque(int x)
{
    asm volatile("" : "+v"(x));
    return x;
}

typedef __attribute__((address_space(3))) void lds_void;

// Copies rows [0, nrows) of a block tile (rows of ROW doubles, contiguous from
// src) into the LDS tile dst in the layout of tix, by direct global-to-LDS
// loads: the instruction writes lane i's 16 bytes at its LDS base + 16 i, so
// wave w fills units [64 (w NDMA + j), 64 (w NDMA + j + 1)) at step j and
// each lane fetches the global unit that belongs at its slot.  Completion is
// counted by vmcnt; the tile is read after a wait and a barrier.
template <int P>
__device__ __forceinline__ void dma_tile(const double *src, double *dst, int nrows, int w, int lane)
{
    using L = Lds<P>;
    const int ln = opaque(lane);
    if (nrows == 16 * L::T) {
        // a whole tile (uniform): no per-lane test
#pragma unroll
        for (int j = 0; j < L::NDMA; ++j) {
            const int base = (w * L::NDMA + j) * 64;
            const int q = base + ln;
            const int a = q / L::UNITS, up = q - a * L::UNITS;
            const int u = up ^ (a & L::SWZ);
            __builtin_amdgcn_global_load_lds((const void *)(src + 2 * (a * L::UNITS + u)),
                                             (lds_void *)(dst + 2 * base), 16, 0, 0);
        }
    } else {
#pragma unroll
        for (int j = 0; j < L::NDMA; ++j) {
            const int base = (w * L::NDMA + j) * 64;
            const int q = base + ln;
            const int a = q / L::UNITS, up = q - a * L::UNITS;
            const int u = up ^ (a & L::SWZ);
            if (a < nrows)
                __builtin_amdgcn_global_load_lds((const void *)(src + 2 * (a * L::UNITS + u)),
                                                 (lds_void *)(dst + 2 * base), 16, 0, 0);
        }
    }
}

// Barrier for LDS hand-offs only: this wave's LDS accesses are complete
// before it (lgkmcnt(0): s_waitcnt immediate 0xC07F leaves vmcnt at its
// maximum 63 and expcnt at 7), and its global loads, stores and copies into
// LDS stay in flight.  (A workgroup fence would wait for those too: the
// copies count as LDS writes, tracked by vmcnt.)  The wait is the builtin, so
// that the compiler's own wait insertion knows of it; the barrier's asm has a
// memory clobber, which keeps the compiler from moving memory accesses
// across it.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_s_waitcnt(0xC07F);
    asm volatile("s_barrier" ::: "memory");
}

// Barrier after which every wave's copies into LDS (and all its other memory
// operations) are complete.
__device__ __forceinline__ void dma_barrier()
{
    __builtin_amdgcn_s_waitcnt(0);
    asm volatile("s_barrier" ::: "memory");
}

// Entry M[k][j] of the normal-mode matrix (App. B) is a function of its row
// type and of the phase q = k j mod P alone: a0 on the centroid row, +-a0 on
// the alternating row (q = 0 or P/2), a1 cos(2 pi q / P) on the cosine rows,
// a1 sin(2 pi q / P) on the sine rows.  The block keeps those 2P + 3 values
// in LDS (copied from M, so the bits are M's): cosines at [0, P), sines at
// [P, 2P), a0 at 2P, the alternating row's two values at 2P + 1 + q/(P/2).
// The matrix-core products take their M operands from there, so that no
// global load waits behind the copies in flight.
template <int P>
__device__ __forceinline__ int m_index(int k, int q)
{
    constexpr int LG = (P == 16) ? 4 : (P == 32 ? 5 : 6);
    static_assert((1 << LG) == P, "P is a power of two");
    // selects rather than branches: k differs between lanes
    int idx = (2 * k < P) ? q : P + q;
    idx = (2 * k == P) ? 2 * P + 1 + (q >> (LG - 1)) : idx;
    return (k == 0) ? 2 * P : idx;
}

// m_index for a fixed row k, as base + ((q & mask) >> shift): the forward
// products' lanes keep one row for the whole pass.
template <int P>
struct MRow {
    int base, mask, shift;
    __device__ __forceinline__ MRow(int k)
    {
        constexpr int LG = (P == 16) ? 4 : (P == 32 ? 5 : 6);
        base = (k == 0) ? 2 * P : (2 * k == P) ? 2 * P + 1 : (2 * k < P) ? 0 : P;
        mask = (k == 0) ? 0 : P - 1;
        shift = (2 * k == P) ? LG - 1 : 0;
    }
    __device__ __forceinline__ int at(int q) const { return base + ((q & mask) >> shift); }
};

// atom-table columns (per atom of a tile); TA_OA holds (orig, active) as two ints
enum { TA_X0 = 0, TA_HM = 3, TA_IM = 4, TA_SG = 5, TA_OA = 6, TA_CREF = 7, TA_C = 10 };

// a lane's running sums and maxima over its tiles (fixcom momentum last)
enum { ACC_EKIN = 0, ACC_ESP, ACC_VIR, ACC_UEXT, ACC_K0, ACC_EMAX, ACC_DMAX, ACC_BAD, ACC_P,
       ACC_COUNT = ACC_P + 3 };

// The block's LDS: the f tile, two y~ tiles (the current one and the next
// one's copy in flight), the atom table and the per-mode table.  Separate
// arrays, so that the compiler sees that a copy into one leaves reads of the
// others free to go ahead.
template <int P>
struct Smem {
    double *f, *y0, *y1, *at, *mk, *mt;
};

// The control block's values for this pass, read once: vector loads (the
// pass writes memory the compiler cannot tell apart from it) that would
// otherwise wait behind the copies in flight at every tile.
struct TileCtl {
    unsigned long long step;
    int closing;        // a closing kick of the last step is pending
    int ucom_now;       // fixcom: the last step's centroid-mode velocity is still to go
    double ucom[3];
};

// a tile's per-atom values in registers: the atom table row, cref, bead 0 of x
enum { RA_CREF = 4, RA_X0 = 7, RA_COUNT = 10 };

}  // namespace

// Processes block tiles first, first + stride, ... (T*16 atoms each) of one
// system and writes one set of partials for the block.
//
// Per block tile n (buffer Y_c of the two y~ tiles):
//   wait for tile n's copies; barrier
//   copy y~ of tile n+1 into Y_(1-c)                       (in flight over the tile)
//   forward products from the f tile; barrier
//   copy f of tile n+1 into the f tile                     (in flight over the rest)
//   update from Y_c, new y~ written over it in place; barrier
//   load v~ and the atom table of tile n+1 into registers
//   inverse products from Y_c; barrier
// so that each tile's reads overlap the previous tile's arithmetic and stores.
// v~ of this lane's four atoms (update layout: atom b0 + 16 tt + 4r + l/16,
// mode 16 mb + l%16) and, in thread t, atom b0 + t's per-atom values, for the
// block tile at b0 of nat >= 1 atoms.  Indices are clamped into the tile
// rather than tested, so that no branch has to wait for the loads (values of
// clamped atoms are never used).
template <int P>
__device__ __forceinline__ void load_tile_regs(const FusedArgs &a, int b0, int nat, int tt, int mb, int l,
                                               int t, double (&rv)[4][3], double (&ratom)[RA_COUNT],
                                               int &rorig)
{
    const int lp = opaque(l), pm = mb * 16 + (lp & 15);
    const int last = b0 + nat - 1;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int ia = min(b0 + tt * 16 + 4 * r + (lp >> 4), last);
        const size_t vb = (size_t)ia * 3 * P + pm;
#pragma unroll
        for (int d = 0; d < 3; ++d) rv[r][d] = a.v[vb + d * P];
    }
    const int ia = b0 + min(t, nat - 1);
#pragma unroll
    for (int q = 0; q < 4; ++q) ratom[q] = a.atoms[ia * 4 + q];
    rorig = a.orig[ia];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        ratom[RA_CREF + d] = a.cref[ia * 3 + d];
        ratom[RA_X0 + d] = a.x[(size_t)ia * 3 * P + d * P];
    }
}

template <int P, bool OB, bool FC, int C>
__device__ __forceinline__ void mfma_tile(const FusedArgs &a, const Smem<P> &sm, const TileCtl &tc,
                                          int bt, int nb, double (&rv)[4][3],
                                          double (&ratom)[RA_COUNT], int &rorig, double *acc)
{
    using L = Lds<P>;
    constexpr int NMB = L::NMB, T = L::T, AW = L::AW;
    constexpr int NK4 = P / 4;        // k-steps of 4
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    const int lr = l & 15, lq = l >> 4;
    const int tt = w / NMB;           // this wave's atom tile within the block
    const int mb = w - tt * NMB;      // this wave's mode block (and bead block)
    const int N = a.N;
    double *sY = C == 0 ? sm.y0 : sm.y1;
    double *sYn = C == 0 ? sm.y1 : sm.y0;
    double *sA = sm.at;
    const unsigned long long step = tc.step;
    const bool ext = !a.pair;
    const bool closing = tc.closing != 0;
    const bool need_f = a.pair != 0;
    const bool ucom_now = FC && tc.ucom_now;
    const double sqrtP = sqrt((double)P);
    const int b0 = bt * 16 * T;
    const int a0 = b0 + tt * 16;      // first atom of this wave's tile
    const bool has_next = nb >= 0;
    const int nb0 = nb * 16 * T;
    const int nnat = has_next ? min(16 * T, N - nb0) : 0;

    // publish this tile's atom table; then every wave's copies are complete
    if (t < 16 * T && b0 + t < N) {
        double *ar = sA + t * AW;
        ar[TA_HM] = ratom[AT_HALF_M];
        ar[TA_IM] = ratom[AT_INV_M];
        ar[TA_SG] = ratom[AT_SIGMA];
        int *oa = reinterpret_cast<int *>(ar + TA_OA);
        oa[0] = rorig;
        oa[1] = ratom[AT_ACTIVE] != 0.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            ar[TA_CREF + d] = ratom[RA_CREF + d];
            ar[TA_X0 + d] = ratom[RA_X0 + d];
        }
    }
    dma_barrier();
    if (has_next) { prio(3); dma_tile<P>(a.yt + (size_t)nb0 * 3 * P, sYn, nnat, w, l); prio(0); }

    // ---- forward products: f~ of mode block mb for the tile's 16 atoms
    // (the positions' modes are carried from the previous step)
    const int ra0 = tt * 16;          // this wave's first row in the tiles
    d4 af[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) af[d] = d4{0.0, 0.0, 0.0, 0.0};
    if (need_f) {
        const int lf = opaque(l), fr = lf & 15, fq = lf >> 4, fm = mb * 16 + fr;
        const double *frow = sm.f + (ra0 + fr) * L::ROW;
        const int fs = (ra0 + fr) & L::SWZ;
        // B operand M^T[bead][mode] = M[fm][4 kb + fq]: phase fm (4 kb + fq) mod P.
        // Rows of atoms past the end hold stale values: their products land in
        // accumulator rows that are never used.
        const MRow<P> mr(fm);
        const int q0 = (fm * fq) & (P - 1), dq = (4 * fm) & (P - 1);
        prio(2);
#pragma unroll 4
        for (int kb = 0; kb < NK4; ++kb) {
            const int cj = swc<P>(fs, 4 * kb + fq);
            const double bm = sm.mt[mr.at(q0 + kb * dq)];
#pragma unroll
            for (int d = 0; d < 3; ++d) af[d] = mfma4(frow[d * P + cj], bm, af[d]);
        }
        prio(0);
    }
    lds_barrier();                    // every wave is done with the f tile
    if (has_next && need_f) { prio(3); dma_tile<P>(a.f + (size_t)nb0 * 3 * P, sm.f, nnat, w, l); prio(0); }

    // ---- per (atom, mode) update: lane l, register r: atom a0 + 4r + uq, mode m
    const int lu = opaque(l), uq = lu >> 4;
    const int m = mb * 16 + (lu & 15);    // this lane's mode
    const double *mk = sm.mk + m;         // coefficient q at mk[q * P]
    const double off = (m == 0) ? sqrtP : 0.0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int ra = 4 * r + uq;
        const int ia = a0 + ra;
        if (ia >= N) continue;
        const int row = ra0 + ra;
        const double *ar = sA + row * AW;
        const double hm = ar[TA_HM], im = ar[TA_IM], sg = ar[TA_SG];
        const int orig = reinterpret_cast<const int *>(ar + TA_OA)[0];
        double *yrow = sY + row * L::ROW + swc<P>(row & L::SWZ, m);   // + d P: mode m of dim d
        double xt[3], ft[3], vt[3], x0[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            xt[d] = yrow[d * P];
            ft[d] = af[d][r];
            x0[d] = ar[TA_X0 + d];
            vt[d] = rv[r][d];
        }
        if (ucom_now && m == 0) {
#pragma unroll
            for (int d = 0; d < 3; ++d) vt[d] -= tc.ucom[d];
        }
        if (ext) {
#pragma unroll
            for (int d = 0; d < 3; ++d) ft[d] = -2.0 * hm * a.omega2 * (xt[d] + off * x0[d]);
        }
        // PILE-L at P*T over one O step (dt in BAOAB, dt/2 in OBABO), noise
        // of step s_ and O step q_ of that step
        auto o_step = [&](unsigned long long s_, unsigned long long q_) {
            double z[3];
            gauss3(a.seed, (unsigned)orig, (unsigned)m, s_, z, (unsigned)q_);
#pragma unroll
            for (int d = 0; d < 3; ++d) vt[d] = mk[MD_C1 * P] * vt[d] + mk[MD_C2 * P] * sg * z[d];
        };
        // A(dt/2): exact free-ring-polymer flow of this mode
        auto a_step = [&]() {
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const double q = xt[d], p = vt[d];
                xt[d] = mk[MD_A00 * P] * q + mk[MD_A01 * P] * p;
                vt[d] = mk[MD_A10 * P] * q + mk[MD_A11 * P] * p;
            }
        };
        if (closing) {
#pragma unroll
            for (int d = 0; d < 3; ++d) vt[d] += a.hdt * im * ft[d];
            // OBABO: the last O of the step being closed
            if (OB && a.nvt) o_step(step - 1, 1);
            if (FC && m == 0) {
#pragma unroll
                for (int d = 0; d < 3; ++d) acc[ACC_P + d] += hm * vt[d];
            }
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const double kd = hm * vt[d] * vt[d];
                acc[ACC_EKIN] += kd;
                if (m == 0) acc[ACC_K0] += kd;
                acc[ACC_ESP] += hm * mk[MD_SPRING * P] * xt[d] * xt[d];
                acc[ACC_VIR] += mk[MD_NONCENTROID * P] * xt[d] * ft[d];
            }
            // OBABO: the closing O's noise before the opening O's, not beside it
            if constexpr (OB) __builtin_amdgcn_sched_barrier(0);
        }
        if constexpr (OB) {
            // O(dt/2), B(dt/2), A(dt) = A(dt/2) A(dt/2)
            if (a.nvt) o_step(step, 0);
#pragma unroll
            for (int d = 0; d < 3; ++d) vt[d] += a.hdt * im * ft[d];
            a_step();
            a_step();
        } else {
            // B(dt/2), A(dt/2), O(dt), A(dt/2)
#pragma unroll
            for (int d = 0; d < 3; ++d) vt[d] += a.hdt * im * ft[d];
            a_step();
            if (a.nvt) o_step(step, 0);
            a_step();
        }
        if (ext) {
            // closing B with the trap force of the new positions (and
            // OBABO's last O), then the estimators of the new state
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                ft[d] = -2.0 * hm * a.omega2 * (xt[d] + off * x0[d]);
                vt[d] += a.hdt * im * ft[d];
            }
            if (OB && a.nvt) o_step(step, 1);
            if (FC && m == 0) {
#pragma unroll
                for (int d = 0; d < 3; ++d) acc[ACC_P + d] += hm * vt[d];
            }
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const double xa = xt[d] + off * x0[d];
                acc[ACC_EKIN] += hm * vt[d] * vt[d];
                acc[ACC_ESP] += hm * mk[MD_SPRING * P] * xt[d] * xt[d];
                acc[ACC_UEXT] += hm * a.omega2 * xa * xa;
                acc[ACC_VIR] += mk[MD_NONCENTROID * P] * xt[d] * ft[d];
            }
        }
        const size_t vb = (size_t)ia * 3 * P + m;
        a.v[vb] = vt[0]; a.v[vb + P] = vt[1]; a.v[vb + 2 * P] = vt[2];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            if (!isfinite(vt[d])) acc[ACC_BAD] = 1.0;
            yrow[d * P] = xt[d];
            // carried to the next step; the centroid mode is re-referenced
            // to the new bead 0 after the inverse
            if (m != 0) a.yt[vb + d * P] = xt[d];
        }
        if (m == 0) {
            double d2 = 0.0, c[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                c[d] = x0[d] + xt[d] / sqrtP;
                sA[row * AW + TA_C + d] = c[d];
                a.cent[ia * 3 + d] = c[d];
                const double dd = c[d] - ar[TA_CREF + d];
                d2 += dd * dd;
            }
            if (reinterpret_cast<const int *>(ar + TA_OA)[1]) acc[ACC_DMAX] = fmax(acc[ACC_DMAX], d2);
            if (a.ncell > 0 && ia < a.n_active) (void)cell_of(a, ia, c);
        }
        // one (atom, mode) at a time: interleaving the four would need more
        // registers than two waves per SIMD have
        __builtin_amdgcn_sched_barrier(0);
    }
    lds_barrier();   // the tile's y~ (all modes) and centroids are in LDS

    // the next tile's v~ and atom table, in flight over the inverse
    // (the last tile reloads its own values, unused: no branch, so that the
    // registers need no copy that would wait for the loads)
    load_tile_regs<P>(a, has_next ? nb0 : b0, has_next ? nnat : min(16 * T, N - b0), tt, mb, l, t, rv,
                      ratom, rorig);

    // ---- inverse for bead block mb: x^T = x_0 + sum_mode y~^T M
    d4 ax[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) ax[d] = d4{0.0, 0.0, 0.0, 0.0};
    {
        const int li = opaque(l), ir = li & 15, iq = li >> 4, ib = mb * 16 + ir;
        const double *irow = sY + (ra0 + ir) * L::ROW;
        const int is = (ra0 + ir) & L::SWZ;
        prio(2);
#pragma unroll 4
        for (int kb = 0; kb < NK4; ++kb) {
            // B operand M[mode][bead], mode 4 kb + iq: phase mode bead mod P
            const int mm = 4 * kb + iq;
            const int cj = swc<P>(is, mm);
            const double bm = sm.mt[m_index<P>(mm, (mm * ib) & (P - 1))];
#pragma unroll
            for (int d = 0; d < 3; ++d) ax[d] = mfma4(irow[d * P + cj], bm, ax[d]);
        }
        prio(0);
    }
    const int bead = mb * 16 + lr;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int ra = 4 * r + lq;
        const int ia = a0 + ra;
        if (ia >= N) continue;
        const int row = ra0 + ra;
        const double *ar = sA + row * AW;
        const size_t xb = (size_t)ia * 3 * P + bead;
        double e2 = 0.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double xj = ar[TA_X0 + d] + ax[d][r];
            a.x[xb + d * P] = xj;
            const double dd = xj - ar[TA_C + d];
            e2 += dd * dd;
            if (!isfinite(xj)) acc[ACC_BAD] = 1.0;
        }
        if (reinterpret_cast<const int *>(ar + TA_OA)[1]) acc[ACC_EMAX] = fmax(acc[ACC_EMAX], e2);
        if (bead == 0) {
            // the next step's reference is this step's new bead 0: only the
            // centroid mode changes, by -sqrt(P) times the bead's offset
#pragma unroll
            for (int d = 0; d < 3; ++d)
                a.yt[xb + d * P] = sY[row * L::ROW + d * P + swc<P>(row & L::SWZ, 0)] - sqrtP * ax[d][r];
        }
    }
    lds_barrier();   // every wave is done with Y_c and the atom table
}

template <int P, bool OB, bool FC>
__device__ __forceinline__ void mfma_tiles(const FusedArgs &a, int first, int stride, double *partial_out)
{
    using L = Lds<P>;
    constexpr int T = L::T;
    __shared__ __attribute__((aligned(16))) double s_f[L::TILE];
    __shared__ __attribute__((aligned(16))) double s_y0[L::TILE];
    __shared__ __attribute__((aligned(16))) double s_y1[L::TILE];
    __shared__ double s_at[L::A_ELEMS];
    __shared__ double s_mk[L::MK_ELEMS];
    __shared__ double s_mt[L::MT_ELEMS];
    const Smem<P> sm{s_f, s_y0, s_y1, s_at, s_mk, s_mt};
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    const int tt = w / L::NMB, mb = w - tt * L::NMB;
    const int N = a.N;
    const int nbt = (N + 16 * T - 1) / (16 * T);

    // The control block, the per-mode table and the first tile's copies and
    // loads are issued together; a spent budget is acted on once they are
    // complete.
    const long long budget = a.ctl->budget;
    TileCtl tc;
    tc.step = a.ctl->step;
    tc.closing = a.pair && !a.ctl->synced;
    tc.ucom_now = FC && a.ctl->ucom_pending;
#pragma unroll
    for (int d = 0; d < 3; ++d) tc.ucom[d] = FC ? a.ctl->ucom[d] : 0.0;
    constexpr int NMK = (8 * P + kBlock - 1) / kBlock;
    double rmk[NMK];
#pragma unroll
    for (int q = 0; q < NMK; ++q) {
        const int e = t + q * kBlock;
        rmk[q] = e < 8 * P ? a.modes[e] : 0.0;
    }
    // M's distinct entries (m_index): row 1 holds the cosines at phase j, row
    // P - 1 the sines at phase P - j, row P/2 the alternating values
    double rmt = 0.0;
    if (t < 2 * P + 3) {
        const int q = t - P;
        rmt = t < P ? a.M[P + t]
            : t < 2 * P ? a.M[(size_t)(P - 1) * P + ((P - q) & (P - 1))]
            : t == 2 * P ? a.M[0] : a.M[(size_t)(P / 2) * P + (t - 2 * P - 1)];
    }
    double rv[4][3];
    double ratom[RA_COUNT] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int rorig = 0;
    if (first < nbt) {
        const int b0 = first * 16 * T, nat = min(16 * T, N - b0);
        { prio(3); dma_tile<P>(a.yt + (size_t)b0 * 3 * P, s_y0, nat, w, l); prio(0); }
        if (a.pair) { prio(3); dma_tile<P>(a.f + (size_t)b0 * 3 * P, s_f, nat, w, l); prio(0); }
        load_tile_regs<P>(a, b0, nat, tt, mb, l, t, rv, ratom, rorig);
    }
    // a system whose step budget is spent takes no step (uniform per block);
    // the copies into LDS must land before the block ends
    if (budget == 0) {
        __builtin_amdgcn_s_waitcnt(0);
        return;
    }
#pragma unroll
    for (int q = 0; q < NMK; ++q) {
        const int e = t + q * kBlock;
        if (e < 8 * P) s_mk[(e & 7) * P + (e >> 3)] = rmk[q];
    }
    if (t < 2 * P + 3) s_mt[t] = rmt;

    double acc[ACC_COUNT];
#pragma unroll
    for (int q = 0; q < ACC_COUNT; ++q) acc[q] = 0.0;
    // tiles in pairs, so that each one's y~ buffer is fixed at compile time
    for (int bt = first; bt < nbt; bt += 2 * stride) {
        const int b1 = bt + stride;
        mfma_tile<P, OB, FC, 0>(a, sm, tc, bt, b1 < nbt ? b1 : -1, rv, ratom, rorig, acc);
        if (b1 >= nbt) break;
        const int b2 = b1 + stride;
        mfma_tile<P, OB, FC, 1>(a, sm, tc, b1, b2 < nbt ? b2 : -1, rv, ratom, rorig, acc);
    }

    // per-block partials (plain stores; k_finalize runs next); the reduction
    // scratch reuses the f tile, free after the last tile's barrier
    double *red = s_f;
    constexpr int NS = FC ? 8 : 5;   // the fixcom momentum only where it is used
    double s4[NS];
    s4[0] = acc[ACC_EKIN]; s4[1] = acc[ACC_ESP]; s4[2] = acc[ACC_VIR]; s4[3] = acc[ACC_UEXT];
    s4[4] = acc[ACC_K0];
    if constexpr (FC) {
        s4[5] = acc[ACC_P]; s4[6] = acc[ACC_P + 1]; s4[7] = acc[ACC_P + 2];
    }
    double m3[3] = {acc[ACC_EMAX], acc[ACC_DMAX], acc[ACC_BAD]};
    block_sum_max<NS, 3>(s4, m3, red);
    if (t == 0) {
        double *pp = partial_out;
        pp[PF_EKIN] = s4[0];
        pp[PF_ESPRING] = s4[1];
        pp[PF_VIR] = s4[2];
        pp[PF_UEXT] = s4[3];
        pp[PF_EMAX] = m3[0];
        pp[PF_DMAX] = m3[1];
        pp[PF_NONFINITE] = m3[2];
        pp[PF_K0] = s4[4];
        pp[PF_PX] = FC ? s4[NS > 5 ? 5 : 0] : 0.0;
        pp[PF_PY] = FC ? s4[NS > 6 ? 6 : 0] : 0.0;
        pp[PF_PZ] = FC ? s4[NS > 7 ? 7 : 0] : 0.0;
    }
}

// OB: the OBABO splitting (a kernel of its own, so that BAOAB keeps its
// register budget).
template <int P, bool OB, bool FC>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2))) void k_fused_mfma(FusedArgs a)
{
    mfma_tiles<P, OB, FC>(a, blockIdx.x, gridDim.x, a.partials + (size_t)blockIdx.x * PF_COUNT);
}

// Batched: one block per item (system, block tile of T x 16 atoms), for the
// systems with this P; the grid is the item count.
template <int P, bool OB>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2))) void k_fused_mfma_batch(
    const FusedArgs *table, const int2 *items, int n_items)
{
    if ((int)blockIdx.x >= n_items) return;
    const int2 item = items[blockIdx.x];
    const FusedArgs &a = table[item.x];
    // (batches hold no fixcom systems)
    // (a stride past every tile: the item's tile alone; 2 stride stays an int)
    mfma_tiles<P, OB, false>(a, item.y, 1 << 29, a.partials + (size_t)item.y * PF_COUNT);
}

namespace {

template <int P>
int grid_for(int N)
{
    int dev = 0, ncu = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess) ncu = prop.multiProcessorCount;
    }
    int per_cu = 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_fused_mfma<P, false, false>, kBlock,
                                                     0) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    const int want = (N + 16 * Lds<P>::T - 1) / (16 * Lds<P>::T);
    const int cap = ncu * per_cu;
    return want < cap ? want : cap;
}

template <int P>
void launch_one(const FusedArgs &a, int grid, hipStream_t s)
{
    const size_t sm = 0;   // the kernel's LDS is static
    if (a.obabo && a.fixcom)
        hipLaunchKernelGGL((k_fused_mfma<P, true, true>), dim3(grid), dim3(kBlock), sm, s, a);
    else if (a.obabo)
        hipLaunchKernelGGL((k_fused_mfma<P, true, false>), dim3(grid), dim3(kBlock), sm, s, a);
    else if (a.fixcom)
        hipLaunchKernelGGL((k_fused_mfma<P, false, true>), dim3(grid), dim3(kBlock), sm, s, a);
    else
        hipLaunchKernelGGL((k_fused_mfma<P, false, false>), dim3(grid), dim3(kBlock), sm, s, a);
}

template <int P>
void launch_batch(bool ob, const FusedArgs *table, const int2 *items, int n_items, int grid,
                  hipStream_t s)
{
    if (ob)
        hipLaunchKernelGGL((k_fused_mfma_batch<P, true>), dim3(grid), dim3(kBlock), 0, s, table, items,
                           n_items);
    else
        hipLaunchKernelGGL((k_fused_mfma_batch<P, false>), dim3(grid), dim3(kBlock), 0, s, table, items,
                           n_items);
}

}  // namespace

bool fused_mfma_supported(int P) { return P == 16 || P == 32 || P == 64; }

int fused_mfma_grid(int N, int P)
{
    switch (P) {
    case 16: return grid_for<16>(N);
    case 32: return grid_for<32>(N);
    case 64: return grid_for<64>(N);
    default: return 0;
    }
}

void launch_fused_mfma(const FusedArgs &a, int grid, hipStream_t s)
{
    switch (a.P) {
    case 16: launch_one<16>(a, grid, s); break;
    case 32: launch_one<32>(a, grid, s); break;
    case 64: launch_one<64>(a, grid, s); break;
    default: break;
    }
}

int mfma_block_tiles(int N, int P)
{
    const int T = kWaves / (P / 16);
    return (N + 16 * T - 1) / (16 * T);
}

void set_mfma_batch_smem()
{
    // the batched kernels' LDS is static: nothing to raise
}

void launch_fused_mfma_batch(int P, bool obabo, const FusedArgs *table, const int2 *items, int n_items,
                             int grid, hipStream_t s)
{
    switch (P) {
    case 16: launch_batch<16>(obabo, table, items, n_items, grid, s); break;
    case 32: launch_batch<32>(obabo, table, items, n_items, grid, s); break;
    case 64: launch_batch<64>(obabo, table, items, n_items, grid, s); break;
    default: break;
    }
}

}  // namespace pimd
