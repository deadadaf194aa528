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
// A block works on T = 64/P tiles of 16 atoms at once.  The f and y~ values of
// those atoms are loaded into LDS with coalesced reads (f in [atom][3P] rows,
// y~ in [dim][atom][mode] rows); each tile is shared by P/16 waves, wave w
// taking mode block (and, in the inverse, bead block) w % (P/16).  Per dim d
// the wave forms
//   f~^T[atom][mode] = sum_bead f^T[atom][bead] M^T[bead][mode]
//   x^T[atom][bead]  = x_0 + sum_mode y~^T[atom][mode] M[mode][bead]
// with the B operands (4 rows x 16 columns of M^T or M) read from global
// memory, where they stay cache resident.
//
// Operand layout of the instruction (checked on the device): A[i][k] in lane
// i + 16k, B[k][j] in lane j + 16k, and accumulator register r of lane l
// holds D[4r + l/16][l%16].  With atoms as rows, lane l holds, for one mode
// (column l%16 of the wave's mode block), the four atoms 4r + l/16: the
// per-(atom, mode) work (B, A, O with one Philox call for the three dims, A)
// runs in registers, and v~ and y~ are read and written as 128-byte segments.
//
// LDS bank swizzle.  A 64-bit LDS access of a wave is served in groups of 16
// or 32 lanes; the banks hold 8-byte words at the word index modulo 16 or 32.
// The operand reads take lane (i, k) -> row i, column c + k (i < 16, k < 4),
// the update takes lane (i, k) -> row 4r + k, column c + i.  Column j of row a
// is stored at j ^ sw(a), sw(a) = (a mod 16) + 16 (a mod 2) when rows are a
// multiple of 32 words long and sw(a) = a mod 16 when they are 16 modulo 32
// (the row stride supplies the 16 (a mod 2) then).  Both patterns then hit
// distinct banks within every group of 16 and of 32 lanes.
#include "pimd_device.h"
#include "pimd_internal.h"

namespace pimd {

typedef double d4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int kWaves = kBlock / 64;

__device__ __forceinline__ d4 mfma4(double a, double b, d4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <int P>
struct Lds {
    static constexpr int NMB = P / 16;            // mode blocks = waves per atom tile
    static constexpr int T = kWaves / NMB;        // atom tiles per block
    static constexpr int XS = 3 * P;              // atom row of the f tile
    static constexpr int PS = P;                  // row of the y~ tile
    static constexpr int XY_ELEMS = 3 * 16 * PS;  // y~ [3][16][PS]
    static constexpr int F_ELEMS = 16 * XS;       // f [16][XS]
    static constexpr int AT_W = 12;               // per-atom row of the atom table
    static constexpr int AT_ELEMS = 16 * AT_W;
    static constexpr int C_ELEMS = 16 * 4;        // centroids [atom][d]
    static constexpr int TILE = XY_ELEMS + F_ELEMS + AT_ELEMS + C_ELEMS;
    static constexpr int MK_ELEMS = 8 * P;        // the per-mode table, shared by the block
    static constexpr int bytes = 8 * (T * TILE + MK_ELEMS);
    static constexpr int NLD = 16 * T * 3 * P / kBlock;   // tile elements per thread
    static_assert(16 * T * 3 * P == NLD * kBlock, "tile elements split evenly");
    static_assert(16 * T <= kBlock, "one thread per atom of the block tile");
};

// column swizzle of row a (a < 16) in a tile whose rows are `row` words long
template <int row>
__device__ __forceinline__ int sw(int a)
{
    static_assert(row % 32 == 0 || row % 32 == 16, "row length 0 or 16 modulo 32");
    return (row % 32 == 0) ? ((a & 15) | ((a & 1) << 4)) : (a & 15);
}

// atom-table columns (per atom of a tile)
enum { TA_X0 = 0, TA_HM = 3, TA_IM = 4, TA_SG = 5, TA_ACT = 6, TA_ORIG = 7, TA_CREF = 8 };

}  // namespace

// Processes block tiles first, first + stride, ... (T*16 atoms each) of one
// system and writes one set of partials for the block.
//
// Per block tile: every global read of the tile (x, f, this lane's v~, the
// per-atom table) is issued at once into registers, before the barrier that
// releases the previous tile's LDS; the forward products read x and f from
// LDS; after a barrier the y~ of the update overwrite the x region; a last
// barrier precedes the inverse products.
template <int P, bool OB, bool FC>
__device__ void mfma_tiles(const FusedArgs &a, int first, int stride, double *smem,
                           double *partial_out)
{
    using L = Lds<P>;
    constexpr int NMB = L::NMB, T = L::T, XS = L::XS, PS = L::PS, NLD = L::NLD, AW = L::AT_W;
    constexpr int NK4 = P / 4;        // k-steps of 4
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    const int lr = l & 15, lq = l >> 4;
    const int tt = w / NMB;           // this wave's atom tile within the block
    const int mb = w - tt * NMB;      // this wave's mode block (and bead block)
    double *sY = smem + tt * L::TILE;             // y~ [3][16][PS]: carried, then new
    double *sF = sY + L::XY_ELEMS;                // [16][XS]: f
    double *sA = sF + L::F_ELEMS;                 // [16][AW]: atom table
    double *sC = sA + L::AT_ELEMS;                // [16][4]: centroids
    // B operands: forward M^T[4kb + lq][mb*16 + lr], inverse M[4kb + lq][mb*16 + lr];
    // both are 4 rows x 16 consecutive columns per instruction (coalesced)
    const double *bmT = a.MT + lq * P + mb * 16 + lr;
    const double *bmM = a.M + lq * P + mb * 16 + lr;

    const int N = a.N;
    // The control block, the per-mode table and the first tile are read
    // together; a spent budget is acted on once the tile's reads are issued.
    const long long budget = a.ctl->budget;
    const unsigned long long step = a.ctl->step;
    const int synced = a.ctl->synced;
    // fixcom: the last step's centroid-mode velocity still to be removed
    const bool ucom_now = FC && a.ctl->ucom_pending;
    const double ucom[3] = {a.ctl->ucom[0], a.ctl->ucom[1], a.ctl->ucom[2]};
    // a system whose step budget is spent takes no step (uniform per block)
    const bool spent = budget == 0;
    const bool ext = !a.pair;
    const bool closing = a.pair && !synced;
    const bool need_f = a.pair != 0;
    const double sqrtP = sqrt((double)P);
    const int m = mb * 16 + lr;       // this lane's mode
    double *sMk = smem + T * L::TILE;             // [8][P]: per-mode coefficients
    constexpr int NMK = (8 * P + kBlock - 1) / kBlock;
    double rmk[NMK];
#pragma unroll
    for (int q = 0; q < NMK; ++q) {
        const int e = t + q * kBlock;
        rmk[q] = e < 8 * P ? a.modes[e] : 0.0;
    }
    const double *mk = sMk + m;                   // coefficient q at mk[q * P]
    const double off = (m == 0) ? sqrtP : 0.0;

    double acc_ekin = 0.0, acc_esp = 0.0, acc_vir = 0.0, acc_uext = 0.0;
    double acc_emax = 0.0, acc_dmax = 0.0, acc_bad = 0.0;
    double acc_p[3] = {0.0, 0.0, 0.0};   // fixcom: sum of hm v~0 after a step's end
    double acc_k0 = 0.0;                 // sum of hm |v~0|^2 at the estimator point

    const int nbt = (N + 16 * T - 1) / (16 * T);
    for (int bt = first; bt < nbt; bt += stride) {
        const int b0 = bt * 16 * T;                    // first atom of the block tile
        const int nat = min(16 * T, N - b0);
        const int nel = nat * 3 * P;
        const int a0 = b0 + tt * 16;                   // first atom of this wave's tile

        // ---- all global reads of the tile, in flight together: the carried
        // normal-mode positions y~ and the forces (coalesced tile copies),
        // this lane's v~, the per-atom table and each atom's bead-0 position
        double ry[NLD], rf[NLD];
        {
            const double *yg = a.yt + (size_t)b0 * 3 * P;
            const double *fg = a.f + (size_t)b0 * 3 * P;
#pragma unroll
            for (int q = 0; q < NLD; ++q) {
                const int e = t + q * kBlock;
                ry[q] = e < nel ? yg[e] : 0.0;
                rf[q] = (need_f && e < nel) ? fg[e] : 0.0;
            }
        }
        double rv[4][3];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int ia = a0 + 4 * r + lq;
            const size_t vb = (size_t)ia * 3 * P + m;
#pragma unroll
            for (int d = 0; d < 3; ++d) rv[r][d] = ia < N ? a.v[vb + d * P] : 0.0;
        }
        double ratom[11] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        if (t < nat) {
            const int ia = b0 + t;
#pragma unroll
            for (int q = 0; q < 4; ++q) ratom[q] = a.atoms[ia * 4 + q];
            ratom[4] = (double)a.orig[ia];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                ratom[5 + d] = a.cref[ia * 3 + d];
                ratom[8 + d] = a.x[(size_t)ia * 3 * P + d * P];
            }
        }

        if (spent) return;
        __syncthreads();                               // previous tile's LDS use is done
        if (bt == first) {
#pragma unroll
            for (int q = 0; q < NMK; ++q) {
                const int e = t + q * kBlock;
                if (e < 8 * P) sMk[(e & 7) * P + (e >> 3)] = rmk[q];
            }
        }
#pragma unroll
        for (int q = 0; q < NLD; ++q) {
            const int e = t + q * kBlock;
            const int at = e / (3 * P), rr = e - at * (3 * P);
            const int d = rr / P, mm = rr - d * P;
            double *tile = smem + (at >> 4) * L::TILE;
            const int a16 = at & 15;
            tile[(d * 16 + a16) * PS + (mm ^ sw<PS>(a16))] = ry[q];      // y~ [d][atom][mode]
            tile[L::XY_ELEMS + a16 * XS + (rr ^ sw<XS>(a16))] = rf[q];   // f [atom][d*P + bead]
        }
        if (t < 16 * T) {
            double *ar = smem + (t >> 4) * L::TILE + L::XY_ELEMS + L::F_ELEMS + (t & 15) * AW;
            ar[TA_HM] = ratom[AT_HALF_M];
            ar[TA_IM] = ratom[AT_INV_M];
            ar[TA_SG] = ratom[AT_SIGMA];
            ar[TA_ACT] = ratom[AT_ACTIVE];
            ar[TA_ORIG] = ratom[4];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                ar[TA_CREF + d] = ratom[5 + d];
                ar[TA_X0 + d] = ratom[8 + d];
            }
        }
        __syncthreads();

        // ---- forward products: f~ of mode block mb for the tile's 16 atoms
        // (the positions' modes are carried from the previous step)
        const bool ok_op = (a0 + lr) < N;
        d4 af[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) af[d] = d4{0.0, 0.0, 0.0, 0.0};
        if (need_f) {
            const double *fr = sF + lr * XS;
            const int swf = sw<XS>(lr);
#pragma unroll 4
            for (int kb = 0; kb < NK4; ++kb) {
                const int bead = 4 * kb + lq;
                const double bm = bmT[4 * kb * P];
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const double fv = ok_op ? fr[(d * P + bead) ^ swf] : 0.0;
                    af[d] = mfma4(fv, bm, af[d]);
                }
            }
        }

        // ---- per (atom, mode) update: lane l, register r: atom a0 + 4r + lq, mode m
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int ra = 4 * r + lq;
            const int ia = a0 + ra;
            if (ia >= N) continue;
            const double *ar = sA + ra * AW;
            const double hm = ar[TA_HM], im = ar[TA_IM], sg = ar[TA_SG];
            const int cy = m ^ sw<PS>(ra);
            double xt[3], ft[3], vt[3], x0[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                xt[d] = sY[(d * 16 + ra) * PS + cy];
                ft[d] = af[d][r];
                x0[d] = ar[TA_X0 + d];
                vt[d] = rv[r][d];
            }
            if (ucom_now && m == 0) {
#pragma unroll
                for (int d = 0; d < 3; ++d) vt[d] -= ucom[d];
            }
            if (ext) {
#pragma unroll
                for (int d = 0; d < 3; ++d) ft[d] = -2.0 * hm * a.omega2 * (xt[d] + off * x0[d]);
            }
            // PILE-L at P*T over one O step (dt in BAOAB, dt/2 in OBABO), noise
            // of step s_ and O step q_ of that step
            auto o_step = [&](unsigned long long s_, unsigned long long q_) {
                double z[3];
                gauss3(a.seed, (unsigned long long)ar[TA_ORIG], (unsigned long long)m, s_, z, q_);
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
                    for (int d = 0; d < 3; ++d) acc_p[d] += hm * vt[d];
                }
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const double kd = hm * vt[d] * vt[d];
                    acc_ekin += kd;
                    if (m == 0) acc_k0 += kd;
                    acc_esp += hm * mk[MD_SPRING * P] * xt[d] * xt[d];
                    acc_vir += mk[MD_NONCENTROID * P] * xt[d] * ft[d];
                }
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
                    for (int d = 0; d < 3; ++d) acc_p[d] += hm * vt[d];
                }
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const double xa = xt[d] + off * x0[d];
                    acc_ekin += hm * vt[d] * vt[d];
                    acc_esp += hm * mk[MD_SPRING * P] * xt[d] * xt[d];
                    acc_uext += hm * a.omega2 * xa * xa;
                    acc_vir += mk[MD_NONCENTROID * P] * xt[d] * ft[d];
                }
            }
            const size_t vb = (size_t)ia * 3 * P + m;
            a.v[vb] = vt[0]; a.v[vb + P] = vt[1]; a.v[vb + 2 * P] = vt[2];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                if (!isfinite(vt[d])) acc_bad = 1.0;
                sY[(d * 16 + ra) * PS + cy] = xt[d];
                // carried to the next step; the centroid mode is re-referenced
                // to the new bead 0 after the inverse
                if (m != 0) a.yt[vb + d * P] = xt[d];
            }
            if (m == 0) {
                double d2 = 0.0, c[3];
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    c[d] = x0[d] + xt[d] / sqrtP;
                    sC[ra * 4 + d] = c[d];
                    a.cent[ia * 3 + d] = c[d];
                    const double dd = c[d] - ar[TA_CREF + d];
                    d2 += dd * dd;
                }
                if (ar[TA_ACT] != 0.0) acc_dmax = fmax(acc_dmax, d2);
                if (a.ncell > 0 && ia < a.n_active) (void)cell_of(a, ia, c);
            }
        }
        __syncthreads();   // the tile's y~ (all modes) and centroids are in LDS

        // ---- inverse for bead block mb: x^T = x_0 + sum_mode y~^T M
        d4 ax[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) ax[d] = d4{0.0, 0.0, 0.0, 0.0};
        const int swy = sw<PS>(lr);
#pragma unroll 4
        for (int kb = 0; kb < NK4; ++kb) {
            const int mm = (4 * kb + lq) ^ swy;
            const double bm = bmM[4 * kb * P];
#pragma unroll
            for (int d = 0; d < 3; ++d) ax[d] = mfma4(sY[(d * 16 + lr) * PS + mm], bm, ax[d]);
        }
        const int bead = mb * 16 + lr;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int ra = 4 * r + lq;
            const int ia = a0 + ra;
            if (ia >= N) continue;
            const double *ar = sA + ra * AW;
            const size_t xb = (size_t)ia * 3 * P + bead;
            double e2 = 0.0;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const double xj = ar[TA_X0 + d] + ax[d][r];
                a.x[xb + d * P] = xj;
                const double dd = xj - sC[ra * 4 + d];
                e2 += dd * dd;
                if (!isfinite(xj)) acc_bad = 1.0;
            }
            if (ar[TA_ACT] != 0.0) acc_emax = fmax(acc_emax, e2);
            if (bead == 0) {
                // the next step's reference is this step's new bead 0: only the
                // centroid mode changes, by -sqrt(P) times the bead's offset
#pragma unroll
                for (int d = 0; d < 3; ++d)
                    a.yt[xb + d * P] = sY[(d * 16 + ra) * PS + sw<PS>(ra)] - sqrtP * ax[d][r];
            }
        }
    }

    // per-block partials (plain stores; k_finalize runs next); the reduction
    // scratch reuses the tiles' LDS once every wave is done with it
    if (spent) return;
    __syncthreads();
    double *red = smem;
    constexpr int NS = FC ? 8 : 5;   // the fixcom momentum only where it is used
    double s4[NS];
    s4[0] = acc_ekin; s4[1] = acc_esp; s4[2] = acc_vir; s4[3] = acc_uext; s4[4] = acc_k0;
    if constexpr (FC) {
        s4[5] = acc_p[0]; s4[6] = acc_p[1]; s4[7] = acc_p[2];
    }
    double m3[3] = {acc_emax, acc_dmax, acc_bad};
    block_sum_max<NS, 3>(s4, m3, red);
    const double emax = m3[0], dmax = m3[1], bad = m3[2];
    if (t == 0) {
        double *pp = partial_out;
        pp[PF_EKIN] = s4[0];
        pp[PF_ESPRING] = s4[1];
        pp[PF_VIR] = s4[2];
        pp[PF_UEXT] = s4[3];
        pp[PF_EMAX] = emax;
        pp[PF_DMAX] = dmax;
        pp[PF_NONFINITE] = bad;
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
    extern __shared__ double smem[];
    mfma_tiles<P, OB, FC>(a, blockIdx.x, gridDim.x, smem, a.partials + (size_t)blockIdx.x * PF_COUNT);
}

// Batched: one block per item (system, block tile of T x 16 atoms), for the
// systems with this P; the grid is the item count.
template <int P, bool OB>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2))) void k_fused_mfma_batch(
    const FusedArgs *table, const int2 *items, int n_items)
{
    extern __shared__ double smem[];
    if ((int)blockIdx.x >= n_items) return;
    const int2 item = items[blockIdx.x];
    const FusedArgs &a = table[item.x];
    // (batches hold no fixcom systems)
    mfma_tiles<P, OB, false>(a, item.y, 1 << 30, smem, a.partials + (size_t)item.y * PF_COUNT);
}

namespace {

template <int P>
int grid_for(int N)
{
    (void)hipFuncSetAttribute((const void *)k_fused_mfma<P, false, false>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, Lds<P>::bytes);
    (void)hipFuncSetAttribute((const void *)k_fused_mfma<P, true, false>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, Lds<P>::bytes);
    (void)hipFuncSetAttribute((const void *)k_fused_mfma<P, false, true>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, Lds<P>::bytes);
    (void)hipFuncSetAttribute((const void *)k_fused_mfma<P, true, true>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, Lds<P>::bytes);
    int dev = 0, ncu = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess) ncu = prop.multiProcessorCount;
    }
    int per_cu = 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_fused_mfma<P, false, false>, kBlock,
                                                     Lds<P>::bytes) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    const int want = (N + 16 * Lds<P>::T - 1) / (16 * Lds<P>::T);
    const int cap = ncu * per_cu;
    return want < cap ? want : cap;
}

template <int P>
void launch_one(const FusedArgs &a, int grid, hipStream_t s)
{
    const size_t sm = Lds<P>::bytes;
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
        hipLaunchKernelGGL((k_fused_mfma_batch<P, true>), dim3(grid), dim3(kBlock), Lds<P>::bytes, s,
                           table, items, n_items);
    else
        hipLaunchKernelGGL((k_fused_mfma_batch<P, false>), dim3(grid), dim3(kBlock), Lds<P>::bytes, s,
                           table, items, n_items);
}

template <int P>
void set_batch_attr()
{
    (void)hipFuncSetAttribute((const void *)k_fused_mfma_batch<P, false>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, Lds<P>::bytes);
    (void)hipFuncSetAttribute((const void *)k_fused_mfma_batch<P, true>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, Lds<P>::bytes);
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
    set_batch_attr<16>();
    set_batch_attr<32>();
    set_batch_attr<64>();
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
