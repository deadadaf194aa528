// HIP kernels of libpimd.so for gfx950 (CDNA4, wave64).
//
// k_fused  : one pass over (y~, v~, f) per step on the FP64 vector ALUs:
//            f~ = M f (App. B; the positions' modes y~ are carried between
//            steps), the pending closing half-kick and the estimators
//            (App. A), then the step's B, A, O, A (BAOAB) or O, B, A, A
//            (OBABO) per mode (Eqs. 1-2, App. D), and the inverse transform.
//            With an external trap the forces are evaluated in normal modes
//            inside the same pass and the whole step is this one kernel.
//            (The matrix-core variant is k_fused_mfma, pimd_fused_mfma.hip.)
// k_pair   : bead-batched short-range forces for all P replicas in one
//            launch (LJ among active atoms + harmonic bonds), each atom's
//            neighbor list rebuilt from the centroid cells when requested;
//            per block, the energy and the cell virial (the pressures of
//            App. A).  k_pair_npt: the same with the box from the control
//            block (the barostat's passes are in pimd_npt.hip).
// k_finalize: one block after the step pass; combines the per-block partials
//            in block order (deterministic), records estimators and running
//            sums, advances the step counter, decides list rebuilds and, at
//            a rebuild, builds the centroid cell lists.
#include "pimd_device.h"
#include "pimd_internal.h"

namespace pimd {

// --------------------------------------------------------------------------
// Fused step kernel (vector ALUs).
// Shared memory: M^T padded [P][P+1], tile X [A][3][P] (the modes y~, then
// the new ones for the inverse), tile F [A][3][P] (f, or v in PREP),
// centroids [A][3], bead-0 references [A][3].
// --------------------------------------------------------------------------
int fused_smem_bytes(int P)
{
    const int A = kBlock / P;
    return (int)sizeof(double) * (P * (P + 1) + 2 * 3 * A * P + 6 * A);
}

// Processes tiles t0, t0 + tstride, ... of one system and writes one set of
// partials.  stage_m = false keeps the matrix already staged in shared
// memory (same system or same P as the previous call of this block).
// FC: the system removes its centroids' center-of-mass velocity (fixcom); a
// separate instantiation, so that the others carry none of its code.
template <bool FC>
__device__ void fused_tiles(const FusedArgs &a, int t0, int tstride, double *smem, double *red,
                           double *partial_out, bool stage_m)
{
    const int P = a.P, N = a.N;
    const int A = kBlock / P;
    const int PS = P + 1;
    double *sMT = smem;                 // sMT[j*PS + k] = M[k][j]
    double *sX = sMT + P * PS;          // [A][3][P]
    double *sF = sX + 3 * A * P;        // [A][3][P]
    double *sC = sF + 3 * A * P;        // [A][3] centroids
    double *sR = sC + 3 * A;            // [A][3] bead-0 reference positions
    const int t = threadIdx.x;

    // The control block, the matrix (for P <= 32) and the first tile are read
    // together: nothing waits for the control block before the tile's reads
    // are issued, and a spent budget is acted on once they are in flight.
    constexpr int NM = 4;               // matrix elements held per thread (P*P <= NM*kBlock)
    const bool m_regs = P * P <= NM * kBlock;
    double mreg[NM];
#pragma unroll
    for (int q = 0; q < NM; ++q) {
        const int e = t + q * kBlock;
        mreg[q] = (stage_m && m_regs && e < P * P) ? a.M[e] : 0.0;
    }
    const long long budget = a.ctl->budget;
    const unsigned long long step = a.ctl->step;
    const int synced = a.ctl->synced;
    // fixcom: the last step's centroid-mode velocity still to be removed
    const bool ucom_now = FC && a.mode == FUSED_STEP && a.ctl->ucom_pending;
    const double ucom[3] = {a.ctl->ucom[0], a.ctl->ucom[1], a.ctl->ucom[2]};
    // a system whose step budget is spent takes no step (uniform per block)
    const bool spent = (a.mode == FUSED_STEP && budget == 0);

    const int mode = a.mode;
    const int ext = !a.pair;                                    // forces in-kernel
    const bool closing = (mode == FUSED_STEP || mode == FUSED_CLOSE) && !synced && a.pair;
    const bool est_now = closing || mode == FUSED_EST;          // estimators of this state
    // f is read whenever a pass may need it (a closing pass finds out from
    // the control block), so that its reads need not wait for that block
    const bool need_f = a.pair && mode != FUSED_PREP;
    const bool inverse = (mode == FUSED_STEP);
    const bool carry = (mode == FUSED_STEP);     // positions' modes carried in yt
    const double sqrtP = sqrt((double)P);

    const int la = t / P, k = t - (t / P) * P;
    const bool lane_ok = la < A;

    double acc_ekin = 0.0, acc_esp = 0.0, acc_vir = 0.0, acc_uext = 0.0;
    double acc_emax = 0.0, acc_dmax = 0.0, acc_bad = 0.0;
    double acc_p[3] = {0.0, 0.0, 0.0};   // fixcom: sum of hm v~0 after a step's end
    double acc_k0 = 0.0;                 // sum of hm |v~0|^2 at the estimator point

    double mk[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) mk[q] = lane_ok ? a.modes[k * 8 + q] : 0.0;

    const int ntiles = (N + A - 1) / A;
    for (int tile = t0; tile < ntiles; tile += tstride) {
        const int a0 = tile * A;
        const int na = min(A, N - a0);
        const int nel = na * 3 * P;
        const bool act = lane_ok && la < na;
        const int i = a0 + la;
        // Every global read of the tile in flight at once, before the barrier
        // that frees the previous tile's LDS: the x tile and the f (or PREP's
        // v) tile, 3 doubles each per thread (A*3P <= 3*256), this lane's v~
        // and per-atom constants.
        // The step pass reads the positions' modes carried from the previous
        // step (y~ relative to bead 0) and each atom's bead-0 position instead
        // of the x tile.
        constexpr int NL = 3;
        const double *xg = a.x + (size_t)a0 * 3 * P;
        const double *fg = need_f ? a.f + (size_t)a0 * 3 * P
                                  : (mode == FUSED_PREP ? a.vin + (size_t)a0 * 3 * P : nullptr);
        double rx[NL], rf[NL];
#pragma unroll
        for (int q = 0; q < NL; ++q) {
            const int e = t + q * kBlock;
            rx[q] = (!carry && e < nel) ? xg[e] : 0.0;
            rf[q] = (fg && e < nel) ? fg[e] : 0.0;
        }
        double hm = 0.0, im = 0.0, sg = 0.0, active = 0.0;
        double vpre[3] = {0.0, 0.0, 0.0}, ypre[3] = {0.0, 0.0, 0.0}, xref[3] = {0.0, 0.0, 0.0};
        double cref[3] = {0.0, 0.0, 0.0};
        unsigned oi = 0;
        if (act) {
            hm = a.atoms[i * 4 + AT_HALF_M];
            im = a.atoms[i * 4 + AT_INV_M];
            sg = a.atoms[i * 4 + AT_SIGMA];
            active = a.atoms[i * 4 + AT_ACTIVE];
            oi = (unsigned)a.orig[i];
            const size_t vb = (size_t)i * 3 * P + k;
            if (mode != FUSED_PREP) {
                vpre[0] = a.v[vb]; vpre[1] = a.v[vb + P]; vpre[2] = a.v[vb + 2 * P];
            }
            if (carry) {
                ypre[0] = a.yt[vb]; ypre[1] = a.yt[vb + P]; ypre[2] = a.yt[vb + 2 * P];
                const size_t xb0 = (size_t)i * 3 * P;
                xref[0] = a.x[xb0]; xref[1] = a.x[xb0 + P]; xref[2] = a.x[xb0 + 2 * P];
            }
            if (k == 0 && (mode == FUSED_STEP || mode == FUSED_PREP)) {
                cref[0] = a.cref[i * 3]; cref[1] = a.cref[i * 3 + 1]; cref[2] = a.cref[i * 3 + 2];
            }
        }
        if (spent) return;
        __syncthreads();   // the previous tile's (or call's) shared-memory reads are done
        if (stage_m && tile == t0) {
            if (m_regs) {
#pragma unroll
                for (int q = 0; q < NM; ++q) {
                    const int e = t + q * kBlock;
                    if (e < P * P) {
                        const int kk = e / P, j = e - kk * P;
                        sMT[j * PS + kk] = mreg[q];
                    }
                }
            } else {
                for (int e = t; e < P * P; e += kBlock) {
                    const int kk = e / P, j = e - kk * P;
                    sMT[j * PS + kk] = a.M[e];
                }
            }
        }
#pragma unroll
        for (int q = 0; q < NL; ++q) {
            const int e = t + q * kBlock;
            if (e < nel) {
                if (!carry) sX[e] = rx[q];
                if (fg) sF[e] = rf[q];
            }
        }
        __syncthreads();

        double xt[3] = {0.0, 0.0, 0.0}, ft[3] = {0.0, 0.0, 0.0}, vt[3] = {0.0, 0.0, 0.0};
        double ref[3] = {0.0, 0.0, 0.0};
        if (act) {
            // Forward transforms of this mode.  Positions are carried relative
            // to the atom's bead 0 for the whole step: y_j = x_j - x_0 (exact),
            // y~ = M y.  Since the non-centroid rows of M sum to zero,
            // y~_k = x~_k for k >= 1 and y~_0 = x~_0 - sqrt(P) x_0; the small
            // relative values keep full absolute accuracy for box-size
            // unwrapped coordinates.  Forces (and v in PREP) have no offset.
            const double *xr = sX + la * 3 * P;
            const double *fr = sF + la * 3 * P;
            const bool tf = need_f || mode == FUSED_PREP;
            if (carry) {
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    xt[d] = ypre[d];
                    ref[d] = xref[d];
                }
                if (tf) {
                    for (int j = 0; j < P; ++j) {
                        const double m = sMT[j * PS + k];
                        ft[0] += m * fr[j];
                        ft[1] += m * fr[P + j];
                        ft[2] += m * fr[2 * P + j];
                    }
                }
            } else {
                const double r0 = xr[0], r1 = xr[P], r2 = xr[2 * P];
                for (int j = 0; j < P; ++j) {
                    const double m = sMT[j * PS + k];
                    xt[0] += m * (xr[j] - r0);
                    xt[1] += m * (xr[P + j] - r1);
                    xt[2] += m * (xr[2 * P + j] - r2);
                    if (tf) {
                        ft[0] += m * fr[j];
                        ft[1] += m * fr[P + j];
                        ft[2] += m * fr[2 * P + j];
                    }
                }
                ref[0] = r0; ref[1] = r1; ref[2] = r2;
            }
            const size_t vb = (size_t)i * 3 * P + k;
            if (mode == FUSED_PREP) {
                // the carried modes of the positions, relative to bead 0
                a.yt[vb] = xt[0]; a.yt[vb + P] = xt[1]; a.yt[vb + 2 * P] = xt[2];
            }
            if (mode == FUSED_PREP) {
                vt[0] = ft[0]; vt[1] = ft[1]; vt[2] = ft[2];
                ft[0] = ft[1] = ft[2] = 0.0;
            } else {
                vt[0] = vpre[0]; vt[1] = vpre[1]; vt[2] = vpre[2];
            }
            if (ucom_now && k == 0) {
#pragma unroll
                for (int d = 0; d < 3; ++d) vt[d] -= ucom[d];
            }
            // absolute mode coordinate x~_k (differs from y~_k only for k = 0)
            const double off = (k == 0) ? sqrtP : 0.0;
            if (ext) {
                // external trap: the normal-mode force is -m mvv2e omega^2 x~
#pragma unroll
                for (int d = 0; d < 3; ++d) ft[d] = -2.0 * hm * a.omega2 * (xt[d] + off * ref[d]);
            }
            // PILE-L at P*T over one O step (dt in BAOAB, dt/2 in OBABO), noise
            // of step s_ and O step q_ of that step
            auto o_step = [&](unsigned long long s_, unsigned long long q_) {
                double z[3];
                gauss3(a.seed, oi, (unsigned)k, s_, z, (unsigned)q_);
#pragma unroll
                for (int d = 0; d < 3; ++d) vt[d] = mk[MD_C1] * vt[d] + mk[MD_C2] * sg * z[d];
            };
            // A(dt/2): exact free-ring-polymer flow of this mode
            auto a_step = [&]() {
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const double q = xt[d], p = vt[d];
                    xt[d] = mk[MD_A00] * q + mk[MD_A01] * p;
                    vt[d] = mk[MD_A10] * q + mk[MD_A11] * p;
                }
            };
            if (closing) {
#pragma unroll
                for (int d = 0; d < 3; ++d) vt[d] += a.hdt * im * ft[d];
                // OBABO: the last O of the step being closed
                if (a.obabo && a.nvt) o_step(step - 1, 1);
                if (FC && k == 0) {
#pragma unroll
                    for (int d = 0; d < 3; ++d) acc_p[d] += hm * vt[d];
                }
            }
            if (est_now) {
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const double kd = hm * vt[d] * vt[d];
                    acc_ekin += kd;
                    if (k == 0) acc_k0 += kd;
                    acc_esp += hm * mk[MD_SPRING] * xt[d] * xt[d];
                    acc_vir += mk[MD_NONCENTROID] * xt[d] * ft[d];
                    const double xa = xt[d] + off * ref[d];
                    acc_uext += hm * a.omega2 * xa * xa;
                }
            }
            if (mode == FUSED_STEP) {
                if (a.obabo) {
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
                        ft[d] = -2.0 * hm * a.omega2 * (xt[d] + off * ref[d]);
                        vt[d] += a.hdt * im * ft[d];
                    }
                    if (a.obabo && a.nvt) o_step(step, 1);
                    if (FC && k == 0) {
#pragma unroll
                        for (int d = 0; d < 3; ++d) acc_p[d] += hm * vt[d];
                    }
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        const double xa = xt[d] + off * ref[d];
                        acc_ekin += hm * vt[d] * vt[d];
                        acc_esp += hm * mk[MD_SPRING] * xt[d] * xt[d];
                        acc_uext += hm * a.omega2 * xa * xa;
                        acc_vir += mk[MD_NONCENTROID] * xt[d] * ft[d];
                    }
                }
            }
            if (mode == FUSED_STEP || mode == FUSED_CLOSE || mode == FUSED_PREP) {
                a.v[vb] = vt[0]; a.v[vb + P] = vt[1]; a.v[vb + 2 * P] = vt[2];
            }
#pragma unroll
            for (int d = 0; d < 3; ++d)
                if (!isfinite(vt[d])) acc_bad = 1.0;
            if (k == 0 && (mode == FUSED_PREP)) {
#pragma unroll
                for (int d = 0; d < 3; ++d) sC[la * 3 + d] = ref[d] + xt[d] / sqrtP;
            }
        }
        if (mode == FUSED_STEP) {
            __syncthreads();   // all reads of sX done
            if (act) {
                const size_t yb = (size_t)i * 3 * P + k;
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    sX[(la * 3 + d) * P + k] = xt[d];
                    // carried to the next step; the centroid mode is
                    // re-referenced to the new bead 0 after the inverse
                    if (k != 0) a.yt[yb + d * P] = xt[d];
                }
                if (k == 0) {
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        sC[la * 3 + d] = ref[d] + xt[d] / sqrtP;
                        sR[la * 3 + d] = ref[d];
                    }
                }
            }
        }
        if (mode == FUSED_STEP || mode == FUSED_PREP) {
            __syncthreads();
            if (act) {
                // bead j = k of atom i: x_j = sum_k M_kj x~_k (STEP) or x as loaded (PREP)
                const int j = k;
                double xj[3];
                if (inverse) {
                    // y_j = sum_k M_kj y~_k (all small), then x_j = x_0 + y_j
                    xj[0] = xj[1] = xj[2] = 0.0;
                    const double *xr = sX + la * 3 * P;
                    for (int m = 0; m < P; ++m) {
                        const double w = sMT[j * PS + m];   // M[m][j]
                        xj[0] += w * xr[m];
                        xj[1] += w * xr[P + m];
                        xj[2] += w * xr[2 * P + m];
                    }
                    const size_t xb = (size_t)i * 3 * P + j;
                    if (j == 0) {
                        // the next step's reference is the new bead 0: only the
                        // centroid mode changes, by -sqrt(P) times its offset
#pragma unroll
                        for (int d = 0; d < 3; ++d)
                            a.yt[xb + d * P] = sX[(la * 3 + d) * P] - sqrtP * xj[d];
                    }
#pragma unroll
                    for (int d = 0; d < 3; ++d) xj[d] += sR[la * 3 + d];
                    a.x[xb] = xj[0]; a.x[xb + P] = xj[1]; a.x[xb + 2 * P] = xj[2];
                } else {
#pragma unroll
                    for (int d = 0; d < 3; ++d) xj[d] = sX[(la * 3 + d) * P + j];
                }
                double e2 = 0.0;
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const double dd = xj[d] - sC[la * 3 + d];
                    e2 += dd * dd;
                    if (!isfinite(xj[d])) acc_bad = 1.0;
                }
                if (active != 0.0) acc_emax = fmax(acc_emax, e2);
                if (j == 0) {
                    double d2 = 0.0, c[3];
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        c[d] = sC[la * 3 + d];
                        a.cent[i * 3 + d] = c[d];
                        const double dd = c[d] - cref[d];
                        d2 += dd * dd;
                    }
                    if (active != 0.0) acc_dmax = fmax(acc_dmax, d2);
                    if (a.ncell > 0 && i < a.n_active) (void)cell_of(a, i, c);
                }
            }
        }
    }

    if (spent) return;
    // ---- per-block partials (plain stores; k_finalize runs after this
    // kernel, so the kernel boundary makes them visible)
    {
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
}

template <bool FC>
__global__ __launch_bounds__(kBlock) void k_fused(FusedArgs a)
{
    extern __shared__ double smem[];
    __shared__ double red[64];
    fused_tiles<FC>(a, blockIdx.x, gridDim.x, smem, red, a.partials + (size_t)blockIdx.x * PF_COUNT,
                    true);
}

// Batched: item (system, tile); the system's arguments come from the table and
// its partials are per tile.  Items are grouped by system, so the matrix is
// restaged only when the system changes.
__global__ __launch_bounds__(kBlock) void k_fused_batch(const FusedArgs *__restrict__ table,
                                                        const int2 *__restrict__ items, int n_items,
                                                        int mode)
{
    extern __shared__ double smem[];
    __shared__ double red[64];
    int prev = -1;
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        // the item is the same for the whole block: scalar loads of its arguments
        const int sys = __builtin_amdgcn_readfirstlane(items[it].x);
        const int tile = __builtin_amdgcn_readfirstlane(items[it].y);
        FusedArgs a = table[sys];
        a.mode = mode;
        // (batches hold no fixcom systems)
        fused_tiles<false>(a, tile, 1 << 30, smem, red, a.partials + (size_t)tile * PF_COUNT,
                           sys != prev);
        prev = sys;
    }
}

// --------------------------------------------------------------------------
// One block, after k_fused: combines its per-block partials (and the force
// kernel's energy partials) in block order, records the estimators and the
// running sums, advances the step counter and decides the neighbor-list
// rebuild for the coming force pass.
// --------------------------------------------------------------------------
// (The cell build at a rebuild, cells_finalize, is in pimd_device.h: the
// barostat's finalize uses it too.)

// FC: the system uses fixcom (its partials carry the centroid momentum)
template <bool FC>
__device__ void finalize_system(const FusedArgs &a, int nblocks, double *red, int *sbuf, int *sflag)
{
    const int t = threadIdx.x;
    const int P = a.P;
    const int mode = a.mode;
    Ctl *c = a.ctl;
    // the control block, thread 0's read-modify-write state and the partials
    // are read together; a spent budget is acted on once they are in
    const long long budget = c->budget;
    const unsigned long long step = c->step;
    const int synced = c->synced;
    const int ext = !a.pair;
    const bool closing = (mode == FUSED_STEP || mode == FUSED_CLOSE) && !synced && a.pair;
    const bool est_now = closing || mode == FUSED_EST;
    const bool est_after = (mode == FUSED_STEP) && ext;

    // thread 0's read-modify-write state, fetched now so that its latency
    // overlaps the partial reductions
    double run_sum[kNumEst], run_sq[kNumEst];
    unsigned long long run_count = 0, n_rebuilds = 0;
    double ebuild = 0.0;
    if (t == 0) {
#pragma unroll
        for (int q = 0; q < kNumEst; ++q) {
            run_sum[q] = c->sum[q];
            run_sq[q] = c->sumsq[q];
        }
        run_count = c->count;
        ebuild = c->ebuild;
        n_rebuilds = c->n_rebuilds;
    }

    // ekin, espring, vir, uext, pair energy, fixcom momentum (3), centroid
    // kinetic sum, cell virial
    double tot[10] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    double mx[3] = {0.0, 0.0, 0.0};   // emax^2, dmax^2, non-finite flag
    // Loads in fixed batches held in registers, so that a batch's reads are in
    // flight together; out-of-range slots add +0, and each thread's sums run
    // in loop order, so the result is that of the plain loop.
    constexpr int NB = 4, NF = 16;
    for (int b0 = t; b0 < nblocks; b0 += NB * kBlock) {
        constexpr int NQ = FC ? PF_COUNT : PF_K0 + 1;
        double pv[NB][PF_COUNT];
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int b = b0 + u * kBlock;
            const double *pp = a.partials + (size_t)(b < nblocks ? b : 0) * PF_COUNT;
#pragma unroll
            for (int q = 0; q < PF_COUNT; ++q) pv[u][q] = (q < NQ && b < nblocks) ? pp[q] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            tot[0] += pv[u][PF_EKIN];
            tot[1] += pv[u][PF_ESPRING];
            tot[2] += pv[u][PF_VIR];
            tot[3] += pv[u][PF_UEXT];
            mx[0] = fmax(mx[0], pv[u][PF_EMAX]);
            mx[1] = fmax(mx[1], pv[u][PF_DMAX]);
            mx[2] = fmax(mx[2], pv[u][PF_NONFINITE]);
            tot[5] += pv[u][PF_PX];
            tot[6] += pv[u][PF_PY];
            tot[7] += pv[u][PF_PZ];
            tot[8] += pv[u][PF_K0];
        }
    }
    // (summed whether or not this pass needs them, so the loads do not wait
    // for the control block)
    if (a.pair) {
        const double2 *fp = reinterpret_cast<const double2 *>(a.fpartials);
        for (int b0 = t; b0 < a.n_fpartials; b0 += NF * kBlock) {
            double2 fv[NF];
#pragma unroll
            for (int u = 0; u < NF; ++u) {
                const int b = b0 + u * kBlock;
                fv[u] = b < a.n_fpartials ? fp[b] : make_double2(0.0, 0.0);
            }
#pragma unroll
            for (int u = 0; u < NF; ++u) {
                tot[4] += fv[u].x;
                tot[9] += fv[u].y;
            }
        }
    }
    block_sum_max<10, 3>(tot, mx, red);
    constexpr int kRedFlag = (10 + 3) * (kBlock / 64);   // first slot past the reduction's
    static_assert(kRedFlag + 2 <= 64, "reduction scratch");
    if (mode == FUSED_STEP && budget == 0) {
        // no step was taken: nothing to combine, and no force pass follows
        if (t == 0) c->ran = 0;
        return;
    }
    const double upair = tot[4];
    const double emax = sqrt(mx[0]), dmax = sqrt(mx[1]), bad = mx[2];

    if (t == 0) {
        // fixcom: a step ended in this pass (closing half-kick, or the whole
        // step with the trap): its centroid momentum Pi = sum hm v~0 fixes the
        // velocity u = Pi / sum hm to remove from every atom's centroid mode,
        // which lowers the kinetic energy by |Pi|^2 / sum hm
        double dekin = 0.0;
        if (FC && (closing || est_after)) {
            const double px = tot[5], py = tot[6], pz = tot[7];
            c->ucom[0] = px * a.inv_hsum;
            c->ucom[1] = py * a.inv_hsum;
            c->ucom[2] = pz * a.inv_hsum;
            c->ucom_pending = 1;
            dekin = (px * px + py * py + pz * pz) * a.inv_hsum;
        } else if (FC && mode == FUSED_STEP) {
            c->ucom_pending = 0;        // the step pass removed it
        }
        if (est_now || est_after) {
            // bosons: the spring energy is V_B, the primitive estimator
            // subtracts EV_B / P, and index 5 holds the virial estimator K_VR
            // = -(1/2P) sum r . F (App. A, bosonic list)
            const double ekin = tot[0] - dekin, esp = a.boson ? a.bres[0] : tot[1], vir = tot[2];
            const double epot = a.pair ? upair : tot[3];
            double v[kNumEst];
            v[0] = ekin;
            v[1] = esp;
            v[2] = epot;
            v[3] = ekin + esp + epot;
            v[4] = a.kT15PN - (a.boson ? a.bres[1] : esp) / (double)P;
            v[5] = (a.boson ? 0.0 : a.kT15N) - vir / (2.0 * (double)P);
            v[6] = ekin * a.temp_norm;
            // pressures, with W = sum_k Tr Xi^k, the force pass's cell virial.
            // P_CV: the centroids' kinetic term (2 sum hm |v~0|^2, after the
            // fixcom removal), minus the centroid virial, plus W, over 3PV.
            // P_PR: 3PNkT - (2S - W)/P over 3V.  P_MD: 2K + W over 3V.
            const double W = tot[9], iP = 1.0 / (double)P;
            v[7] = a.lists ? (2.0 * (tot[8] - dekin) - vir + W) * iP * a.inv_3v : 0.0;
            v[8] = a.lists ? (2.0 * a.kT15PN - (2.0 * esp - W) * iP) * a.inv_3v : 0.0;
            v[9] = a.lists ? (2.0 * ekin + W) * a.inv_3v : 0.0;
            for (int q = 0; q < kNumEst; ++q) c->value[q] = v[q];
            c->est_step = est_after ? step + 1 : step;
            if (mode != FUSED_EST) {
                c->count = run_count + 1;
                for (int q = 0; q < kNumEst; ++q) {
                    c->sum[q] = run_sum[q] + v[q];
                    c->sumsq[q] = run_sq[q] + v[q] * v[q];
                }
            }
        }
        if (mode == FUSED_STEP) {
            c->step = step + 1;
            c->synced = ext ? 1 : 0;
            if (budget > 0) c->budget = budget - 1;
        } else if (mode == FUSED_CLOSE) {
            c->synced = 1;
        }
        c->ran = 1;
        const bool rebuild = a.lists && (mode == FUSED_PREP ||
                                        (mode == FUSED_STEP && dmax + emax > 0.5 * a.skin + ebuild));
        const double rlist = a.rc + a.skin + 2.0 * emax;
        if (rebuild) {
            c->rebuild = 1;
            c->ebuild = emax;
            c->rlist = rlist;
            c->n_rebuilds = n_rebuilds + 1;
        } else if (a.lists && mode == FUSED_STEP) {
            c->rebuild = 0;
        }
        if (bad != 0.0) c->nonfinite = 1;
        // this pass's decision, for the cell build below (slots past the
        // reduction's, which other threads may still be reading)
        red[kRedFlag] = rebuild ? 1.0 : 0.0;
        red[kRedFlag + 1] = rlist;
    }
    // the centroid cell lists of a rebuild (cells recorded by this pass)
    if (a.lists && a.ncell > 0 && (mode == FUSED_STEP || mode == FUSED_PREP)) {
        __syncthreads();
        const bool rb = red[kRedFlag] != 0.0;
        const double rl = red[kRedFlag + 1];
        __syncthreads();
        if (rb) cells_finalize(a, a.icw, rl, sbuf, sflag);
    }
}

template <bool FC>
__global__ __launch_bounds__(kBlock) void k_finalize(FusedArgs a, int nblocks)
{
    __shared__ double red[64];
    __shared__ __align__(16) int sbuf[4 * kMaxCells];
    __shared__ int sflag[1];
    finalize_system<FC>(a, nblocks, red, sbuf, sflag);
}

// Batched: block s finalizes system s from its per-tile partials.
__global__ __launch_bounds__(kBlock) void k_finalize_batch(const FusedArgs *table,
                                                           const int *nparts, int n_sys, int mode)
{
    __shared__ double red[64];
    __shared__ __align__(16) int sbuf[4 * kMaxCells];
    __shared__ int sflag[1];
    for (int sidx = blockIdx.x; sidx < n_sys; sidx += gridDim.x) {
        FusedArgs a = table[sidx];
        a.mode = mode;
        // (batches hold no fixcom systems)
        if (nparts[sidx] > 0) finalize_system<false>(a, nparts[sidx], red, sbuf, sflag);
        __syncthreads();
    }
}

int fused_grid(int N, int P)
{
    const int A = kBlock / P;
    const int ntiles = (N + A - 1) / A;
    int dev = 0, ncu = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess) ncu = prop.multiProcessorCount;
    }
    // large P needs more than the default 64 KB of dynamic LDS per block
    (void)hipFuncSetAttribute((const void *)k_fused<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              fused_smem_bytes(P));
    (void)hipFuncSetAttribute((const void *)k_fused<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              fused_smem_bytes(P));
    int per_cu = 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_fused<false>, kBlock, fused_smem_bytes(P)) !=
            hipSuccess || per_cu < 1)
        per_cu = 1;
    const int cap = ncu * per_cu;
    return ntiles < cap ? ntiles : cap;
}

void launch_fused(const FusedArgs &a, int grid, hipStream_t s)
{
    if (a.boson) {
        launch_boson_pass(a, grid, s);   // Cartesian beads (pimd_boson.hip)
        return;
    }
    if (a.fixcom)
        hipLaunchKernelGGL(k_fused<true>, dim3(grid), dim3(kBlock), fused_smem_bytes(a.P), s, a);
    else
        hipLaunchKernelGGL(k_fused<false>, dim3(grid), dim3(kBlock), fused_smem_bytes(a.P), s, a);
}

void launch_finalize(const FusedArgs &a, int fused_blocks, hipStream_t s)
{
    if (a.fixcom)
        hipLaunchKernelGGL(k_finalize<true>, dim3(1), dim3(kBlock), 0, s, a, fused_blocks);
    else
        hipLaunchKernelGGL(k_finalize<false>, dim3(1), dim3(kBlock), 0, s, a, fused_blocks);
}

// --------------------------------------------------------------------------
// Pair forces.  Block = A = kBlock/(S P) atoms, thread (atom, sub-group, bead).
// When the control block requests it, each atom's lanes first rebuild that
// atom's list with entries |c_i - c_j + s L| < rlist: from the centroid cells
// (the 2R+1 cells per dim around the atom's cell, in a fixed order) or, when
// the box has too few cells, by scanning every active atom's centroid and
// every periodic image within reach, in (j, image) order.
// --------------------------------------------------------------------------
__device__ __forceinline__ int pack_shift(int sx, int sy, int sz)
{
    return (sx + 512) | ((sy + 512) << 10) | ((sz + 512) << 20);
}
constexpr int kNoShift = 512 | (512 << 10) | (512 << 20);   // pack_shift(0, 0, 0)
// Word 3 of a raw buffer resource on gfx9-family parts (data format 32,
// no swizzle, no index stride): offsets are plain byte offsets.
constexpr int kBufferRsrcWord3 = 0x00020000;
__device__ __forceinline__ void unpack_shift(int p, double &sx, double &sy, double &sz)
{
    sx = (double)((p & 1023) - 512);
    sy = (double)(((p >> 10) & 1023) - 512);
    sz = (double)(((p >> 20) & 1023) - 512);
}

// Blocks are dispatched round-robin over the 8 XCDs; map them so that each
// XCD gets a contiguous range of tiles (neighboring atoms, hence a shared
// neighborhood in that XCD's L2).  A bijection on [0, gridDim.x).
__device__ __forceinline__ int xcd_tile(int b, int nb)
{
    constexpr int kXcd = 8;
    const int q = nb / kXcd, r = nb % kXcd;
    const int xcd = b % kXcd, idx = b / kXcd;
    return (xcd < r) ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
}

// Half of each ordered pair's energy 4 eps (sr12 - sr6) - ushift and of its
// cell virial r . F = 24 eps (2 sr12 - sr6), from the thread's sums.
__device__ __forceinline__ void lj_energy_virial(double s12, double s6, int np, double eps4,
                                                 double eps24, double ushift, double &e, double &w)
{
    e += 0.5 * (eps4 * (s12 - s6) - ushift * (double)np);
    w += 0.5 * eps24 * (2.0 * s12 - s6);
}

// DIAG: also the pair's r_a F_a per dimension into wd (the diagonal of the
// cell virial, for the anisotropic barostat)
template <bool DIAG = false>
__device__ __forceinline__ void lj_accumulate(double dx, double dy, double dz, double rc2,
                                              double sig2, double eps24,
                                              double &fx, double &fy, double &fz,
                                              double &s12, double &s6, int &np,
                                              double *wd = nullptr)
{
    const double r2 = dx * dx + dy * dy + dz * dz;
    if (r2 < rc2) {
        // 1/r2: the hardware reciprocal (about 2^-24 relative) refined by one
        // Newton step, instead of the IEEE division sequence.  Measured over
        // 4e6 values in [0.5, 4096): at most 11 ulp from the correctly
        // rounded 1/r2 (a second step makes it exact there); the pair force,
        // a polynomial in 1/r2 of degree 7, then carries ~1e-14 relative,
        // far inside the FP64 parity bar.
        double ir2 = __builtin_amdgcn_rcp(r2);
        ir2 = fma(fma(-r2, ir2, 1.0), ir2, ir2);
        const double sr2 = sig2 * ir2;
        const double sr6 = sr2 * sr2 * sr2, sr12 = sr6 * sr6;
        const double fr = eps24 * (2.0 * sr12 - sr6) * ir2;
        // the pair energy and virial are linear in (sr12, sr6, 1): their sums
        // are formed once per thread (lj_energy_virial)
        s12 += sr12; s6 += sr6; ++np;
        fx += fr * dx; fy += fr * dy; fz += fr * dz;
        if constexpr (DIAG) {
            wd[0] += fr * dx * dx; wd[1] += fr * dy * dy; wd[2] += fr * dz * dz;
        }
    }
}

// Harmonic bonds of atom i at bead k (minimum image), added to its force and
// to the thread's energy and virial sums.  A partner flagged kBondOwned has
// no lane of its own (an atom outside the LJ whose only bond is this one): its
// force is minus this bond's force, written here, and the whole bond's energy
// and virial are counted here (otherwise each side counts half).  The
// partner's force is the exact negative of what its own lanes would compute,
// since the minimum-image difference is antisymmetric.
template <bool DIAG = false>
__device__ __forceinline__ void bond_forces(const PairArgs &a, int i, int k, double xi, double yi,
                                            double zi, double L0, double L1, double L2,
                                            double &fx, double &fy, double &fz, double &e,
                                            double &wv, double *wd = nullptr)
{
    const int P = a.P, P3 = 3 * P;
    const double *__restrict__ X = a.x;
    for (int bb = 0; bb < kMaxBonds; ++bb) {
        const int jr = a.bond_j[i * kMaxBonds + bb];
        if (jr < 0) break;
        const bool owned = (jr & kBondOwned) != 0;
        const int j = jr & ~kBondOwned;
        const size_t jb = (size_t)j * P3 + k;
        double dx = xi - X[jb], dy = yi - X[jb + P], dz = zi - X[jb + 2 * P];
        dx -= L0 * rint(dx / L0);
        dy -= L1 * rint(dy / L1);
        dz -= L2 * rint(dz / L2);
        const double r = sqrt(dx * dx + dy * dy + dz * dz);
        const double dr = r - a.bond_r0;
        const double fr = -2.0 * a.bond_k * dr / r;
        const double share = owned ? 1.0 : 0.5;   // each bond is seen from both atoms
        e += share * a.bond_k * dr * dr;
        wv += share * fr * r * r;
        fx += fr * dx; fy += fr * dy; fz += fr * dz;
        if constexpr (DIAG) {
            wd[0] += share * fr * dx * dx; wd[1] += share * fr * dy * dy; wd[2] += share * fr * dz * dz;
        }
        if (owned) {
            a.f[jb] = -(fr * dx);
            a.f[jb + P] = -(fr * dy);
            a.f[jb + 2 * P] = -(fr * dz);
        }
    }
}

// Thread = (atom, sub-group s, bead k).  The S sub-groups of an atom share
// its neighbor list (entry q goes to sub-group q mod S) and their partial
// forces are combined in sub-group order through shared memory; S > 1 only
// when the system alone would leave the GPU with few waves to hide latency.
// BOXDEV: the box lengths come from the control block (a barostat moves them)
// DIAG: the block also writes the diagonal of its cell virial (a.fdiag)
// PAIRED (even P, pair_lanes_paired): in the force loop each lane takes two
// consecutive beads of 2S sub-groups of P/2 lanes, so every gather is a
// 16-byte load: half the load instructions of one bead per lane, which is
// what the loop's gathers are limited by when the rows come from L2.
template <bool BOXDEV = false, bool DIAG = false, bool PAIRED = false>
__device__ void pair_tile(const PairArgs &a, int tile, int *s_cnt, double *red, double *s_f)
{
    const int P = a.P, S = a.S;
    const int G = S * P;                    // lanes per atom
    const int A = kBlock / G;               // atoms per block
    const int t = threadIdx.x;
    const int la = t / G, g = t - la * G;   // atom slot, lane within the atom's group
    const int sg = g / P, k = g - sg * P;   // sub-group, bead
    const int i = tile * A + la;
    const bool act = (la < A) && (i < a.n_forced);
    const double L0 = BOXDEV ? a.ctl->box[0] : a.box[0];
    const double L1 = BOXDEV ? a.ctl->box[1] : a.box[1];
    const double L2 = BOXDEV ? a.ctl->box[2] : a.box[2];
    if (!a.ctl->ran) return;   // the system took no step (uniform per block)

    // A list cutoff that is not finite (non-finite positions) or that would
    // need more than kMaxImages periodic images per dim skips the build and
    // flags the state; the image loops below are therefore always bounded.
    constexpr int kMaxImages = 8;
    const double rl_in = a.ctl->rlist;
    const bool rl_ok = isfinite(rl_in) && rl_in > 0.0 && rl_in <= kMaxImages * L0 &&
                       rl_in <= kMaxImages * L1 && rl_in <= kMaxImages * L2;
    if (a.ctl->rebuild && !rl_ok) {
        if (tile == 0 && t == 0) a.ctl->nonfinite = 1;
    }
    // Lists from the sorted centroid cells: the first min(G, 64) lanes of each
    // atom's group (they lie in one wave) scan the 2R+1 cells per dim around
    // the atom's cell, cells and their atoms in a fixed order; wave ballots
    // place the hits.  Image shifts come from the integer box indices kept at
    // binning and the wrap of the stencil cell.
    const bool wave_aligned = (G % 64 == 0) || (64 % G == 0);
    const bool use_cells = a.ctl->rebuild && rl_ok && a.ctl->cell_ok && wave_aligned;
    if (use_cells) {
        const double rl2 = rl_in * rl_in;
        const int Gb = G < 64 ? G : 64;
        const int lane = t & 63;
        const int gbase = lane - g;
        const unsigned long long gmask = (Gb == 64) ? ~0ull : (((1ull << Gb) - 1ull) << gbase);
        const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
        int total = 0;
        const bool builder = act && i < a.n_active && g < Gb;
        if (builder) {
            const int4 ii = a.cinfo[i];
            const int nx = a.nc[0], ny = a.nc[1], nz = a.nc[2], ccap = a.cell_cap;
            const int cx = ii.x % nx, cy = (ii.x / nx) % ny, cz = ii.x / (nx * ny);
            const int R0 = a.ctl->cell_R[0], R1 = a.ctl->cell_R[1], R2 = a.ctl->cell_R[2];
            const int sx_n = 2 * R0 + 1, sy_n = 2 * R1 + 1;
            const int NS = sx_n * sy_n * (2 * R2 + 1);
            const double ci0 = a.cent[i * 3], ci1 = a.cent[i * 3 + 1], ci2 = a.cent[i * 3 + 2];
            int2 *mylist = a.nbr + (size_t)i * a.cap;
            // stencil cell s (fixed order, x fastest) and the image it wraps to
            auto stencil = [&](int s, int &kx, int &ky, int &kz) {
                const int ox = s % sx_n - R0, oy = (s / sx_n) % sy_n - R1, oz = s / (sx_n * sy_n) - R2;
                int qx = cx + ox, qy = cy + oy, qz = cz + oz;
                kx = qx < 0 ? -1 : (qx >= nx ? 1 : 0);
                ky = qy < 0 ? -1 : (qy >= ny ? 1 : 0);
                kz = qz < 0 ? -1 : (qz >= nz ? 1 : 0);
                qx -= kx * nx; qy -= ky * ny; qz -= kz * nz;
                return (qz * ny + qy) * nx + qx;
            };
            auto entry = [&](int cell, int q) {
                CellEntry e = {{0.0, 0.0, 0.0}, -1, {0, 0, 0}, 0};
                if (q < ccap) e = a.cell_ent[(size_t)cell * ccap + q];
                return e;
            };
            auto test = [&](const CellEntry &e, bool in, int kx, int ky, int kz) {
                const int j = e.j;
                const int sx = e.nb[0] - ii.y - kx, sy = e.nb[1] - ii.z - ky, sz = e.nb[2] - ii.w - kz;
                const double ex = ci0 - e.c[0] + sx * L0;
                const double ey = ci1 - e.c[1] + sy * L1;
                const double ez = ci2 - e.c[2] + sz * L2;
                const bool pass = in && (j != i) && (ex * ex + ey * ey + ez * ez < rl2);
                const unsigned long long hit = __ballot(pass) & gmask;
                if (pass) {
                    const int w = total + __popcll(hit & below);
                    if (w < a.cap) mylist[w] = make_int2(j * 3 * P, pack_shift(sx, sy, sz));
                }
                total += __popcll(hit);
            };
            // one cell ahead: the next cell's count and first entries are in
            // flight while the current one is tested
            int kx, ky, kz;
            int cell = stencil(0, kx, ky, kz);
            int n = a.cell_scnt[cell];
            CellEntry e = entry(cell, g);
            for (int s = 0; s < NS; ++s) {
                const int ccell = cell, cn = n, ckx = kx, cky = ky, ckz = kz;
                const CellEntry ce = e;
                if (s + 1 < NS) {
                    cell = stencil(s + 1, kx, ky, kz);
                    n = a.cell_scnt[cell];
                    e = entry(cell, g);
                }
                test(ce, g < cn, ckx, cky, ckz);
                for (int q0 = Gb; q0 < cn; q0 += Gb)
                    test(entry(ccell, q0 + g), q0 + g < cn, ckx, cky, ckz);
            }
        }
        if (act && g == 0) {
            if (i < a.n_active) {
                if (total > a.cap) {
                    a.ctl->overflow = 1;
                    total = a.cap;
                }
                a.nbr_count[i] = total;
            } else {
                a.nbr_count[i] = 0;
            }
            a.cref[i * 3] = a.cent[i * 3];
            a.cref[i * 3 + 1] = a.cent[i * 3 + 1];
            a.cref[i * 3 + 2] = a.cent[i * 3 + 2];
        }
        __threadfence_block();
        __syncthreads();
    }
    if (a.ctl->rebuild && rl_ok && !use_cells) {
        const double rl = rl_in;
        const double rl2 = rl * rl;
        const bool big = (L0 >= 2.0 * rl) && (L1 >= 2.0 * rl) && (L2 >= 2.0 * rl);
        const int R0 = big ? 0 : min((int)ceil(rl / L0), kMaxImages),
                  R1 = big ? 0 : min((int)ceil(rl / L1), kMaxImages),
                  R2 = big ? 0 : min((int)ceil(rl / L2), kMaxImages);
        const bool builder = act && i < a.n_active;
        double ci[3] = {0.0, 0.0, 0.0};
        if (builder) {
            ci[0] = a.cent[i * 3]; ci[1] = a.cent[i * 3 + 1]; ci[2] = a.cent[i * 3 + 2];
        }
        int total = 0;
        int2 *mylist = a.nbr + (size_t)(builder ? i : 0) * a.cap;
        for (int j0 = 0; j0 < a.n_active; j0 += G) {
            const int j = j0 + g;
            int cnt = 0;
            double dx = 0, dy = 0, dz = 0;
            int bx = 0, by = 0, bz = 0;
            const bool cand = builder && j < a.n_active;
            if (cand) {
                dx = ci[0] - a.cent[j * 3];
                dy = ci[1] - a.cent[j * 3 + 1];
                dz = ci[2] - a.cent[j * 3 + 2];
                bx = -(int)rint(dx / L0);
                by = -(int)rint(dy / L1);
                bz = -(int)rint(dz / L2);
                for (int ox = -R0; ox <= R0; ++ox)
                    for (int oy = -R1; oy <= R1; ++oy)
                        for (int oz = -R2; oz <= R2; ++oz) {
                            const int sx = bx + ox, sy = by + oy, sz = bz + oz;
                            if (j == i && sx == 0 && sy == 0 && sz == 0) continue;
                            const double ex = dx + sx * L0, ey = dy + sy * L1, ez = dz + sz * L2;
                            if (ex * ex + ey * ey + ez * ez < rl2) ++cnt;
                        }
            }
            s_cnt[t] = cnt;
            __syncthreads();
            int off = 0, chunk = 0;
            if (la < A) {
                for (int q = 0; q < G; ++q) {
                    const int c = s_cnt[la * G + q];
                    if (q < g) off += c;
                    chunk += c;
                }
            }
            if (cand && cnt > 0) {
                int w = total + off;
                for (int ox = -R0; ox <= R0; ++ox)
                    for (int oy = -R1; oy <= R1; ++oy)
                        for (int oz = -R2; oz <= R2; ++oz) {
                            const int sx = bx + ox, sy = by + oy, sz = bz + oz;
                            if (j == i && sx == 0 && sy == 0 && sz == 0) continue;
                            const double ex = dx + sx * L0, ey = dy + sy * L1, ez = dz + sz * L2;
                            if (ex * ex + ey * ey + ez * ez < rl2) {
                                if (w < a.cap) mylist[w] = make_int2(j * 3 * P, pack_shift(sx, sy, sz));
                                ++w;
                            }
                        }
            }
            total += chunk;
            __syncthreads();
        }
        if (act && g == 0) {
            if (i < a.n_active) {
                if (total > a.cap) {
                    a.ctl->overflow = 1;
                    total = a.cap;
                }
                a.nbr_count[i] = total;
            } else {
                a.nbr_count[i] = 0;
            }
            a.cref[i * 3] = a.cent[i * 3];
            a.cref[i * 3 + 1] = a.cent[i * 3 + 1];
            a.cref[i * 3 + 2] = a.cent[i * 3 + 2];
        }
        __threadfence_block();
        __syncthreads();
    }

    double e = 0.0, wv = 0.0, s12 = 0.0, s6 = 0.0;
    double wd[3] = {0.0, 0.0, 0.0};   // DIAG: sum of fr r_a^2 over the thread's pairs
    int np = 0;
    double fx = 0.0, fy = 0.0, fz = 0.0;
    const int P3 = 3 * P;
    const size_t ib = (size_t)i * P3 + k;
    const double *__restrict__ X = a.x;
    double xi = 0.0, yi = 0.0, zi = 0.0;
    const int cnt = (act && i < a.n_active) ? a.nbr_count[i] : 0;
    // PAIRED: lane = (atom, sub-group sg2 of 2S, bead pair kp) takes beads
    // 2 kp and 2 kp + 1 of every 2S-th entry of the atom's list
    const int P2 = P / 2, S2 = 2 * S;
    const int sg2 = PAIRED ? g / P2 : 0, kp = PAIRED ? g - sg2 * P2 : 0;
    double pxi[2] = {0.0, 0.0}, pyi[2] = {0.0, 0.0}, pzi[2] = {0.0, 0.0};
    double pf[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (act) {
        if constexpr (PAIRED) {
            const size_t pb = (size_t)i * P3 + 2 * kp;
#pragma unroll
            for (int b2 = 0; b2 < 2; ++b2) {
                pxi[b2] = X[pb + b2]; pyi[b2] = X[pb + P + b2]; pzi[b2] = X[pb + 2 * P + b2];
            }
        } else {
            xi = X[ib]; yi = X[ib + P]; zi = X[ib + 2 * P];
        }
    }
    // The block's list entries pass through LDS, up to C = kPairStage/A per
    // atom at a time, in one coalesced copy: the loop then waits only on the
    // bead-row gathers.  Entry q still goes to sub-group q mod S (q mod 2S
    // with bead pairs), in order.
    __shared__ int2 s_lst[kPairStage];
    if (g == 0) s_cnt[la] = cnt;
    __syncthreads();
    int nmax = 0;
    for (int u = 0; u < A; ++u) nmax = max(nmax, s_cnt[u]);
    const int C = kPairStage / A;
    const double eps4 = 4.0 * a.lj_eps, eps24 = 24.0 * a.lj_eps;
    const double rc2 = a.rc2, sig2 = a.lj_sig2, ush = a.lj_ushift;
    const long long x_bytes = (long long)a.N * 3 * P * 8;
    for (int c0 = 0; c0 < nmax; c0 += C) {
        const int span = min(C, nmax - c0);
        for (int e2 = t; e2 < A * span; e2 += kBlock) {
            const int aa = e2 / span, qq = c0 + (e2 - aa * span);
            if (qq < s_cnt[aa]) s_lst[e2] = a.nbr[(size_t)(tile * A + aa) * a.cap + qq];
        }
        __syncthreads();
        const int2 *ls = s_lst + la * span;                 // entry q at ls[q - c0]
        const int qend = min(cnt, c0 + span);
        int q = c0 + sg;
        if constexpr (PAIRED) {
            typedef double dbl2 __attribute__((ext_vector_type(2)));
            // the buffer's range is the position array (pair_lanes_paired
            // keeps it under 2 GiB)
            const __amdgpu_buffer_rsrc_t xr =
                __builtin_amdgcn_make_buffer_rsrc((void *)X, (short)0, (int)x_bytes, kBufferRsrcWord3);
            // (the lane's bead offset in the vector offset, the dim's row
            // offset in the scalar one)
            const unsigned kx = (unsigned)(2 * kp) * 8u;
            const int ry = __builtin_amdgcn_readfirstlane(P * 8), rz = 2 * ry;
            // (the image shift costs vector work only where it is not zero)
            auto pair2 = [&](const int2 en, const dbl2 xj, const dbl2 yj, const dbl2 zj) {
                double dx[2], dy[2], dz[2];
#pragma unroll
                for (int b2 = 0; b2 < 2; ++b2) {
                    dx[b2] = pxi[b2] - xj[b2]; dy[b2] = pyi[b2] - yj[b2]; dz[b2] = pzi[b2] - zj[b2];
                }
                if (en.y != kNoShift) {
                    double sx, sy, sz;
                    unpack_shift(en.y, sx, sy, sz);
#pragma unroll
                    for (int b2 = 0; b2 < 2; ++b2) {
                        dx[b2] += sx * L0; dy[b2] += sy * L1; dz[b2] += sz * L2;
                    }
                }
#pragma unroll
                for (int b2 = 0; b2 < 2; ++b2)
                    lj_accumulate<DIAG>(dx[b2], dy[b2], dz[b2], rc2, sig2, eps24, pf[3 * b2],
                                        pf[3 * b2 + 1], pf[3 * b2 + 2], s12, s6, np, wd);
            };
            auto rows = [&](const int2 en, dbl2 &xj, dbl2 &yj, dbl2 &zj) {
                const unsigned vo = (unsigned)en.x * 8u + kx;
                xj = __builtin_bit_cast(dbl2, __builtin_amdgcn_raw_buffer_load_b128(xr, vo, 0, 0));
                yj = __builtin_bit_cast(dbl2, __builtin_amdgcn_raw_buffer_load_b128(xr, vo, ry, 0));
                zj = __builtin_bit_cast(dbl2, __builtin_amdgcn_raw_buffer_load_b128(xr, vo, rz, 0));
            };
            // two entries per iteration: all six gathers issued before any use
            for (q = c0 + sg2; q + S2 < qend; q += 2 * S2) {
                const int2 en0 = ls[q - c0], en1 = ls[q + S2 - c0];
                dbl2 xj0, yj0, zj0, xj1, yj1, zj1;
                rows(en0, xj0, yj0, zj0);
                rows(en1, xj1, yj1, zj1);
                pair2(en0, xj0, yj0, zj0);
                pair2(en1, xj1, yj1, zj1);
            }
            if (q < qend) {
                const int2 en = ls[q - c0];
                dbl2 xj, yj, zj;
                rows(en, xj, yj, zj);
                pair2(en, xj, yj, zj);
            }
        }
        // four entries per iteration: all gathers issued before any use
        if (!PAIRED) for (; q + 3 * S < qend; q += 4 * S) {
            int2 en[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) en[u] = ls[q - c0 + u * S];
            double xj[4], yj[4], zj[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int jb = en[u].x + k;
                xj[u] = X[jb]; yj[u] = X[jb + P]; zj[u] = X[jb + 2 * P];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                double sx, sy, sz;
                unpack_shift(en[u].y, sx, sy, sz);
                lj_accumulate<DIAG>(xi - xj[u] + sx * L0, yi - yj[u] + sy * L1, zi - zj[u] + sz * L2,
                                    rc2, sig2, eps24, fx, fy, fz, s12, s6, np, wd);
            }
        }
        if (!PAIRED) for (; q < qend; q += S) {
            const int2 en = ls[q - c0];
            double sx, sy, sz;
            unpack_shift(en.y, sx, sy, sz);
            const int jb = en.x + k;
            lj_accumulate<DIAG>(xi - X[jb] + sx * L0, yi - X[jb + P] + sy * L1,
                                zi - X[jb + 2 * P] + sz * L2, rc2, sig2, eps24, fx, fy, fz, s12, s6,
                                np, wd);
        }
        __syncthreads();
    }
    if constexpr (PAIRED) {
        // back to one bead per lane: the sub-group 0 lanes sum the 2S
        // sub-groups' forces of their bead in sub-group order (the staged
        // entries are no longer needed, so their LDS holds the partials:
        // A * 2S * 3P = 6 kBlock doubles)
        double *s2 = reinterpret_cast<double *>(s_lst);
        if (la < A) {
#pragma unroll
            for (int b2 = 0; b2 < 2; ++b2)
#pragma unroll
                for (int d = 0; d < 3; ++d) s2[((la * S2 + sg2) * 3 + d) * P + 2 * kp + b2] = pf[3 * b2 + d];
        }
        __syncthreads();
        if (act && sg == 0) {
            for (int u = 0; u < S2; ++u) {
                fx += s2[((la * S2 + u) * 3 + 0) * P + k];
                fy += s2[((la * S2 + u) * 3 + 1) * P + k];
                fz += s2[((la * S2 + u) * 3 + 2) * P + k];
            }
            xi = X[ib]; yi = X[ib + P]; zi = X[ib + 2 * P];
        }
    }
    lj_energy_virial(s12, s6, np, eps4, eps24, ush, e, wv);
#pragma unroll
    for (int d = 0; d < 3; ++d) wd[d] *= 0.5;   // half of each ordered pair, as the trace
    if (act && sg == 0) bond_forces<DIAG>(a, i, k, xi, yi, zi, L0, L1, L2, fx, fy, fz, e, wv, wd);
    if (!PAIRED && S > 1) {
        s_f[t * 3] = fx; s_f[t * 3 + 1] = fy; s_f[t * 3 + 2] = fz;
        __syncthreads();
        if (act && sg == 0) {
            for (int u = 1; u < S; ++u) {
                const int o = (la * G + u * P + k) * 3;
                fx += s_f[o]; fy += s_f[o + 1]; fz += s_f[o + 2];
            }
        }
    }
    if (act && sg == 0) {
        a.f[ib] = fx; a.f[ib + P] = fy; a.f[ib + 2 * P] = fz;
    }
    // block sums (fixed order): energy, then the cell virial after all partials
    if constexpr (DIAG) {
        double e5[5] = {e, wv, wd[0], wd[1], wd[2]};
        block_sum<5>(e5, red);
        if (t == 0) {
            reinterpret_cast<double2 *>(a.fpartials)[tile] = make_double2(e5[0], e5[1]);
            a.fdiag[(size_t)tile * 3] = e5[2];
            a.fdiag[(size_t)tile * 3 + 1] = e5[3];
            a.fdiag[(size_t)tile * 3 + 2] = e5[4];
        }
    } else {
        double e1[2] = {e, wv};
        block_sum<2>(e1, red);
        if (t == 0) reinterpret_cast<double2 *>(a.fpartials)[tile] = make_double2(e1[0], e1[1]);
    }
}

// --------------------------------------------------------------------------
// Cluster-pair force pass.  Block b takes the A = kBlock/P consecutive
// atoms b*A ... (thread = atom, bead); its LJ-active atoms share one neighbor
// list (the union of their lists) with, per entry, a mask of the atoms that
// use it, built at list rebuilds in index order.  Each neighbor's P bead rows
// are staged in LDS once per block (double-buffered chunks) and read by every
// atom of the block that has it as a neighbor, instead of one gather per atom.
// Every pair of the block is taken in one frame: atom q's centroid is moved by
// whole boxes u_q next to atom 0's, and each entry carries the image of j
// nearest to atom 0.  That image is the pair's minimum image whenever
// r_list + (cluster radius) < L/2, which the build checks; a block where it
// fails (or whose list would overflow its LDS) uses the per-atom lists.
// --------------------------------------------------------------------------

__device__ void cluster_tile(const PairArgs &a, int b, double *smem, int *s_cnt, double *red,
                             double *s_f)
{
    const int P = a.P, A = kBlock / P, P3 = 3 * P;
    const int t = threadIdx.x;
    const int la = t / P, k = t - la * P;
    const int i0 = b * A;
    const int i = i0 + la;
    const bool act = (la < A) && (i < a.n_forced);
    const int na = min(A, a.n_active - i0);             // LJ-active atoms of the block (> 0)
    const bool lj = act && la < na;
    const double L0 = a.box[0], L1 = a.box[1], L2 = a.box[2];
    if (!a.ctl->ran) return;

    // per-atom fallback, decided at the last rebuild (uniform per block)
    PairArgs a1 = a;
    a1.S = 1;
    const bool rebuild = a.ctl->rebuild != 0;
    double *sCp = smem;                                   // [A][3] frame centroids
    int4 *sEnt = reinterpret_cast<int4 *>(smem + 2 * kClusterRows);
    if (rebuild) {
        const double rl = a.ctl->rlist;
        const double rl2 = rl * rl;
        // frame: centroids of the block's active atoms moved next to atom 0's
        if (t < na) {
            const double c0x = a.cent[i0 * 3], c0y = a.cent[i0 * 3 + 1], c0z = a.cent[i0 * 3 + 2];
            const double cx = a.cent[(i0 + t) * 3], cy = a.cent[(i0 + t) * 3 + 1],
                         cz = a.cent[(i0 + t) * 3 + 2];
            const double ux = -rint((cx - c0x) / L0), uy = -rint((cy - c0y) / L1),
                         uz = -rint((cz - c0z) / L2);
            sCp[t * 3] = cx + ux * L0;
            sCp[t * 3 + 1] = cy + uy * L1;
            sCp[t * 3 + 2] = cz + uz * L2;
            const bool uok = fabs(ux) < 500.0 && fabs(uy) < 500.0 && fabs(uz) < 500.0;
            a.cframe[i0 + t] = uok ? pack_shift((int)ux, (int)uy, (int)uz) : pack_shift(0, 0, 0);
            s_cnt[t] = uok ? 0 : 1;
        }
        __syncthreads();
        int ok = 1;
        {
            double r2max = 0.0;
            for (int q = 0; q < na; ++q) {
                const double dx = sCp[q * 3] - sCp[0], dy = sCp[q * 3 + 1] - sCp[1],
                             dz = sCp[q * 3 + 2] - sCp[2];
                r2max = fmax(r2max, dx * dx + dy * dy + dz * dz);
                if (s_cnt[q]) ok = 0;
            }
            const double lmin = fmin(L0, fmin(L1, L2));
            if (!(isfinite(rl) && rl > 0.0 && rl + sqrt(r2max) < 0.5 * lmin)) ok = 0;
        }
        __syncthreads();
        int total = 0;
        if (ok) {
            int4 *cl = a.clist + (size_t)b * a.ccap;
            const double c0x = sCp[0], c0y = sCp[1], c0z = sCp[2];
            const int w = t >> 6, lane = t & 63;
            const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
            for (int j0 = 0; j0 < a.n_active; j0 += kBlock) {
                const int j = j0 + t;
                int mask = 0, sx = 0, sy = 0, sz = 0;
                if (j < a.n_active) {
                    const double cx = a.cent[j * 3], cy = a.cent[j * 3 + 1], cz = a.cent[j * 3 + 2];
                    const double fx = -rint((c0x - cx) / L0), fy = -rint((c0y - cy) / L1),
                                 fz = -rint((c0z - cz) / L2);
                    if (fabs(fx) < 500.0 && fabs(fy) < 500.0 && fabs(fz) < 500.0) {
                        sx = (int)fx; sy = (int)fy; sz = (int)fz;
                        const double jx = cx - sx * L0, jy = cy - sy * L1, jz = cz - sz * L2;
                        for (int q = 0; q < na; ++q) {
                            if (j == i0 + q) continue;
                            const double ex = sCp[q * 3] - jx, ey = sCp[q * 3 + 1] - jy,
                                         ez = sCp[q * 3 + 2] - jz;
                            if (ex * ex + ey * ey + ez * ez < rl2) mask |= 1 << q;
                        }
                    }
                }
                // place the hits in index order: wave ballots, then wave offsets
                const unsigned long long hit = __ballot(mask != 0);
                if (lane == 0) s_cnt[w] = __popcll(hit);
                __syncthreads();
                int off = total;
                for (int u = 0; u < w; ++u) off += s_cnt[u];
                int chunk = 0;
                for (int u = 0; u < kBlock / 64; ++u) chunk += s_cnt[u];
                if (mask != 0) {
                    const int wpos = off + __popcll(hit & below);
                    if (wpos < a.ccap) cl[wpos] = make_int4(j * P3, pack_shift(sx, sy, sz), mask, 0);
                }
                total += chunk;
                __syncthreads();
            }
            if (total > a.ccap || total > kClusterMax) ok = 0;
        }
        if (t == 0) {
            a.cmode[b] = ok ? 0 : 1;
            a.ccount[b] = ok ? total : 0;
        }
        if (ok && act) {
            a.cref[i * 3] = a.cent[i * 3];
            a.cref[i * 3 + 1] = a.cent[i * 3 + 1];
            a.cref[i * 3 + 2] = a.cent[i * 3 + 2];
        }
        if (!ok) {
            // the per-atom path of this block rebuilds its own lists
            __syncthreads();
            pair_tile(a1, b, s_cnt, red, s_f);
            return;
        }
        __threadfence_block();
        __syncthreads();
    } else if (a.cmode[b] != 0) {
        pair_tile(a1, b, s_cnt, red, s_f);
        return;
    }

    // ---- forces
    const double *__restrict__ X = a.x;
    const int n = a.ccount[b];
    for (int q = t; q < n; q += kBlock) sEnt[q] = a.clist[(size_t)b * a.ccap + q];
    double xi = 0.0, yi = 0.0, zi = 0.0;
    const size_t ib = (size_t)i * P3 + k;
    if (act) {
        xi = X[ib]; yi = X[ib + P]; zi = X[ib + 2 * P];
    }
    double xf = xi, yf = yi, zf = zi;                    // in the cluster's frame
    if (lj) {
        double ux, uy, uz;
        unpack_shift(a.cframe[i], ux, uy, uz);
        xf += ux * L0; yf += uy * L1; zf += uz * L2;
    }
    const double eps4 = 4.0 * a.lj_eps, eps24 = 24.0 * a.lj_eps;
    const double rc2 = a.rc2, sig2 = a.lj_sig2, ush = a.lj_ushift;
    double e = 0.0, wv = 0.0, fx = 0.0, fy = 0.0, fz = 0.0, s12 = 0.0, s6 = 0.0;
    int np = 0;
    const int CH = kClusterRows / P3;                    // rows per chunk
    const int nch = (n + CH - 1) / CH;
    constexpr int NR = kClusterRows / kBlock;             // staged doubles per thread
    double rr[NR];
    __syncthreads();                                      // the entries are in LDS
    auto fetch = [&](int c) {
#pragma unroll
        for (int v = 0; v < NR; ++v) {
            const int q = t + v * kBlock;
            const int u = q / P3, r = q - u * P3;
            const int e_ = c * CH + u;
            rr[v] = (u < CH && e_ < n) ? X[sEnt[e_].x + r] : 0.0;
        }
    };
    auto stage = [&](int c) {
        double *buf = smem + (c & 1) * kClusterRows;
#pragma unroll
        for (int v = 0; v < NR; ++v) buf[t + v * kBlock] = rr[v];
    };
    if (nch > 0) {
        fetch(0);
        stage(0);
    }
    __syncthreads();
    for (int c = 0; c < nch; ++c) {
        if (c + 1 < nch) fetch(c + 1);
        const double *buf = smem + (c & 1) * kClusterRows;
        const int nu = min(CH, n - c * CH);
        if (lj) {
            for (int u = 0; u < nu; ++u) {
                const int4 en = sEnt[c * CH + u];
                if ((en.z >> la) & 1) {
                    const double *row = buf + u * P3;
                    double sx, sy, sz;
                    unpack_shift(en.y, sx, sy, sz);
                    lj_accumulate(xf - row[k] + sx * L0, yf - row[P + k] + sy * L1,
                                  zf - row[2 * P + k] + sz * L2, rc2, sig2, eps24,
                                  fx, fy, fz, s12, s6, np);
                }
            }
        }
        if (c + 1 < nch) stage(c + 1);
        __syncthreads();
    }
    lj_energy_virial(s12, s6, np, eps4, eps24, ush, e, wv);
    if (act) {
        bond_forces(a, i, k, xi, yi, zi, L0, L1, L2, fx, fy, fz, e, wv);
        a.f[ib] = fx; a.f[ib + P] = fy; a.f[ib + 2 * P] = fz;
    }
    double e1[2] = {e, wv};
    block_sum<2>(e1, red);
    if (t == 0) reinterpret_cast<double2 *>(a.fpartials)[b] = make_double2(e1[0], e1[1]);
}

template <bool PAIRED>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(PAIRED ? 5 : 6))) void k_pair(PairArgs a)
{
    __shared__ int s_cnt[kBlock];
    __shared__ double red[64];
    __shared__ double s_f[kBlock * 3];
    // Tiles holding LJ-active atoms come first.  Each of the two tile ranges
    // is laid out contiguously per XCD, so both are spread over all XCDs.
    const int b = blockIdx.x, nA = a.n_active_tiles;
    const int tile = (b < nA) ? xcd_tile(b, nA) : nA + xcd_tile(b - nA, gridDim.x - nA);
    pair_tile<false, false, PAIRED>(a, tile, s_cnt, red, s_f);
}
// The same pass with the active tiles on cluster lists (a kernel of its own,
// so that the per-atom kernel keeps its register budget).
__global__ __launch_bounds__(kBlock) void k_pair_clusters(PairArgs a)
{
    __shared__ int s_cnt[kBlock];
    __shared__ double red[64];
    __shared__ double s_f[kBlock * 3];
    extern __shared__ double s_dyn[];
    const int b = blockIdx.x, nA = a.n_active_tiles;
    const int tile = (b < nA) ? xcd_tile(b, nA) : nA + xcd_tile(b - nA, gridDim.x - nA);
    if (tile < a.n_clusters)
        cluster_tile(a, tile, s_dyn, s_cnt, red, s_f);
    else
        pair_tile(a, tile, s_cnt, red, s_f);
}

// Batched: one (system, tile) item per block (grid = item count).  Per-atom
// lists only, so that the kernel keeps the per-atom kernel's register budget;
// the systems with paired lanes and the others are two item lists.
template <bool PAIRED>
__global__ __launch_bounds__(kBlock) void k_pair_batch(const PairArgs *__restrict__ table,
                                                       const int2 *__restrict__ items, int n_items)
{
    __shared__ int s_cnt[kBlock];
    __shared__ double red[64];
    __shared__ double s_f[kBlock * 3];
    if ((int)blockIdx.x >= n_items) return;
    // the item is the same for the whole block: scalar loads of its arguments
    const int sys = __builtin_amdgcn_readfirstlane(items[blockIdx.x].x);
    const int tile = __builtin_amdgcn_readfirstlane(items[blockIdx.x].y);
    const PairArgs a = table[sys];
    pair_tile<false, false, PAIRED>(a, tile, s_cnt, red, s_f);
}

// The same with cluster lists for the systems that use them.
__global__ __launch_bounds__(kBlock) void k_pair_batch_clusters(const PairArgs *table,
                                                                const int2 *items, int n_items)
{
    __shared__ int s_cnt[kBlock];
    __shared__ double red[64];
    __shared__ double s_f[kBlock * 3];
    extern __shared__ double s_dyn[];
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int2 item = items[it];
        const PairArgs a = table[item.x];
        // (a system without cluster lists sums as it does alone: k_pair)
        if (item.y < a.n_clusters)
            cluster_tile(a, item.y, s_dyn, s_cnt, red, s_f);
        else if (a.n_clusters == 0 && a.paired)
            pair_tile<false, false, true>(a, item.y, s_cnt, red, s_f);
        else
            pair_tile(a, item.y, s_cnt, red, s_f);
        __syncthreads();
    }
}

int pair_subgroups(int N, int P)
{
    int dev = 0, ncu = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess) ncu = prop.multiProcessorCount;
    }
    // aim for at least 16 waves per CU
    const long long target = 16LL * 64 * ncu;
    int S = 1;
    while (2 * S * P <= kBlock && (long long)N * P * S < target) S *= 2;
    return S;
}

int pair_grid(int N, int P, int S)
{
    const int A = kBlock / (S * P);
    return (N + A - 1) / A;
}

int pair_active_tiles(int n_active, int P, int S)
{
    const int A = kBlock / (S * P);
    return (n_active + A - 1) / A;
}

void launch_fused_batch(const FusedArgs *table, const int2 *items, int n_items, int mode,
                        int smem_bytes, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_fused_batch, dim3(grid), dim3(kBlock), smem_bytes, s, table, items,
                       n_items, mode);
}

void launch_finalize_batch(const FusedArgs *table, const int *nparts, int n_sys, int mode,
                           hipStream_t s)
{
    const int grid = n_sys < 1024 ? n_sys : 1024;
    hipLaunchKernelGGL(k_finalize_batch, dim3(grid), dim3(kBlock), 0, s, table, nparts, n_sys, mode);
}

void launch_pair_batch(const PairArgs *table, const int2 *items, int n_items, int grid,
                       bool clusters, bool paired, hipStream_t s)
{
    if (clusters)
        hipLaunchKernelGGL(k_pair_batch_clusters, dim3(grid), dim3(kBlock), kClusterSmem, s, table,
                           items, n_items);
    else if (paired)
        hipLaunchKernelGGL(k_pair_batch<true>, dim3(n_items), dim3(kBlock), 0, s, table, items, n_items);
    else
        hipLaunchKernelGGL(k_pair_batch<false>, dim3(n_items), dim3(kBlock), 0, s, table, items, n_items);
}

void set_batch_smem(int smem_bytes)
{
    (void)hipFuncSetAttribute((const void *)k_fused_batch, hipFuncAttributeMaxDynamicSharedMemorySize,
                              smem_bytes);
}

// The force pass's cluster path uses kClusterSmem bytes of dynamic LDS.
void set_pair_smem()
{
    (void)hipFuncSetAttribute((const void *)k_pair_clusters, hipFuncAttributeMaxDynamicSharedMemorySize,
                              kClusterSmem);
    (void)hipFuncSetAttribute((const void *)k_pair_batch_clusters,
                              hipFuncAttributeMaxDynamicSharedMemorySize, kClusterSmem);
}

// The force pass of a system under a barostat (per-atom lists; cells binned
// in the moving box).
template <bool PAIRED>
__global__ __launch_bounds__(kBlock) void k_pair_npt(PairArgs a)
{
    __shared__ int s_cnt[kBlock];
    __shared__ double red[64];
    __shared__ double s_f[kBlock * 3];
    const int b = blockIdx.x, nA = a.n_active_tiles;
    const int tile = (b < nA) ? xcd_tile(b, nA) : nA + xcd_tile(b - nA, gridDim.x - nA);
    if (a.fdiag)
        pair_tile<true, true, PAIRED>(a, tile, s_cnt, red, s_f);
    else
        pair_tile<true, false, PAIRED>(a, tile, s_cnt, red, s_f);
}

void launch_pair_npt(const PairArgs &a, int grid, hipStream_t s)
{
    if (a.paired)
        hipLaunchKernelGGL(k_pair_npt<true>, dim3(grid), dim3(kBlock), 0, s, a);
    else
        hipLaunchKernelGGL(k_pair_npt<false>, dim3(grid), dim3(kBlock), 0, s, a);
}

void launch_pair(const PairArgs &a, int grid, hipStream_t s)
{
    if (a.n_clusters)
        hipLaunchKernelGGL(k_pair_clusters, dim3(grid), dim3(kBlock), kClusterSmem, s, a);
    else if (a.paired)
        hipLaunchKernelGGL(k_pair<true>, dim3(grid), dim3(kBlock), 0, s, a);
    else
        hipLaunchKernelGGL(k_pair<false>, dim3(grid), dim3(kBlock), 0, s, a);
}

// --------------------------------------------------------------------------
// Layout conversion between the host layout [P][N][3] (caller's atom order)
// and the device layout [N][3][P] (internal order).
// --------------------------------------------------------------------------
__global__ void k_import(const double *src, double *dst, const int *orig, int N, int P)
{
    const size_t n = (size_t)N * 3 * P;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
         e += (size_t)gridDim.x * blockDim.x) {
        const int k = (int)(e % P);
        const int d = (int)((e / P) % 3);
        const int i = (int)(e / (3 * (size_t)P));
        dst[e] = src[((size_t)k * N + orig[i]) * 3 + d];
    }
}

void launch_import(const double *src, double *dst, const int *orig, int N, int P, hipStream_t s)
{
    const size_t n = (size_t)N * 3 * P;
    const int grid = (int)((n + 255) / 256 < 65536 ? (n + 255) / 256 : 65536);
    hipLaunchKernelGGL(k_import, dim3(grid), dim3(256), 0, s, src, dst, orig, N, P);
}

// x: device positions; v: device normal-mode velocities; writes host-layout
// positions and Cartesian momenta p = m M^T v~.
__global__ void k_export(const double *x, const double *v, const double *mass, const double *M,
                         const int *orig, double *xdst, double *pdst, int N, int P)
{
    const size_t n = (size_t)N * 3 * P;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
         e += (size_t)gridDim.x * blockDim.x) {
        const int j = (int)(e % P);
        const int d = (int)((e / P) % 3);
        const int i = (int)(e / (3 * (size_t)P));
        const size_t base = ((size_t)i * 3 + d) * P;
        double s = 0.0;
        for (int m = 0; m < P; ++m) s += M[(size_t)m * P + j] * v[base + m];
        const size_t o = ((size_t)j * N + orig[i]) * 3 + d;
        if (xdst) xdst[o] = x[e];
        if (pdst) pdst[o] = mass[i] * s;
    }
}

void launch_export(const double *x, const double *v, const double *mass, const double *M,
                   const int *orig, double *xdst, double *pdst, int N, int P, hipStream_t s)
{
    const size_t n = (size_t)N * 3 * P;
    const int grid = (int)((n + 255) / 256 < 65536 ? (n + 255) / 256 : 65536);
    hipLaunchKernelGGL(k_export, dim3(grid), dim3(256), 0, s, x, v, mass, M, orig, xdst, pdst, N,
                       P);
}

// --------------------------------------------------------------------------
// Control-block maintenance (kernels, so that graphs never hold memsets).
// --------------------------------------------------------------------------
__global__ void k_ctl_reset_sums(Ctl *c)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        c->count = 0;
        for (int q = 0; q < kNumEst; ++q) {
            c->sum[q] = 0.0;
            c->sumsq[q] = 0.0;
        }
    }
}

// fixcom: remove a pending centroid-mode velocity from every atom (mode 0 of
// v~ for each dim), then clear the flag in a launch of its own.
__global__ void k_apply_ucom(FusedArgs a)
{
    if (!a.ctl->ucom_pending) return;
    const double u0 = a.ctl->ucom[0], u1 = a.ctl->ucom[1], u2 = a.ctl->ucom[2];
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < a.N; i += gridDim.x * blockDim.x) {
        const size_t b = (size_t)i * 3 * a.P;
        a.v[b] -= u0;
        a.v[b + a.P] -= u1;
        a.v[b + 2 * (size_t)a.P] -= u2;
    }
}

__global__ void k_clear_ucom(Ctl *c)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) c->ucom_pending = 0;
}

void launch_apply_ucom(const FusedArgs &a, hipStream_t s)
{
    const int grid = (a.N + 255) / 256 < 1024 ? (a.N + 255) / 256 : 1024;
    hipLaunchKernelGGL(k_apply_ucom, dim3(grid), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_clear_ucom, dim3(1), dim3(64), 0, s, a.ctl);
}

__global__ void k_store_energy(double *dst, double v)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        dst[0] = v;     // the caller's potential energy
        dst[1] = 0.0;   // no cell virial for forces from outside
    }
}

void launch_store_energy(double *dst, double v, hipStream_t s)
{
    hipLaunchKernelGGL(k_store_energy, dim3(1), dim3(64), 0, s, dst, v);
}

__global__ void k_ctl_init(Ctl *c, unsigned long long step)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        c->step = step;
        c->synced = 1;
        c->rebuild = 1;
        c->rlist = 0.0;
        c->ebuild = 0.0;
        c->nonfinite = 0;
        c->overflow = 0;
        c->n_rebuilds = 0;
        c->budget = -1;
        c->ran = 1;
        c->cell_ok = 0;
        c->ucom[0] = c->ucom[1] = c->ucom[2] = 0.0;
        c->ucom_pending = 0;
        c->est_step = step;
        c->count = 0;
        for (int q = 0; q < kNumEst; ++q) {
            c->value[q] = 0.0;
            c->sum[q] = 0.0;
            c->sumsq[q] = 0.0;
        }
    }
}

__global__ void k_ctl_set_budget(Ctl *c, long long budget)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) c->budget = budget;
}

void launch_ctl_set_budget(Ctl *ctl, long long budget, hipStream_t s)
{
    hipLaunchKernelGGL(k_ctl_set_budget, dim3(1), dim3(64), 0, s, ctl, budget);
}

void launch_ctl_reset_sums(Ctl *ctl, hipStream_t s)
{
    hipLaunchKernelGGL(k_ctl_reset_sums, dim3(1), dim3(64), 0, s, ctl);
}

void launch_ctl_init(Ctl *ctl, unsigned long long step, hipStream_t s)
{
    hipLaunchKernelGGL(k_ctl_init, dim3(1), dim3(64), 0, s, ctl, step);
}

}  // namespace pimd
