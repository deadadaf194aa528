// The BZP barostat (App. E): NpT, or NpH with both thermostats off;
// isotropic (one v_W) or anisotropic (one v_W per dimension, each driven by
// the diagonal element of the centroid-virial stress tensor in its
// dimension and scaling the centroids and the box in that dimension).
// An OBABO step at a synchronized state is
//   O(dt/2) on the beads and on v_W; B(dt/2) on v_W and the beads together;
//   A(dt): the centroid mode under the barostat, the other modes by the free
//   ring-polymer flow, L <- exp(dt v_W) L; forces in the new box;
//   B(dt/2); O(dt/2) on v_W and on the beads.
// A BAOAB step is B(dt/2); A(dt/2); O(dt) on the beads and on v_W; A(dt/2)
// with the new v_W; forces; B(dt/2).
// The barostat's force is (3/W)[P V (P_CV - P_ext) + P kB T], the value for
// which the enthalpy H + K_W + U_W + J_W (App. A) is conserved in NpH.  Its
// kick is the exact flow of the kick: the centroid kinetic term, linear in
// time along the kick, integrates to h sum m|v~0|^2 + h^2 sum f~0.v~0 +
// (h^3/3) sum |f~0|^2/m from the momenta at the kick's start.  Its O step
// over a time t uses c1 = exp(-t/tau_0) and noise sqrt(P kB T / W) z, z the
// first Gaussian of counter (2^64 - 1, 0, s, q).
//
// The kicks need sums over all atoms taken between per-element updates, so a
// step is two passes, each followed by a one-block finalize (scalar barostat
// work), then the force pass in the new box.
#include "pimd_internal.h"
#include "pimd_device.h"

namespace pimd {

int npt_grid(int N, int P)
{
    const int A = kBlock / P;
    return (N + A - 1) / A;
}

// sinh(u)/u, by its Taylor series near 0
__device__ __forceinline__ double sinhc(double u)
{
    if (fabs(u) < 1e-3) {
        const double u2 = u * u;
        return 1.0 + u2 / 6.0 * (1.0 + u2 / 20.0 * (1.0 + u2 / 42.0));
    }
    return sinh(u) / u;
}

// v_W after a kick of length h.  k0x2 = sum m |v~0|^2, fv = sum f~0 . v~0,
// f2 = sum |f~0|^2 / m at the kick's start; k0x2 - vir + w = 3 P V P_CV.
__device__ double baro_kick(const NptArgs &a, double vw, double h, double k0x2, double vir,
                            double w, double V, double fv, double f2)
{
    const double W = a.wmass;
    return vw + h / W * (k0x2 - vir + w - 3.0 * (double)a.f.P * V * a.p_ext + 3.0 * a.kTP) +
           h * h / W * fv + h * h * h / (3.0 * W) * f2;
}

// One dimension's v_W after a kick of length h (anisotropic): the sums are
// that dimension's; k0x2 - vir + w = P V P_CV^aa.
__device__ double baro_kick_dim(const NptArgs &a, double vw, double h, double k0x2, double vir,
                                double w, double V, double fv, double f2)
{
    const double W = a.wmass;
    return vw + h / W * (k0x2 - vir + w - (double)a.f.P * V * a.p_ext + a.kTP) + h * h / W * fv +
           h * h * h / (3.0 * W) * f2;
}

// v_W's O step q of step s
__device__ double baro_o(const NptArgs &a, double vw, unsigned long long s, unsigned long long q)
{
    double z[3];
    gauss3(a.f.seed, kBaroNoiseIndex, 0u, s, z, (unsigned)q);
    return a.bc1 * vw + a.bc2 * a.bsig * z[0];
}

// The three v_Wa's O step q of step s (anisotropic): the three Gaussians of
// the barostat's counter, one per dimension
__device__ void baro_o3(const NptArgs &a, double vw[3], unsigned long long s, unsigned long long q)
{
    double z[3];
    gauss3(a.f.seed, kBaroNoiseIndex, 0u, s, z, (unsigned)q);
#pragma unroll
    for (int d = 0; d < 3; ++d) vw[d] = a.bc1 * vw[d] + a.bc2 * a.bsig * z[d];
}

// v_W of dimension d: the isotropic one, or that dimension's
__device__ __forceinline__ double vw_of(const NptArgs &a, const Ctl *c, int d)
{
    return a.aniso ? c->vwa[d] : c->vw;
}

// Pass A.  Thread = (atom, mode); a block holds kBlock/P whole atoms.
// Pending closing kick (with the barostat's sums before it) and O(dt/2) of the
// last step; the estimators' sums; with NPT_STEP the opening O(dt/2) and the
// barostat's sums after it.  Writes v~ and f~.
__global__ __launch_bounds__(kBlock) void k_npt_a(NptArgs na, int mode)
{
    const FusedArgs &a = na.f;
    const int P = a.P, N = a.N, A = kBlock / P;
    __shared__ double sX[3 * kBlock];
    __shared__ double sF[3 * kBlock];
    __shared__ double red[NP_COUNT_ANISO * (kBlock / 64)];
    const int t = threadIdx.x, la = t / P, k = t - la * P;
    const int i = blockIdx.x * A + la;
    const bool act = la < A && i < N;
    const unsigned long long step = a.ctl->step;
    const bool closing = mode != NPT_EST && !a.ctl->synced;
    const bool opening = mode == NPT_STEP;
    const bool an = na.aniso != 0;
    const size_t vb = (size_t)i * 3 * P + k;
    if (act) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            sX[(la * 3 + d) * P + k] = a.x[vb + d * P];
            sF[(la * 3 + d) * P + k] = a.f[vb + d * P];
        }
    }
    __syncthreads();
    double acc[NP_COUNT_ANISO];
#pragma unroll
    for (int q = 0; q < NP_COUNT_ANISO; ++q) acc[q] = 0.0;
    if (act) {
        const double *xr = sX + la * 3 * P, *fr = sF + la * 3 * P;
        const double *Mk = a.M + (size_t)k * P;
        double yt[3] = {0.0, 0.0, 0.0}, ft[3] = {0.0, 0.0, 0.0}, vt[3];
        for (int j = 0; j < P; ++j) {
            const double m = Mk[j];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                yt[d] += m * (xr[d * P + j] - xr[d * P]);
                ft[d] += m * fr[d * P + j];
            }
        }
        const double hm = a.atoms[i * 4 + AT_HALF_M], im = a.atoms[i * 4 + AT_INV_M];
        const double sg = a.atoms[i * 4 + AT_SIGMA];
        const unsigned oi = (unsigned)a.orig[i];
        const double *mk = a.modes + k * 8;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            vt[d] = a.v[vb + d * P];
            na.ft[vb + d * P] = ft[d];
        }
        auto o_step = [&](unsigned long long s_, unsigned long long q_) {
            double z[3];
            gauss3(a.seed, oi, (unsigned)k, s_, z, (unsigned)q_);
#pragma unroll
            for (int d = 0; d < 3; ++d) vt[d] = mk[MD_C1] * vt[d] + mk[MD_C2] * sg * z[d];
        };
        if (closing) {
            if (k == 0) {
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    acc[NP_K0A] += hm * vt[d] * vt[d];
                    acc[NP_FVA] += ft[d] * vt[d];
                    if (an) {
                        acc[NP_K0A3 + d] += hm * vt[d] * vt[d];
                        acc[NP_FVA3 + d] += ft[d] * vt[d];
                    }
                }
            }
#pragma unroll
            for (int d = 0; d < 3; ++d) vt[d] += a.hdt * im * ft[d];
            if (a.obabo && a.nvt) o_step(step - 1, 1);
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            acc[NP_EKIN] += hm * vt[d] * vt[d];
            acc[NP_ESPRING] += hm * mk[MD_SPRING] * yt[d] * yt[d];
            acc[NP_VIR] += mk[MD_NONCENTROID] * yt[d] * ft[d];
            if (an) acc[NP_VIR3 + d] += mk[MD_NONCENTROID] * yt[d] * ft[d];
            if (k == 0) {
                acc[NP_K0] += hm * vt[d] * vt[d];
                acc[NP_F2] += ft[d] * ft[d] * im;
                if (an) acc[NP_F23 + d] += ft[d] * ft[d] * im;
            }
        }
        if (opening) {
            if (a.obabo && a.nvt) o_step(step, 0);
            if (k == 0) {
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    acc[NP_K0B] += hm * vt[d] * vt[d];
                    acc[NP_FVB] += ft[d] * vt[d];
                    if (an) {
                        acc[NP_K0B3 + d] += hm * vt[d] * vt[d];
                        acc[NP_FVB3 + d] += ft[d] * vt[d];
                    }
                }
            }
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            a.v[vb + d * P] = vt[d];
            if (!isfinite(vt[d])) acc[NP_BAD] = 1.0;
        }
    }
    if (an) {
        block_sum<NP_COUNT_ANISO>(acc, red);
    } else {
        double acc0[NP_COUNT];
#pragma unroll
        for (int q = 0; q < NP_COUNT; ++q) acc0[q] = acc[q];
        block_sum<NP_COUNT>(acc0, red);
#pragma unroll
        for (int q = 0; q < NP_COUNT; ++q) acc[q] = acc0[q];
    }
    if (t == 0) {
        double *pp = na.part + (size_t)blockIdx.x * NP_COUNT_ANISO;
#pragma unroll
        for (int q = 0; q < NP_COUNT_ANISO; ++q) pp[q] = acc[q];
    }
}

// Pass A's finalize (one block): the closing barostat kick and O step, the
// estimators of the synchronized state, then the opening O step and kick.
__global__ __launch_bounds__(kBlock) void k_npt_fin_a(NptArgs na, int mode, int nblocks)
{
    const FusedArgs &a = na.f;
    Ctl *c = a.ctl;
    // pass A's sums, then the force pass's energy and cell virial, then
    // (anisotropic) the diagonal of the cell virial
    constexpr int NT0 = NP_COUNT + 2;
    constexpr int TE = NP_COUNT_ANISO, TW = TE + 1, TD = TE + 2, NT = TE + 5;
    __shared__ double red[NT * (kBlock / 64)];
    const int t = threadIdx.x;
    const bool an = na.aniso != 0;
    double tot[NT];
#pragma unroll
    for (int q = 0; q < NT; ++q) tot[q] = 0.0;
    for (int b = t; b < nblocks; b += kBlock) {
#pragma unroll
        for (int q = 0; q < NP_COUNT_ANISO; ++q)
            if (an || q < NP_COUNT) tot[q] += na.part[(size_t)b * NP_COUNT_ANISO + q];
    }
    const double2 *fp = reinterpret_cast<const double2 *>(a.fpartials);
    for (int b = t; b < a.n_fpartials; b += kBlock) {
        const double2 e = fp[b];
        tot[TE] += e.x;
        tot[TW] += e.y;
        if (an) {
#pragma unroll
            for (int d = 0; d < 3; ++d) tot[TD + d] += na.fdiag[(size_t)b * 3 + d];
        }
    }
    if (an) {
        block_sum<NT>(tot, red);
    } else {
        // the isotropic barostat's sums alone, in the order they always had
        double t0[NT0];
#pragma unroll
        for (int q = 0; q < NP_COUNT; ++q) t0[q] = tot[q];
        t0[NP_COUNT] = tot[TE];
        t0[NP_COUNT + 1] = tot[TW];
        block_sum<NT0>(t0, red);
#pragma unroll
        for (int q = 0; q < NP_COUNT; ++q) tot[q] = t0[q];
        tot[TE] = t0[NP_COUNT];
        tot[TW] = t0[NP_COUNT + 1];
    }
    if (t != 0) return;
    const unsigned long long step = c->step;
    const bool closing = mode != NPT_EST && !c->synced;
    const bool est_now = closing || mode == NPT_EST;
    const double h = a.hdt, P = (double)a.P;
    const double V = c->box[0] * c->box[1] * c->box[2];
    const double vir = tot[NP_VIR], w = tot[TW], f2 = tot[NP_F2];
    double vw = c->vw;
    double vwa[3] = {c->vwa[0], c->vwa[1], c->vwa[2]};
    // the kicks: one v_W, or each dimension's with that dimension's sums
    auto kick = [&](int k0, int fv, int k03, int fv3) {
        if (an) {
#pragma unroll
            for (int d = 0; d < 3; ++d)
                vwa[d] = baro_kick_dim(na, vwa[d], h, 2.0 * tot[k03 + d], tot[NP_VIR3 + d], tot[TD + d], V,
                                       tot[fv3 + d], tot[NP_F23 + d]);
        } else {
            vw = baro_kick(na, vw, h, 2.0 * tot[k0], vir, w, V, tot[fv], f2);
        }
    };
    auto o_step = [&](unsigned long long s_, unsigned long long q_) {
        if (an)
            baro_o3(na, vwa, s_, q_);
        else
            vw = baro_o(na, vw, s_, q_);
    };
    if (closing) {
        kick(NP_K0A, NP_FVA, NP_K0A3, NP_FVA3);
        if (a.obabo && a.nvt) o_step(step - 1, 1);
    }
    if (est_now) {
        const double ekin = tot[NP_EKIN], esp = tot[NP_ESPRING], epot = tot[TE];
        const double i3v = 1.0 / (3.0 * V), iP = 1.0 / P;
        double v[kNumEst];
        v[0] = ekin;
        v[1] = esp;
        v[2] = epot;
        v[3] = ekin + esp + epot;
        v[4] = a.kT15PN - esp * iP;
        v[5] = a.kT15N - vir / (2.0 * P);
        v[6] = ekin * a.temp_norm;
        v[7] = (2.0 * tot[NP_K0] - vir + w) * iP * i3v;
        v[8] = (2.0 * a.kT15PN - (2.0 * esp - w) * iP) * i3v;
        v[9] = (2.0 * ekin + w) * i3v;
        // K_W + U_W + J_W (App. A), with J_W = -P kB T ln V; anisotropic:
        // the three barostat velocities' kinetic energies
        const double kw = an ? 0.5 * na.wmass * (vwa[0] * vwa[0] + vwa[1] * vwa[1] + vwa[2] * vwa[2])
                             : 0.5 * na.wmass * vw * vw;
        const double eb = kw + P * na.p_ext * V - na.kTP * log(V);
        c->volume = V;
        c->ebaro = eb;
        c->enthalpy = v[3] + eb;
        for (int q = 0; q < kNumEst; ++q) c->value[q] = v[q];
        c->est_step = step;
        if (mode != NPT_EST) {
            c->count = c->count + 1;
            for (int q = 0; q < kNumEst; ++q) {
                c->sum[q] += v[q];
                c->sumsq[q] += v[q] * v[q];
            }
        }
    }
    if (closing) c->synced = 1;
    if (mode == NPT_STEP) {
        if (a.obabo && a.nvt) o_step(step, 0);
        kick(NP_K0B, NP_FVB, NP_K0B3, NP_FVB3);
    }
    c->vw = vw;
#pragma unroll
    for (int d = 0; d < 3; ++d) c->vwa[d] = vwa[d];
    if (tot[NP_BAD] != 0.0) c->nonfinite = 1;
    c->ran = 1;
}

// Pass B.  Thread = (atom, mode) for the kick and the A step, then
// (atom, bead) for the inverse transform.  Writes v~, x and the centroids.
__global__ __launch_bounds__(kBlock) void k_npt_b(NptArgs na)
{
    const FusedArgs &a = na.f;
    const int P = a.P, N = a.N, A = kBlock / P;
    __shared__ double sX[3 * kBlock];
    __shared__ double red[64];
    const int t = threadIdx.x, la = t / P, k = t - la * P;
    const int i = blockIdx.x * A + la;
    const bool act = la < A && i < N;
    const unsigned long long step = a.ctl->step;
    // v_W per dimension (the isotropic one three times); BAOAB: v_W for the
    // second A(dt/2), after its O(dt) (noise alone, so every thread forms it;
    // the finalize forms the same value)
    double vw[3], vw2[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) vw[d] = vw2[d] = vw_of(na, a.ctl, d);
    if (!a.obabo && a.nvt) {
        if (na.aniso) {
            baro_o3(na, vw2, step, 0);
        } else {
            const double v2 = baro_o(na, vw[0], step, 0);
#pragma unroll
            for (int d = 0; d < 3; ++d) vw2[d] = v2;
        }
    }
    const size_t vb = (size_t)i * 3 * P + k;
    const double sqrtP = sqrt((double)P);
    if (act) {
#pragma unroll
        for (int d = 0; d < 3; ++d) sX[(la * 3 + d) * P + k] = a.x[vb + d * P];
    }
    __syncthreads();
    double yt[3] = {0.0, 0.0, 0.0}, x0[3] = {0.0, 0.0, 0.0};
    double active = 0.0;
    if (act) {
        const double *xr = sX + la * 3 * P;
        const double *Mk = a.M + (size_t)k * P;
#pragma unroll
        for (int d = 0; d < 3; ++d) x0[d] = xr[d * P];
        for (int j = 0; j < P; ++j) {
            const double m = Mk[j];
#pragma unroll
            for (int d = 0; d < 3; ++d) yt[d] += m * (xr[d * P + j] - x0[d]);
        }
        const double im = a.atoms[i * 4 + AT_INV_M];
        const double sg = a.atoms[i * 4 + AT_SIGMA];
        active = a.atoms[i * 4 + AT_ACTIVE];
        const double *mk = a.modes + k * 8;
        double vt[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) vt[d] = a.v[vb + d * P] + a.hdt * im * na.ft[vb + d * P];
        // A over a time t_: the centroid under the barostat (velocity vw_),
        // in absolute coordinates x~0 = y~0 + sqrt(P) x_0; the other modes by
        // the free ring-polymer flow, A(dt/2) n_ times
        auto a_flow = [&](double t_, const double *vw_, int n_) {
            if (k == 0) {
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const double u = t_ * vw_[d];
                    const double e = exp(u), ei = exp(-u), s = t_ * sinhc(u);
                    const double X = e * (yt[d] + sqrtP * x0[d]) + s * vt[d];
                    vt[d] *= ei;
                    yt[d] = X - sqrtP * x0[d];
                }
            } else {
                for (int rep = 0; rep < n_; ++rep) {
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        const double q = yt[d], p = vt[d];
                        yt[d] = mk[MD_A00] * q + mk[MD_A01] * p;
                        vt[d] = mk[MD_A10] * q + mk[MD_A11] * p;
                    }
                }
            }
        };
        if (a.obabo) {
            a_flow(na.dt, vw, 2);
        } else {
            // A(dt/2), O(dt) on the beads (the step's one draw), A(dt/2)
            a_flow(a.hdt, vw, 1);
            if (a.nvt) {
                double z[3];
                gauss3(a.seed, (unsigned)a.orig[i], (unsigned)k, step, z, 0u);
#pragma unroll
                for (int d = 0; d < 3; ++d) vt[d] = mk[MD_C1] * vt[d] + mk[MD_C2] * sg * z[d];
            }
            a_flow(a.hdt, vw2, 1);
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) a.v[vb + d * P] = vt[d];
    }
    __syncthreads();   // every read of the x tile is done
    if (act) {
#pragma unroll
        for (int d = 0; d < 3; ++d) sX[(la * 3 + d) * P + k] = yt[d];
    }
    __syncthreads();
    double m3[3] = {0.0, 0.0, 0.0};   // dmax^2, emax^2, non-finite
    if (act) {
        // bead j = k: x_j = x_0 + sum_m M[m][j] y~_m
        const double *yr = sX + la * 3 * P;
        double xj[3] = {0.0, 0.0, 0.0};
        for (int m = 0; m < P; ++m) {
            const double w = a.M[(size_t)m * P + k];
#pragma unroll
            for (int d = 0; d < 3; ++d) xj[d] += w * yr[d * P + m];
        }
        double c[3], e2 = 0.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            xj[d] += x0[d];
            a.x[vb + d * P] = xj[d];
            c[d] = x0[d] + yr[d * P] / sqrtP;
            const double dd = xj[d] - c[d];
            e2 += dd * dd;
            if (!isfinite(xj[d])) m3[2] = 1.0;
        }
        if (active != 0.0) m3[1] = e2;
        if (k == 0) {
            // displacement from the last build's centroid carried along by the
            // box scaling (per dimension) since that build
            double sd[3];
#pragma unroll
            for (int d = 0; d < 3; ++d)
                sd[d] = a.obabo ? exp(na.dt * vw[d]) : exp(a.hdt * vw[d]) * exp(a.hdt * vw2[d]);
            double d2 = 0.0;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const double g = a.ctl->box[d] * sd[d] / a.ctl->box_build[d];
                a.cent[i * 3 + d] = c[d];
                const double dd = c[d] - g * a.cref[i * 3 + d];
                d2 += dd * dd;
            }
            if (active != 0.0) m3[0] = d2;
            if (a.ncell > 0 && i < a.n_active) {
                // the centroid's cell in the box after this step's scaling
                double bn[3], icw[3];
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    bn[d] = a.ctl->box[d] * sd[d];
                    icw[d] = (double)a.nc[d] / bn[d];
                }
                (void)cell_of_in(a, i, c, bn, icw);
            }
        }
    }
    block_maxv<3>(m3, red);
    if (t == 0) {
        double *pp = na.part + (size_t)blockIdx.x * 3;
        pp[0] = m3[0];
        pp[1] = m3[1];
        pp[2] = m3[2];
    }
}

// Pass B's finalize (one block): the box follows v_W, the step counter
// advances, and the neighbor lists are rebuilt when a bead pair inside rc
// may be missing: with g the box's scaling since the build, a pair's
// centroid distance then was at most (rc + 2 E + 2 dmax) / g, which must not
// exceed the lists' cutoff.
__global__ __launch_bounds__(kBlock) void k_npt_fin_b(NptArgs na, int nblocks)
{
    const FusedArgs &a = na.f;
    Ctl *c = a.ctl;
    __shared__ double red[64];
    __shared__ __align__(16) int sbuf[4 * kMaxCells];
    __shared__ int sflag[1];
    __shared__ double s_dec[5];   // rebuild flag, r_list, new box
    const int t = threadIdx.x;
    double m3[3] = {0.0, 0.0, 0.0};
    for (int b = t; b < nblocks; b += kBlock) {
#pragma unroll
        for (int q = 0; q < 3; ++q) m3[q] = fmax(m3[q], na.part[(size_t)b * 3 + q]);
    }
    block_maxv<3>(m3, red);
    if (t == 0) {
        if (na.aniso) {
            double v1[3] = {c->vwa[0], c->vwa[1], c->vwa[2]}, v2[3] = {v1[0], v1[1], v1[2]};
            if (a.obabo) {
#pragma unroll
                for (int d = 0; d < 3; ++d) c->box[d] *= exp(na.dt * v1[d]);
            } else {
                if (a.nvt) baro_o3(na, v2, c->step, 0);
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    c->box[d] = c->box[d] * exp(a.hdt * v1[d]) * exp(a.hdt * v2[d]);
                    c->vwa[d] = v2[d];
                }
            }
        } else if (a.obabo) {
            const double s = exp(na.dt * c->vw);
#pragma unroll
            for (int d = 0; d < 3; ++d) c->box[d] *= s;
        } else {
            // the two A(dt/2), around v_W's O(dt)
            const double vw1 = c->vw;
            const double vw2 = a.nvt ? baro_o(na, vw1, c->step, 0) : vw1;
            const double s1 = exp(a.hdt * vw1), s2 = exp(a.hdt * vw2);
#pragma unroll
            for (int d = 0; d < 3; ++d) c->box[d] = c->box[d] * s1 * s2;
            c->vw = vw2;
        }
        c->step = c->step + 1;
        c->synced = 0;
        if (c->budget > 0) c->budget = c->budget - 1;
        const double dmax = sqrt(m3[0]), emax = sqrt(m3[1]);
        // the smallest scaling of any dimension since the build bounds a
        // pair's distance then by its distance now over g
        double g = c->box[0] / c->box_build[0];
        if (na.aniso) {
#pragma unroll
            for (int d = 1; d < 3; ++d) g = fmin(g, c->box[d] / c->box_build[d]);
        }
        const bool rebuild = a.rc + 2.0 * (emax + dmax) > g * c->rlist;
        const double rl = a.rc + a.skin + 2.0 * emax;
        if (rebuild) {
            c->rebuild = 1;
            c->ebuild = emax;
            c->rlist = rl;
            c->n_rebuilds = c->n_rebuilds + 1;
#pragma unroll
            for (int d = 0; d < 3; ++d) c->box_build[d] = c->box[d];
        } else {
            c->rebuild = 0;
        }
        if (m3[2] != 0.0) c->nonfinite = 1;
        c->ran = 1;
        s_dec[0] = rebuild ? 1.0 : 0.0;
        s_dec[1] = rl;
#pragma unroll
        for (int d = 0; d < 3; ++d) s_dec[2 + d] = c->box[d];
    }
    // the centroid cell lists of a rebuild, binned in the new box by pass B
    if (a.ncell > 0) {
        __syncthreads();
        if (s_dec[0] != 0.0) {
            double icw[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) icw[d] = (double)a.nc[d] / s_dec[2 + d];
            cells_finalize(a, icw, s_dec[1], sbuf, sflag);
        }
    }
}

__global__ void k_npt_init(Ctl *c, double b0, double b1, double b2, double vw, double vx,
                           double vy, double vz)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        c->box[0] = c->box_build[0] = b0;
        c->box[1] = c->box_build[1] = b1;
        c->box[2] = c->box_build[2] = b2;
        c->vw = vw;
        c->vwa[0] = vx;
        c->vwa[1] = vy;
        c->vwa[2] = vz;
        c->volume = b0 * b1 * b2;
        c->ebaro = 0.0;
        c->enthalpy = 0.0;
    }
}

void launch_npt_init(Ctl *ctl, const double box[3], const double vw[3], hipStream_t s)
{
    hipLaunchKernelGGL(k_npt_init, dim3(1), dim3(64), 0, s, ctl, box[0], box[1], box[2], vw[0], vw[0],
                       vw[1], vw[2]);
}

void launch_npt_a(const NptArgs &a, int mode, hipStream_t s)
{
    const int grid = npt_grid(a.f.N, a.f.P);
    hipLaunchKernelGGL(k_npt_a, dim3(grid), dim3(kBlock), 0, s, a, mode);
    hipLaunchKernelGGL(k_npt_fin_a, dim3(1), dim3(kBlock), 0, s, a, mode, grid);
}

void launch_npt_b(const NptArgs &a, hipStream_t s)
{
    const int grid = npt_grid(a.f.N, a.f.P);
    hipLaunchKernelGGL(k_npt_b, dim3(grid), dim3(kBlock), 0, s, a);
    hipLaunchKernelGGL(k_npt_fin_b, dim3(1), dim3(kBlock), 0, s, a, grid);
}

}  // namespace pimd
