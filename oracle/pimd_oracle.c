/*
 * pimd_oracle.c -- plain CPU FP64 reference for the ring-polymer BAOAB step
 * with the PILE-L thermostat (arXiv:2602.13553).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by tests, the smoke check and the
 * benchmark's CPU-baseline leg; never by the product path.
 *
 * Built with -O2 -ffp-contract=off (no FMA contraction, no fast-math).  The
 * force loops carry an OpenMP pragma so the CPU baseline can use the host's
 * cores; every reduction is done serially afterwards in a fixed order, so the
 * result does not depend on the thread count.
 */
#include "pimd_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

static const double PI = 3.14159265358979323846;

/* ------------------------------------------------------------------------
 * Normal-mode matrix, App. B Eq. (B1).  Row i is the mode, column j the bead.
 *   i = 0                 : 1/sqrt(P)
 *   i = P/2 (P even)      : (-1)^j / sqrt(P)
 *   1 <= i <= floor(P/2)  : sqrt(2/P) cos(2 pi i j / P)
 *   floor(P/2) < i < P    : sqrt(2/P) sin(2 pi i j / P)
 * For P even the row i = P/2 matches both the second and third case; the
 * second (normalized) one is taken.  The angle's integer part (i*j mod P) is
 * reduced before the trigonometric call; this changes only rounding.
 * Pinned: orthogonality, M A M^T = diag(lambda), equality with the real-DFT
 * form built from numpy.fft, and the hand values for P = 1, 2.
 * --------------------------------------------------------------------- */
void orc_nm_matrix(int32_t P, double *M)
{
    const double inv_sqrt_p = 1.0 / sqrt((double)P);
    const double sqrt_2_p = sqrt(2.0 / (double)P);
    for (int32_t i = 0; i < P; ++i) {
        for (int32_t j = 0; j < P; ++j) {
            double v;
            long long ij = ((long long)i * (long long)j) % P;
            double ang = 2.0 * PI * (double)ij / (double)P;
            if (i == 0)
                v = inv_sqrt_p;
            else if ((P % 2 == 0) && (i == P / 2))
                v = (j % 2 == 0) ? inv_sqrt_p : -inv_sqrt_p;
            else if (i <= P / 2)
                v = sqrt_2_p * cos(ang);
            else
                v = sqrt_2_p * sin(ang);
            M[(size_t)i * P + j] = v;
        }
    }
}

/* Eq. (B2): lambda_k = 4 sin^2(k pi / P), attached to row k of M.  These are
 * the eigenvalues of the circulant ring Laplacian that M diagonalizes. */
void orc_mode_lambda(int32_t P, double *lam)
{
    for (int32_t k = 0; k < P; ++k) {
        double s = sin(PI * (double)k / (double)P);
        lam[k] = 4.0 * s * s;
    }
}

/* Eq. B1 evaluated in x87 extended precision (64-bit mantissa), used by the
 * transforms below.  Same definition as orc_nm_matrix, higher precision. */
static void nm_matrix_ext(int32_t P, long double *M)
{
    const long double pi = 3.141592653589793238462643383279502884L;
    const long double inv_sqrt_p = 1.0L / sqrtl((long double)P);
    const long double sqrt_2_p = sqrtl(2.0L / (long double)P);
    for (int32_t i = 0; i < P; ++i)
        for (int32_t j = 0; j < P; ++j) {
            long long ij = ((long long)i * (long long)j) % P;
            long double ang = 2.0L * pi * (long double)ij / (long double)P;
            long double v;
            if (i == 0)
                v = inv_sqrt_p;
            else if ((P % 2 == 0) && (i == P / 2))
                v = (j % 2 == 0) ? inv_sqrt_p : -inv_sqrt_p;
            else if (i <= P / 2)
                v = sqrt_2_p * cosl(ang);
            else
                v = sqrt_2_p * sinl(ang);
            M[(size_t)i * P + j] = v;
        }
}

/* Transforms: each element is one dot product of a row (or column) of M with
 * the bead (or mode) values of one atom and dim.  Both M and the sum are
 * carried in x87 extended precision and the result is rounded to FP64 once,
 * so every transformed value is the correctly rounded exact value up to a
 * 2^-11 ulp margin.  Reason: positions are unwrapped and of box size (about
 * 70 A for the water workload) while the non-centroid modes are 0.01-0.1 A.
 * In FP64, (i) the rounded entries of a non-centroid row do not sum to zero
 * exactly, which adds a spurious x * 5e-16 to that mode, and (ii) the
 * summation leaves ~1e-13 A; the stiff ring-polymer springs (m omega_k^2 up
 * to ~100 amu/fs^2) turn either into ~1e-12 relative momentum error within
 * 10 steps.  Extended precision removes both. */
void orc_to_normal(int32_t P, int32_t N, const double *a, double *at)
{
    long double *M = (long double *)malloc(sizeof(long double) * (size_t)P * P);
    nm_matrix_ext(P, M);
    for (int32_t i = 0; i < N; ++i)
        for (int32_t d = 0; d < 3; ++d)
            for (int32_t k = 0; k < P; ++k) {
                long double s = 0.0L;
                for (int32_t j = 0; j < P; ++j)
                    s += M[(size_t)k * P + j] * (long double)a[((size_t)j * N + i) * 3 + d];
                at[((size_t)k * N + i) * 3 + d] = (double)s;
            }
    free(M);
}

/* Eq. (B3): the inverse is the transpose. */
void orc_from_normal(int32_t P, int32_t N, const double *at, double *a)
{
    long double *M = (long double *)malloc(sizeof(long double) * (size_t)P * P);
    nm_matrix_ext(P, M);
    for (int32_t i = 0; i < N; ++i)
        for (int32_t d = 0; d < 3; ++d)
            for (int32_t j = 0; j < P; ++j) {
                long double s = 0.0L;
                for (int32_t k = 0; k < P; ++k)
                    s += M[(size_t)k * P + j] * (long double)at[((size_t)k * N + i) * 3 + d];
                a[((size_t)j * N + i) * 3 + d] = (double)s;
            }
    free(M);
}

/* ------------------------------------------------------------------------
 * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of
 *   (hi0, lo0) = M0 * c0, (hi1, lo1) = M1 * c2   (32 x 32 -> 64-bit products),
 *   c <- (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0),
 * with the key bumped by the Weyl constants between rounds.
 * Pinned against the generator authors' published known answers.
 * --------------------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)M0 * c0, p1 = (uint64_t)M1 * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c0 = n0; c1 = (uint32_t)p1; c2 = n2; c3 = (uint32_t)p0;
        k0 += W0; k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Uniform on (0, 1]: the word plus one, times 2^-32. */
static double u01_open0(uint32_t w)
{
    return ((double)w + 1.0) * (1.0 / 4294967296.0);
}

/* Box-Muller on the four words: (z0, z1) from (u0, u1), z2 from (u2, u3).
 * The paper leaves the generator unspecified (App. D only asks for
 * independent N(0,1) numbers); this keyed, counter-based stream is this
 * implementation's reading.  Counter (i, k, s mod 2^32, floor(s / 2^32) +
 * q 2^31), key (seed mod 2^32, floor(seed / 2^32)): i < 2^32 (an atom, or
 * 2^32 - 1 for the barostat's own noise), k < 2^32, s < 2^31 * 2^32.
 * Pinned by moment tests. */
void orc_gaussians(uint64_t seed, uint32_t i, uint32_t k, uint64_t s, double z[3])
{
    orc_gaussians_q(seed, i, k, s, 0, z);
}

void orc_gaussians_q(uint64_t seed, uint32_t i, uint32_t k, uint64_t s, uint32_t q, double z[3])
{
    const uint32_t ctr[4] = {i, k, (uint32_t)s, (uint32_t)(s >> 32) | (q << 31)};
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t w[4];
    orc_philox4x32_10(ctr, key, w);
    double u0 = u01_open0(w[0]), u1 = u01_open0(w[1]);
    double u2 = u01_open0(w[2]), u3 = u01_open0(w[3]);
    double r0 = sqrt(-2.0 * log(u0));
    double r2 = sqrt(-2.0 * log(u2));
    z[0] = r0 * cos(2.0 * PI * u1);
    z[1] = r0 * sin(2.0 * PI * u1);
    z[2] = r2 * cos(2.0 * PI * u3);
}

/* ------------------------------------------------------------------------
 * Free ring polymer in normal modes.  With physical masses (fmmode
 * physical) the spring part of Eq. 1 is sum_k 1/2 m omega_k^2 x~_k^2 with
 * omega_k = sqrt(lambda_k) omega_n and omega_n = P kB T / hbar (Eq. 2).  The
 * paper does not print the position update; the A step is read as the exact
 * flow of that quadratic Hamiltonian over a time h.
 * Pinned: det A = 1, A(h)A(h) = A(2h), energy conservation of the free ring
 * polymer at zero friction.
 * --------------------------------------------------------------------- */
static double omega_n(const orc_system *sys)
{
    return (double)sys->n_beads * sys->kB * sys->temp / sys->hbar;
}

static double omega_k(const orc_system *sys, int32_t k)
{
    double s = sin(PI * (double)k / (double)sys->n_beads);
    return 2.0 * omega_n(sys) * fabs(s);
}

void orc_free_rp_matrix(const orc_system *sys, int32_t k, double h, double A[4])
{
    double w = (k == 0) ? 0.0 : omega_k(sys, k);
    if (w == 0.0) {
        A[0] = 1.0; A[1] = h; A[2] = 0.0; A[3] = 1.0;
    } else {
        double c = cos(w * h), s = sin(w * h);
        A[0] = c; A[1] = s / w; A[2] = -w * s; A[3] = c;
    }
}

/* App. D, Eqs. (D1)-(D2): tau_0 = tau; tau_k = scale / (2 omega_k) for k >= 1;
 * c1 = exp(-dt/tau_k), c2 = sqrt(1 - c1^2).  The O step spans one full dt. */
void orc_pile_coeffs(const orc_system *sys, int32_t k, double *c1, double *c2)
{
    if (sys->nve) { *c1 = 1.0; *c2 = 0.0; return; }
    double tau_k = (k == 0) ? sys->tau : sys->tau_scale / (2.0 * omega_k(sys, k));
    /* the O step lasts dt in BAOAB and dt/2 for each of OBABO's two */
    double t_o = (sys->integrator == 1) ? 0.5 * sys->dt : sys->dt;
    double a = exp(-t_o / tau_k);
    *c1 = a;
    *c2 = sqrt(1.0 - a * a);
}

/* ------------------------------------------------------------------------
 * Forces.  Every bead is an independent copy of the physical system (the
 * U(r^(k)) term of Eq. 1).  Pair potential: Lennard-Jones among lj_active
 * atoms, truncated at rc with the energy shifted so that u(rc) = 0 and the
 * force left unshifted, summed over all periodic images with
 * |r_ij + n L| < rc (i = j only for n != 0).  Bonds: U = K (r - r0)^2 with the
 * minimum-image bond vector.  Harmonic trap: U = 1/2 m omega^2 |r|^2.
 * Pinned: finite differences of U, Newton's third law, image sum = minimum
 * image for large boxes, small box = replicated large box.
 * --------------------------------------------------------------------- */
static void lj_pair(double eps, double sig, double rc2, double ushift, double r2,
                    double *u, double *fr)
{
    /* u(r) and fr = -(du/dr)/r, for r2 < rc2 */
    (void)rc2;
    double sr2 = sig * sig / r2;
    double sr6 = sr2 * sr2 * sr2;
    double sr12 = sr6 * sr6;
    *u = 4.0 * eps * (sr12 - sr6) - ushift;
    *fr = 24.0 * eps * (2.0 * sr12 - sr6) / r2;
}

double orc_forces_bead(const orc_system *sys, const double *xk, double *fk)
{
    const int32_t N = sys->n_atoms;
    double *eat = (double *)calloc((size_t)N, sizeof(double));
    memset(fk, 0, sizeof(double) * 3 * (size_t)N);

    if (sys->pot == ORC_POT_HARMONIC) {
        for (int32_t i = 0; i < N; ++i) {
            double kk = sys->mass[i] * sys->omega * sys->omega * sys->mvv2e;
            double r2 = 0.0;
            for (int d = 0; d < 3; ++d) {
                fk[3 * i + d] = -kk * xk[3 * i + d];
                r2 += xk[3 * i + d] * xk[3 * i + d];
            }
            eat[i] = 0.5 * kk * r2;
        }
    } else if (sys->pot == ORC_POT_PAIR) {
        const double L0 = sys->box[0], L1 = sys->box[1], L2 = sys->box[2];
        const double rc = sys->lj_rc, rc2 = rc * rc;
        const double eps = sys->lj_eps, sig = sys->lj_sigma;
        double src2 = sig * sig / rc2, src6 = src2 * src2 * src2;
        const double ushift = 4.0 * eps * (src6 * src6 - src6);
        const int minimg = (L0 >= 2.0 * rc) && (L1 >= 2.0 * rc) && (L2 >= 2.0 * rc);
        const int n0 = (int)ceil(rc / L0) + 1, n1 = (int)ceil(rc / L1) + 1,
                  n2 = (int)ceil(rc / L2) + 1;
        if (eps != 0.0) {
#pragma omp parallel for schedule(dynamic, 16)
            for (int32_t i = 0; i < N; ++i) {
                if (sys->lj_active && !sys->lj_active[i]) continue;
                double fx = 0.0, fy = 0.0, fz = 0.0, e = 0.0;
                for (int32_t j = 0; j < N; ++j) {
                    if (sys->lj_active && !sys->lj_active[j]) continue;
                    double dx = xk[3 * i] - xk[3 * j];
                    double dy = xk[3 * i + 1] - xk[3 * j + 1];
                    double dz = xk[3 * i + 2] - xk[3 * j + 2];
                    if (minimg) {
                        if (j == i) continue;
                        dx -= L0 * nearbyint(dx / L0);
                        dy -= L1 * nearbyint(dy / L1);
                        dz -= L2 * nearbyint(dz / L2);
                        double r2 = dx * dx + dy * dy + dz * dz;
                        if (r2 < rc2) {
                            double u, fr;
                            lj_pair(eps, sig, rc2, ushift, r2, &u, &fr);
                            e += 0.5 * u;
                            fx += fr * dx; fy += fr * dy; fz += fr * dz;
                        }
                    } else {
                        for (int a = -n0; a <= n0; ++a)
                            for (int b = -n1; b <= n1; ++b)
                                for (int c = -n2; c <= n2; ++c) {
                                    if (j == i && a == 0 && b == 0 && c == 0) continue;
                                    double ex = dx + a * L0, ey = dy + b * L1, ez = dz + c * L2;
                                    double r2 = ex * ex + ey * ey + ez * ez;
                                    if (r2 < rc2) {
                                        double u, fr;
                                        lj_pair(eps, sig, rc2, ushift, r2, &u, &fr);
                                        e += 0.5 * u;
                                        fx += fr * ex; fy += fr * ey; fz += fr * ez;
                                    }
                                }
                    }
                }
                fk[3 * i] = fx; fk[3 * i + 1] = fy; fk[3 * i + 2] = fz;
                eat[i] = e;
            }
        }
        /* bonds: serial, in the given order */
        for (int32_t b = 0; b < sys->n_bonds; ++b) {
            int32_t i = sys->bonds[2 * b], j = sys->bonds[2 * b + 1];
            double d[3];
            for (int a = 0; a < 3; ++a) {
                d[a] = xk[3 * i + a] - xk[3 * j + a];
                if (sys->box[a] > 0.0) d[a] -= sys->box[a] * nearbyint(d[a] / sys->box[a]);
            }
            double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            double dr = r - sys->bond_r0;
            double u = sys->bond_k * dr * dr;
            double fr = -2.0 * sys->bond_k * dr / r;
            for (int a = 0; a < 3; ++a) {
                fk[3 * i + a] += fr * d[a];
                fk[3 * j + a] -= fr * d[a];
            }
            eat[i] += 0.5 * u;
            eat[j] += 0.5 * u;
        }
    }
    double U = 0.0;
    for (int32_t i = 0; i < N; ++i) U += eat[i];
    free(eat);
    return U;
}

double orc_virial_bead(const orc_system *sys, const double *xk)
{
    const int32_t N = sys->n_atoms;
    if (sys->pot != ORC_POT_PAIR || !(sys->box[0] > 0.0)) return 0.0;
    const double L0 = sys->box[0], L1 = sys->box[1], L2 = sys->box[2];
    const double rc = sys->lj_rc, rc2 = rc * rc;
    const double eps = sys->lj_eps, sig = sys->lj_sigma;
    double src2 = sig * sig / rc2, src6 = src2 * src2 * src2;
    const double ushift = 4.0 * eps * (src6 * src6 - src6);
    const int minimg = (L0 >= 2.0 * rc) && (L1 >= 2.0 * rc) && (L2 >= 2.0 * rc);
    const int n0 = (int)ceil(rc / L0) + 1, n1 = (int)ceil(rc / L1) + 1, n2 = (int)ceil(rc / L2) + 1;
    /* every ordered pair (i, j, image) once, half each: r . F = fr r^2; per
     * atom, then summed in atom order */
    double *wat = (double *)calloc((size_t)(N > 0 ? N : 1), sizeof(double));
    if (eps != 0.0) {
#pragma omp parallel for schedule(dynamic, 16)
        for (int32_t i = 0; i < N; ++i) {
            if (sys->lj_active && !sys->lj_active[i]) continue;
            double wi = 0.0;
            for (int32_t j = 0; j < N; ++j) {
                if (sys->lj_active && !sys->lj_active[j]) continue;
                double dx = xk[3 * i] - xk[3 * j];
                double dy = xk[3 * i + 1] - xk[3 * j + 1];
                double dz = xk[3 * i + 2] - xk[3 * j + 2];
                if (minimg) {
                    /* at most one image of j within rc: the nearest */
                    if (j == i) continue;
                    dx -= L0 * nearbyint(dx / L0);
                    dy -= L1 * nearbyint(dy / L1);
                    dz -= L2 * nearbyint(dz / L2);
                    double r2 = dx * dx + dy * dy + dz * dz;
                    if (r2 < rc2) {
                        double u, fr;
                        lj_pair(eps, sig, rc2, ushift, r2, &u, &fr);
                        wi += 0.5 * fr * r2;
                    }
                    continue;
                }
                for (int a = -n0; a <= n0; ++a)
                    for (int b = -n1; b <= n1; ++b)
                        for (int c = -n2; c <= n2; ++c) {
                            if (j == i && a == 0 && b == 0 && c == 0) continue;
                            double ex = dx + a * L0, ey = dy + b * L1, ez = dz + c * L2;
                            double r2 = ex * ex + ey * ey + ez * ez;
                            if (r2 < rc2) {
                                double u, fr;
                                lj_pair(eps, sig, rc2, ushift, r2, &u, &fr);
                                wi += 0.5 * fr * r2;
                            }
                        }
            }
            wat[i] = wi;
        }
    }
    double w = 0.0;
    for (int32_t i = 0; i < N; ++i) w += wat[i];
    free(wat);
    for (int32_t b = 0; b < sys->n_bonds; ++b) {
        int32_t i = sys->bonds[2 * b], j = sys->bonds[2 * b + 1];
        double d[3];
        for (int a = 0; a < 3; ++a) {
            d[a] = xk[3 * i + a] - xk[3 * j + a];
            d[a] -= sys->box[a] * nearbyint(d[a] / sys->box[a]);
        }
        double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        double fr = -2.0 * sys->bond_k * (r - sys->bond_r0) / r;
        w += fr * r * r;
    }
    return w;
}

void orc_virial_bead_diag(const orc_system *sys, const double *xk, double w[3])
{
    const int32_t N = sys->n_atoms;
    w[0] = w[1] = w[2] = 0.0;
    if (sys->pot != ORC_POT_PAIR || !(sys->box[0] > 0.0)) return;
    const double L[3] = {sys->box[0], sys->box[1], sys->box[2]};
    const double rc = sys->lj_rc, rc2 = rc * rc;
    const double eps = sys->lj_eps, sig = sys->lj_sigma;
    double src2 = sig * sig / rc2, src6 = src2 * src2 * src2;
    const double ushift = 4.0 * eps * (src6 * src6 - src6);
    const int minimg = (L[0] >= 2.0 * rc) && (L[1] >= 2.0 * rc) && (L[2] >= 2.0 * rc);
    const int n0 = minimg ? 0 : (int)ceil(rc / L[0]) + 1, n1 = minimg ? 0 : (int)ceil(rc / L[1]) + 1,
              n2 = minimg ? 0 : (int)ceil(rc / L[2]) + 1;
    /* every ordered pair (i, j, image) once, half each: (r_a)(F_a) = fr r_a^2
     * (the nearest image alone when every box length is at least 2 rc);
     * per atom, then summed in atom order */
    double *wat = (double *)calloc(3 * (size_t)(N > 0 ? N : 1), sizeof(double));
    if (eps != 0.0) {
#pragma omp parallel for schedule(dynamic, 16)
        for (int32_t i = 0; i < N; ++i) {
            if (sys->lj_active && !sys->lj_active[i]) continue;
            double wi[3] = {0.0, 0.0, 0.0};
            for (int32_t j = 0; j < N; ++j) {
                if (sys->lj_active && !sys->lj_active[j]) continue;
                double d0 = xk[3 * i] - xk[3 * j];
                double d1 = xk[3 * i + 1] - xk[3 * j + 1];
                double d2 = xk[3 * i + 2] - xk[3 * j + 2];
                if (minimg) {
                    d0 -= L[0] * nearbyint(d0 / L[0]);
                    d1 -= L[1] * nearbyint(d1 / L[1]);
                    d2 -= L[2] * nearbyint(d2 / L[2]);
                }
                for (int a = -n0; a <= n0; ++a)
                    for (int b = -n1; b <= n1; ++b)
                        for (int c = -n2; c <= n2; ++c) {
                            if (j == i && a == 0 && b == 0 && c == 0) continue;
                            const double e[3] = {d0 + a * L[0], d1 + b * L[1], d2 + c * L[2]};
                            const double r2 = e[0] * e[0] + e[1] * e[1] + e[2] * e[2];
                            if (r2 < rc2) {
                                double u, fr;
                                lj_pair(eps, sig, rc2, ushift, r2, &u, &fr);
                                for (int q = 0; q < 3; ++q) wi[q] += 0.5 * fr * e[q] * e[q];
                            }
                        }
            }
            for (int q = 0; q < 3; ++q) wat[3 * (size_t)i + q] = wi[q];
        }
    }
    for (int32_t i = 0; i < N; ++i)
        for (int q = 0; q < 3; ++q) w[q] += wat[3 * (size_t)i + q];
    free(wat);
    for (int32_t b = 0; b < sys->n_bonds; ++b) {
        int32_t i = sys->bonds[2 * b], j = sys->bonds[2 * b + 1];
        double d[3];
        for (int a = 0; a < 3; ++a) {
            d[a] = xk[3 * i + a] - xk[3 * j + a];
            d[a] -= sys->box[a] * nearbyint(d[a] / sys->box[a]);
        }
        double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        double fr = -2.0 * sys->bond_k * (r - sys->bond_r0) / r;
        for (int a = 0; a < 3; ++a) w[a] += fr * d[a] * d[a];
    }
}

void orc_forces(const orc_system *sys, const double *x, double *f, double *U)
{
    const size_t stride = 3 * (size_t)sys->n_atoms;
    for (int32_t k = 0; k < sys->n_beads; ++k)
        U[k] = orc_forces_bead(sys, x + k * stride, f + k * stride);
}

/* ------------------------------------------------------------------------
 * One BAOAB step in normal modes (Sec. IV.A; Sec. III.C lists BAOAB):
 *   B  v~ += (dt/2) f~/m        with f~ = M f
 *   A  (x~, v~) <- A(dt/2)       with x~ = M x
 *   O  v~ <- c1 v~ + c2 sqrt(P kB T / m) eta     (Eq. D2, thermostat at P T)
 *   A  (x~, v~) <- A(dt/2)
 *      x = M^T x~, f = F(x)
 *   B  v~ += (dt/2) f~/m        with f~ = M f
 * The noise eta for mode k, atom i, dim a at step s is orc_gaussians(seed,
 * i, k, s)[a].
 * --------------------------------------------------------------------- */
/* Half-kick B(h): v~ += h (M f) / m, f in energy/length, v~ in length/time. */
static void orc_kick(const orc_system *sys, double *vt, const double *f, double *ft)
{
    const int32_t P = sys->n_beads, N = sys->n_atoms;
    const double h = 0.5 * sys->dt;
    const double ftm2v = 1.0 / sys->mvv2e;
    orc_to_normal(P, N, f, ft);
    for (int32_t k = 0; k < P; ++k)
        for (int32_t i = 0; i < N; ++i)
            for (int d = 0; d < 3; ++d) {
                size_t e = ((size_t)k * N + i) * 3 + d;
                vt[e] += h * ft[e] * ftm2v / sys->mass[i];
            }
}

/* O step q of step s alone (OBABO): v~ <- c1 v~ + c2 sigma z, mode by mode. */
static void orc_o_step(const orc_system *sys, double *vt, uint64_t s, uint64_t q)
{
    const int32_t P = sys->n_beads, N = sys->n_atoms;
    const double ftm2v = 1.0 / sys->mvv2e;
    if (sys->nve) return;
    for (int32_t k = 0; k < P; ++k) {
        double c1, c2;
        orc_pile_coeffs(sys, k, &c1, &c2);
        for (int32_t i = 0; i < N; ++i) {
            double sigma = sqrt((double)P * sys->kB * sys->temp * ftm2v / sys->mass[i]);
            const uint64_t id = sys->atom_id ? (uint64_t)sys->atom_id[i] : (uint64_t)i;
            double z[3];
            orc_gaussians_q(sys->seed, (uint32_t)id, (uint32_t)k, s, (uint32_t)q, z);
            for (int d = 0; d < 3; ++d) {
                size_t e = ((size_t)k * N + i) * 3 + d;
                vt[e] = c1 * vt[e] + c2 * sigma * z[d];
            }
        }
    }
}

/* OBABO's first part of step s: O(dt/2) (q = 0), B(dt/2) with the current
 * positions' forces, A(dt) as A(dt/2) twice, and the new positions. */
static void orc_step_positions_obabo(const orc_system *sys, double *x, double *vt,
                                     const double *f, uint64_t *step)
{
    const int32_t P = sys->n_beads, N = sys->n_atoms;
    const size_t n = (size_t)P * N * 3;
    const double h = 0.5 * sys->dt;
    double *xt = (double *)malloc(sizeof(double) * n);
    double *ft = (double *)malloc(sizeof(double) * n);
    double Ah[4];
    const uint64_t s = *step;
    orc_o_step(sys, vt, s, 0);
    orc_kick(sys, vt, f, ft);
    orc_to_normal(P, N, x, xt);
    for (int32_t k = 0; k < P; ++k) {
        orc_free_rp_matrix(sys, k, h, Ah);
        for (int32_t i = 0; i < N; ++i)
            for (int d = 0; d < 3; ++d) {
                size_t e = ((size_t)k * N + i) * 3 + d;
                for (int rep = 0; rep < 2; ++rep) {
                    double q = xt[e], p = vt[e];
                    xt[e] = Ah[0] * q + Ah[1] * p;
                    vt[e] = Ah[2] * q + Ah[3] * p;
                }
            }
    }
    orc_from_normal(P, N, xt, x);
    *step = s + 1;
    free(xt);
    free(ft);
}

/* The first part of step s: B(dt/2) with the forces f of the current
 * positions, then A(dt/2), O(dt) with the noise of step s, A(dt/2), and the
 * new Cartesian positions.  The step counter advances to s + 1; the closing
 * B(dt/2) waits for the forces of the new positions (orc_step_kick). */
void orc_step_positions(const orc_system *sys, double *x, double *vt, const double *f,
                        uint64_t *step)
{
    if (sys->integrator == 1) {
        orc_step_positions_obabo(sys, x, vt, f, step);
        return;
    }
    const int32_t P = sys->n_beads, N = sys->n_atoms;
    const size_t n = (size_t)P * N * 3;
    const double h = 0.5 * sys->dt;
    const double ftm2v = 1.0 / sys->mvv2e;
    double *xt = (double *)malloc(sizeof(double) * n);
    double *ft = (double *)malloc(sizeof(double) * n);
    double Ah[4], c1, c2;
    const uint64_t s = *step;
    /* B */
    orc_kick(sys, vt, f, ft);
    /* A, O, A */
    orc_to_normal(P, N, x, xt);
    for (int32_t k = 0; k < P; ++k) {
        orc_free_rp_matrix(sys, k, h, Ah);
        orc_pile_coeffs(sys, k, &c1, &c2);
        for (int32_t i = 0; i < N; ++i) {
            double sigma = sqrt((double)P * sys->kB * sys->temp * ftm2v / sys->mass[i]);
            double z[3] = {0.0, 0.0, 0.0};
            const uint64_t id = sys->atom_id ? (uint64_t)sys->atom_id[i] : (uint64_t)i;
            if (!sys->nve) orc_gaussians(sys->seed, (uint32_t)id, (uint32_t)k, s, z);
            for (int d = 0; d < 3; ++d) {
                size_t e = ((size_t)k * N + i) * 3 + d;
                double q = xt[e], p = vt[e];
                double q1 = Ah[0] * q + Ah[1] * p;
                double p1 = Ah[2] * q + Ah[3] * p;
                if (!sys->nve) p1 = c1 * p1 + c2 * sigma * z[d];
                xt[e] = Ah[0] * q1 + Ah[1] * p1;
                vt[e] = Ah[2] * q1 + Ah[3] * p1;
            }
        }
    }
    orc_from_normal(P, N, xt, x);
    *step = s + 1;
    free(xt);
    free(ft);
}

/* fixcom: the centroid of atom i moves with v~0_i / sqrt(P) (row 0 of M is
 * 1/sqrt(P)), so removing the centroids' center-of-mass velocity V from every
 * bead subtracts sqrt(P) V = sum_j m_j v~0_j / sum_j m_j from every atom's
 * centroid mode and leaves the other modes alone. */
static void orc_remove_com(const orc_system *sys, double *vt)
{
    const int32_t N = sys->n_atoms;
    double msum = 0.0, p[3] = {0.0, 0.0, 0.0};
    for (int32_t i = 0; i < N; ++i) {
        msum += sys->mass[i];
        for (int d = 0; d < 3; ++d) p[d] += sys->mass[i] * vt[(size_t)i * 3 + d];
    }
    for (int32_t i = 0; i < N; ++i)
        for (int d = 0; d < 3; ++d) vt[(size_t)i * 3 + d] -= p[d] / msum;
}

/* The closing B(dt/2) of step s, with the forces f of the new positions, for
 * OBABO the step's second O(dt/2) (q = 1), and the fixcom removal. */
void orc_step_kick(const orc_system *sys, double *vt, const double *f, uint64_t s)
{
    const size_t n = (size_t)sys->n_beads * sys->n_atoms * 3;
    double *ft = (double *)malloc(sizeof(double) * n);
    orc_kick(sys, vt, f, ft);
    if (sys->integrator == 1) orc_o_step(sys, vt, s, 1);
    if (sys->fixcom) orc_remove_com(sys, vt);
    free(ft);
}

void orc_step(const orc_system *sys, double *x, double *vt, double *f, double *U,
              uint64_t *step, int32_t nsteps)
{
    for (int32_t it = 0; it < nsteps; ++it) {
        orc_step_positions(sys, x, vt, f, step);
        /* forces at the new positions, then B (and OBABO's last O) */
        orc_forces(sys, x, f, U);
        orc_step_kick(sys, vt, f, *step - 1);
    }
}

/* ------------------------------------------------------------------------
 * Estimators, App. A.  Read with omega_n^2 wherever the printed formulas
 * show omega_n (dimensional analysis), and with the 1/P on the spring sum of
 * K_PR (Eq. A5), which the printed formula lacks.
 *   K    = sum_k sum_i 1/2 m |v~_i^k|^2
 *   S    = sum_k sum_i 1/2 m omega_n^2 |r_i^k - r_i^(k+1)|^2   (bead form)
 *   K_PR = 3 P N kB T / 2 - S / P
 *   K_CV = 3 N kB T / 2 - (1/2P) sum_k sum_i (r_i^k - r_i^c) . F_i^k
 *   temp = 2 K / (3 N P^2 kB)
 * and, with a periodic box of volume V and W = sum_k Tr Xi^k (orc_virial_bead),
 *   P_CV = (sum_i m |v~_i^0|^2 - sum_k sum_i (r_i^k - r_i^c) . F_i^k + W) / (3 P V)
 *   P_PR = (3 P N kB T - (2 S - W) / P) / (3 V)
 *   P_MD = (2 K + W) / (3 V)
 * P_PR as printed lacks the virial and the 1/P; it is read as kB T times the
 * volume derivative of the log of the ring polymer's Boltzmann weight, the
 * beads' potentials carrying 1/P (the weight of K_PR's 1/P). P_MD is the
 * pressure of the extended classical system of P beads per atom.
 * --------------------------------------------------------------------- */
void orc_estimators(const orc_system *sys, const double *x, const double *vt,
                    const double *f, const double *U, orc_est *out)
{
    const int32_t P = sys->n_beads, N = sys->n_atoms;
    const double wn = omega_n(sys);
    const double kT = sys->kB * sys->temp;
    double ekin = 0.0, espring = 0.0, epot = 0.0, vir = 0.0;
    for (int32_t k = 0; k < P; ++k) {
        int32_t kp = (k + 1) % P;
        for (int32_t i = 0; i < N; ++i) {
            double m = sys->mass[i];
            for (int d = 0; d < 3; ++d) {
                double v = vt[((size_t)k * N + i) * 3 + d];
                ekin += 0.5 * m * sys->mvv2e * v * v;
                double dr = x[((size_t)k * N + i) * 3 + d] - x[((size_t)kp * N + i) * 3 + d];
                espring += 0.5 * m * sys->mvv2e * wn * wn * dr * dr;
            }
        }
        epot += U[k];
    }
    for (int32_t i = 0; i < N; ++i)
        for (int d = 0; d < 3; ++d) {
            double c = 0.0;
            for (int32_t k = 0; k < P; ++k) c += x[((size_t)k * N + i) * 3 + d];
            c /= (double)P;
            for (int32_t k = 0; k < P; ++k) {
                size_t e = ((size_t)k * N + i) * 3 + d;
                vir += (x[e] - c) * f[e];
            }
        }
    out->ekin = ekin;
    out->espring = espring;
    out->epot = epot;
    out->etot = ekin + espring + epot;
    out->kprim = 1.5 * (double)P * (double)N * kT - espring / (double)P;
    out->kcv = 1.5 * (double)N * kT - vir / (2.0 * (double)P);
    out->temp = 2.0 * ekin / (3.0 * (double)N * (double)P * (double)P * sys->kB);
    /* P_CV = (sum_i m v~0_i^2 - sum_k sum_i (r_i^k - r_i^c) . F_i^k + sum_k Tr Xi^k) / (3 P V)
     * (App. A); the first term with mvv2e, as every kinetic term here */
    out->pcv = out->ppr = out->pmd = 0.0;
    if (sys->pot == ORC_POT_PAIR && sys->box[0] > 0.0) {
        double k0 = 0.0, w = 0.0;
        for (int32_t i = 0; i < N; ++i)
            for (int d = 0; d < 3; ++d) {
                double v = vt[(size_t)i * 3 + d];   /* mode 0 */
                k0 += sys->mass[i] * sys->mvv2e * v * v;
            }
        for (int32_t k = 0; k < P; ++k) w += orc_virial_bead(sys, x + (size_t)k * N * 3);
        const double V = sys->box[0] * sys->box[1] * sys->box[2];
        out->pcv = (k0 - vir + w) / (3.0 * (double)P * V);
        out->ppr = (3.0 * (double)P * (double)N * kT - (2.0 * espring - w) / (double)P) / (3.0 * V);
        out->pmd = (2.0 * ekin + w) / (3.0 * V);
    }
}

double orc_spring_energy_nm(const orc_system *sys, const double *x)
{
    const int32_t P = sys->n_beads, N = sys->n_atoms;
    const size_t n = (size_t)P * N * 3;
    const double wn = omega_n(sys);
    double *lam = (double *)malloc(sizeof(double) * (size_t)P);
    double *xt = (double *)malloc(sizeof(double) * n);
    orc_mode_lambda(P, lam);
    orc_to_normal(P, N, x, xt);
    double s = 0.0;
    for (int32_t k = 0; k < P; ++k)
        for (int32_t i = 0; i < N; ++i)
            for (int d = 0; d < 3; ++d) {
                double q = xt[((size_t)k * N + i) * 3 + d];
                s += 0.5 * sys->mass[i] * sys->mvv2e * wn * wn * lam[k] * q * q;
            }
    free(lam); free(xt);
    return s;
}

double orc_kcv_nm(const orc_system *sys, const double *x, const double *f)
{
    const int32_t P = sys->n_beads, N = sys->n_atoms;
    const size_t n = (size_t)P * N * 3;
    double *xt = (double *)malloc(sizeof(double) * n);
    double *ft = (double *)malloc(sizeof(double) * n);
    orc_to_normal(P, N, x, xt);
    orc_to_normal(P, N, f, ft);
    double vir = 0.0;
    for (int32_t k = 1; k < P; ++k)
        for (size_t e = (size_t)k * N * 3; e < (size_t)(k + 1) * N * 3; ++e) vir += xt[e] * ft[e];
    free(xt); free(ft);
    return 1.5 * (double)N * sys->kB * sys->temp - vir / (2.0 * (double)P);
}

/* ------------------------------------------------------------------------
 * BZP barostat, App. E, isotropic.  An OBABO step (the splitting of the
 * paper's example input) at a synchronized state (forces f of x in box L):
 *   O(dt/2) on the beads (q = 0) and on v_W;
 *   B(dt/2): v_W and v~ kicked together;
 *   A(dt): the centroid mode under the barostat, the other modes by the free
 *          ring-polymer flow (A(dt/2) twice), L <- exp(dt v_W) L;
 *   forces of the new positions in the new box;
 *   B(dt/2); O(dt/2) on v_W and on the beads (q = 1).
 * A BAOAB step: B(dt/2); A(dt/2) with the centroid under the barostat;
 * O(dt) on the beads and on v_W (q = 0); A(dt/2) with the new v_W; forces;
 * B(dt/2).
 * Readings of App. E:
 *  - the barostat's force is (3/W)[P V (P_CV - P_ext) + P kB T]: the printed
 *    1/(n kB T) is read as n kB T, the value for which App. A's enthalpy
 *    H + K_W + U_W + J_W (J_W = -P kB T ln V) is a constant of the NpH motion;
 *  - B is the exact flow of the kick: v~0 moves linearly over the kick, so the
 *    centroid kinetic term integrates to h K + h^2 F~0.v~0 + h^3 |F~0|^2/(3m)
 *    from the momenta at the kick's start, which is what the printed h^2 and
 *    h^3 terms are;
 *  - the scaling acts on the centroid mode only (the one mode that P_CV's
 *    kinetic term and F~0.v~0 see);
 *  - the barostat's thermostat is an O step over dt/2 with c1 = exp(-dt/(2 tau_0))
 *    (tau_0 as printed) and noise sqrt(P kB T / W) z (W for the printed m_i);
 *    z is the first Gaussian of counter (2^64 - 1, 0, s, q).
 * --------------------------------------------------------------------- */
double orc_baro_mass(const orc_system *sys)
{
    return 3.0 * (double)sys->n_beads * (double)sys->n_atoms * sys->kB * sys->temp * sys->tau_p *
           sys->tau_p;
}

double orc_sinhc(double u)
{
    if (fabs(u) < 1e-3) {
        const double u2 = u * u;
        return 1.0 + u2 / 6.0 * (1.0 + u2 / 20.0 * (1.0 + u2 / 42.0));
    }
    return sinh(u) / u;
}

static orc_system orc_in_box(const orc_system *sys, const orc_baro *b)
{
    orc_system s = *sys;
    for (int d = 0; d < 3; ++d) s.box[d] = b->box[d];
    return s;
}

void orc_baro_kick(const orc_system *sys0, orc_baro *b, const double *x, const double *vt,
                   const double *f, double h)
{
    const orc_system sb = orc_in_box(sys0, b);
    const orc_system *sys = &sb;
    const int32_t P = sys->n_beads, N = sys->n_atoms;
    const size_t n = (size_t)P * N * 3;
    const double kT = sys->kB * sys->temp, W = orc_baro_mass(sys);
    const double V = sys->box[0] * sys->box[1] * sys->box[2];
    double *ft = (double *)malloc(sizeof(double) * n);
    orc_to_normal(P, N, f, ft);
    /* centroid sums (mode 0 rows of v~ and f~) */
    double k0 = 0.0, fv = 0.0, f2 = 0.0;
    for (int32_t i = 0; i < N; ++i)
        for (int d = 0; d < 3; ++d) {
            const double v = vt[(size_t)i * 3 + d], F = ft[(size_t)i * 3 + d];
            k0 += sys->mass[i] * sys->mvv2e * v * v;
            fv += F * v;
            f2 += F * F / (sys->mass[i] * sys->mvv2e);
        }
    /* sum_k sum_i (r - r_c) . F and the cell virial */
    double vir = 0.0, w = 0.0;
    for (int32_t i = 0; i < N; ++i)
        for (int d = 0; d < 3; ++d) {
            double c = 0.0;
            for (int32_t k = 0; k < P; ++k) c += x[((size_t)k * N + i) * 3 + d];
            c /= (double)P;
            for (int32_t k = 0; k < P; ++k) {
                const size_t e = ((size_t)k * N + i) * 3 + d;
                vir += (x[e] - c) * f[e];
            }
        }
    if (sys->aniso) {
        /* one v_W per dimension, driven by the diagonal of the centroid-virial
         * stress tensor: P V P_CV^aa = k0_a - vir_a + w_a */
        double k0a[3] = {0.0, 0.0, 0.0}, fva[3] = {0.0, 0.0, 0.0}, f2a[3] = {0.0, 0.0, 0.0};
        double vira[3] = {0.0, 0.0, 0.0}, wa[3] = {0.0, 0.0, 0.0};
        for (int32_t i = 0; i < N; ++i)
            for (int d = 0; d < 3; ++d) {
                const double v = vt[(size_t)i * 3 + d], F = ft[(size_t)i * 3 + d];
                k0a[d] += sys->mass[i] * sys->mvv2e * v * v;
                fva[d] += F * v;
                f2a[d] += F * F / (sys->mass[i] * sys->mvv2e);
                double c = 0.0;
                for (int32_t k = 0; k < P; ++k) c += x[((size_t)k * N + i) * 3 + d];
                c /= (double)P;
                for (int32_t k = 0; k < P; ++k) {
                    const size_t e = ((size_t)k * N + i) * 3 + d;
                    vira[d] += (x[e] - c) * f[e];
                }
            }
        for (int32_t k = 0; k < P; ++k) {
            double wk[3];
            orc_virial_bead_diag(sys, x + (size_t)k * N * 3, wk);
            for (int d = 0; d < 3; ++d) wa[d] += wk[d];
        }
        for (int d = 0; d < 3; ++d)
            b->vwa[d] += h / W * (k0a[d] - vira[d] + wa[d] - (double)P * V * sys->p_ext + (double)P * kT) +
                         h * h / W * fva[d] + h * h * h / (3.0 * W) * f2a[d];
        free(ft);
        return;
    }
    for (int32_t k = 0; k < P; ++k) w += orc_virial_bead(sys, x + (size_t)k * N * 3);
    /* 3 P V P_CV = k0 - vir + w */
    b->vw += h / W * (k0 - vir + w - 3.0 * (double)P * V * sys->p_ext + 3.0 * (double)P * kT) +
             h * h / W * fv + h * h * h / (3.0 * W) * f2;
    free(ft);
}

void orc_baro_centroid_flow(double vw, double t, double *xt0, double *vt0)
{
    const double u = t * vw;
    const double e = exp(u), ei = exp(-u), s = t * orc_sinhc(u);
    *xt0 = e * *xt0 + s * *vt0;
    *vt0 = ei * *vt0;
}

/* v_W's O step over t: dt/2 in OBABO (q = 0, 1), dt in BAOAB (q = 0) */
static void orc_baro_o(const orc_system *sys, orc_baro *b, uint64_t s, uint64_t q)
{
    if (sys->nve) return;
    const double h = sys->integrator == 1 ? 0.5 * sys->dt : sys->dt;
    const double c1 = exp(-h / sys->tau), c2 = sqrt(1.0 - c1 * c1);
    const double sigma = sqrt((double)sys->n_beads * sys->kB * sys->temp / orc_baro_mass(sys));
    double z[3];
    orc_gaussians_q(sys->seed, 0xFFFFFFFFu, 0, s, (uint32_t)q, z);
    if (sys->aniso)
        for (int d = 0; d < 3; ++d) b->vwa[d] = c1 * b->vwa[d] + c2 * sigma * z[d];
    else
        b->vw = c1 * b->vw + c2 * sigma * z[0];
}

/* the centroid modes under the barostat over t, and the box with them */
static void orc_baro_flow_all(const orc_system *sys, orc_baro *b, double t, double *xt, double *vt)
{
    const int32_t N = sys->n_atoms;
    for (int32_t i = 0; i < N; ++i)
        for (int d = 0; d < 3; ++d) {
            const size_t e = (size_t)i * 3 + d;
            orc_baro_centroid_flow(sys->aniso ? b->vwa[d] : b->vw, t, &xt[e], &vt[e]);
        }
    for (int d = 0; d < 3; ++d) b->box[d] *= exp(t * (sys->aniso ? b->vwa[d] : b->vw));
}

void orc_npt_step(const orc_system *sys0, orc_baro *b, double *x, double *vt, double *f,
                  double *U, uint64_t *step, int32_t nsteps)
{
    const int32_t P = sys0->n_beads, N = sys0->n_atoms;
    const size_t n = (size_t)P * N * 3;
    const double h = 0.5 * sys0->dt;
    double *xt = (double *)malloc(sizeof(double) * n);
    double *ft = (double *)malloc(sizeof(double) * n);
    for (int32_t it = 0; it < nsteps; ++it) {
        orc_system sys = orc_in_box(sys0, b);
        const uint64_t s = *step;
        if (sys0->integrator != 1) {
            /* BAOAB: B(dt/2) on v_W and the beads; A(dt/2) with the centroid
             * under the barostat; O(dt) on the beads and on v_W; A(dt/2);
             * forces in the new box; B(dt/2) */
            orc_baro_kick(&sys, b, x, vt, f, h);
            orc_kick(&sys, vt, f, ft);
            orc_to_normal(P, N, x, xt);
            double Ah[4], c1, c2;
            for (int half = 0; half < 2; ++half) {
                for (int32_t k = 1; k < P; ++k) {
                    orc_free_rp_matrix(&sys, k, h, Ah);
                    for (int32_t i = 0; i < N; ++i)
                        for (int d = 0; d < 3; ++d) {
                            const size_t e = ((size_t)k * N + i) * 3 + d;
                            const double q = xt[e], p = vt[e];
                            xt[e] = Ah[0] * q + Ah[1] * p;
                            vt[e] = Ah[2] * q + Ah[3] * p;
                        }
                }
                orc_baro_flow_all(&sys, b, h, xt, vt);
                if (half == 0 && !sys.nve) {
                    /* O(dt) on the beads' modes, then on v_W */
                    for (int32_t k = 0; k < P; ++k) {
                        orc_pile_coeffs(&sys, k, &c1, &c2);
                        for (int32_t i = 0; i < N; ++i) {
                            const double sigma = sqrt((double)P * sys.kB * sys.temp *
                                                      (1.0 / sys.mvv2e) / sys.mass[i]);
                            const uint64_t id = sys.atom_id ? (uint64_t)sys.atom_id[i] : (uint64_t)i;
                            double z[3];
                            orc_gaussians(sys.seed, (uint32_t)id, (uint32_t)k, s, z);
                            for (int d = 0; d < 3; ++d) {
                                const size_t e = ((size_t)k * N + i) * 3 + d;
                                vt[e] = c1 * vt[e] + c2 * sigma * z[d];
                            }
                        }
                    }
                    orc_baro_o(&sys, b, s, 0);
                }
            }
            orc_from_normal(P, N, xt, x);
            *step = s + 1;
            sys = orc_in_box(sys0, b);
            orc_forces(&sys, x, f, U);
            orc_baro_kick(&sys, b, x, vt, f, h);
            orc_kick(&sys, vt, f, ft);
            continue;
        }
        /* O */
        orc_o_step(&sys, vt, s, 0);
        orc_baro_o(&sys, b, s, 0);
        /* B */
        orc_baro_kick(&sys, b, x, vt, f, h);
        orc_kick(&sys, vt, f, ft);
        /* A */
        orc_to_normal(P, N, x, xt);
        double Ah[4];
        for (int32_t k = 1; k < P; ++k) {
            orc_free_rp_matrix(&sys, k, h, Ah);
            for (int32_t i = 0; i < N; ++i)
                for (int d = 0; d < 3; ++d) {
                    const size_t e = ((size_t)k * N + i) * 3 + d;
                    for (int rep = 0; rep < 2; ++rep) {
                        const double q = xt[e], p = vt[e];
                        xt[e] = Ah[0] * q + Ah[1] * p;
                        vt[e] = Ah[2] * q + Ah[3] * p;
                    }
                }
        }
        orc_baro_flow_all(&sys, b, sys.dt, xt, vt);
        orc_from_normal(P, N, xt, x);
        *step = s + 1;
        /* forces in the new box */
        sys = orc_in_box(sys0, b);
        orc_forces(&sys, x, f, U);
        /* B, O */
        orc_baro_kick(&sys, b, x, vt, f, h);
        orc_kick(&sys, vt, f, ft);
        orc_baro_o(&sys, b, s, 1);
        orc_o_step(&sys, vt, s, 1);
    }
    free(xt);
    free(ft);
}

void orc_baro_energies(const orc_system *sys, const orc_baro *b, double etot, double out[5])
{
    const double P = (double)sys->n_beads, kT = sys->kB * sys->temp;
    const double V = b->box[0] * b->box[1] * b->box[2];
    const double kw = sys->aniso ? 0.5 * orc_baro_mass(sys) *
                                       (b->vwa[0] * b->vwa[0] + b->vwa[1] * b->vwa[1] + b->vwa[2] * b->vwa[2])
                                 : 0.5 * orc_baro_mass(sys) * b->vw * b->vw;
    const double uw = P * sys->p_ext * V;
    const double jw = -P * kT * log(V);
    out[0] = V;
    out[1] = kw;
    out[2] = uw;
    out[3] = jw;
    out[4] = etot + kw + uw + jw;
}

/* ------------------------------------------------------------------------
 * Bosonic exchange: the recursion over the cycle containing the last
 * particle, and its gradient by reverse accumulation through the same
 * recursion (each V[n] is a soft minimum of E[n,k] + V[n-k] with weights
 * w[n,k] = exp(-beta_n (E[n,k] + V[n-k] - V[n])) / n summing to one).
 * Plain O(N^3 P): every E[n,k] is summed out, no prefix sums.
 *
 * Extended precision: every energy, V[n], weight, adjoint and probability is
 * held in x87 extended precision (64-bit significand) and rounded to FP64
 * once, at the output.  The exponent of each weight is a difference of
 * quantities of the size of V_B (every E[n,k] + V[n-k] carries all inner
 * ring energies), so FP64 arithmetic would leave a relative error of about
 * beta_n eps V_B in the weights, 1e-12 and more at a few hundred particles.
 * The steps and their order are those of the FP64 recursion.
 * --------------------------------------------------------------------- */
static long double orc_sq3l(const double *a, const double *b)
{
    long double s = 0.0L;
    for (int d = 0; d < 3; ++d) {
        const long double u = (long double)a[d] - (long double)b[d];
        s += u * u;
    }
    return s;
}

/* a - b, under the minimum image in every dimension with box[d] > 0 (box may
 * be NULL: no periodicity); the image is chosen in double precision, like
 * the pair forces' minimum image. */
static void orc_link_vec(const double *a, const double *b, const double *box, long double out[3])
{
    for (int d = 0; d < 3; ++d) {
        double u = a[d] - b[d];
        long double ul = (long double)a[d] - (long double)b[d];
        if (box && box[d] > 0.0) ul -= (long double)box[d] * (long double)nearbyint(u / box[d]);
        out[d] = ul;
    }
}

double orc_boson_spring(int32_t N, int32_t P, double kspring, double beta_n, const double *x,
                        const double *box, double *f, double *prob, double *ev)
{
    /* bead j of particle l (0-based) at x + (j*N + l)*3 */
#define XB(j, l) (x + ((size_t)(j) * N + (l)) * 3)
    typedef long double ld;
    const ld ks = (ld)kspring, bn = (ld)beta_n;
    ld *eint = (ld *)calloc((size_t)N, sizeof(ld));
    ld *link = (ld *)calloc((size_t)N * N, sizeof(ld));   /* [l][l'] */
    ld *E = (ld *)calloc((size_t)(N + 1) * (N + 1), sizeof(ld));   /* E[n][k] */
    ld *V = (ld *)calloc((size_t)(N + 1), sizeof(ld));
    ld *w = (ld *)calloc((size_t)(N + 1) * (N + 1), sizeof(ld));
    ld *adj = (ld *)calloc((size_t)(N + 1), sizeof(ld));
    ld *pl = (ld *)calloc((size_t)N * N, sizeof(ld));
    for (int32_t l = 0; l < N; ++l)
        for (int32_t j = 0; j + 1 < P; ++j) eint[l] += ks * orc_sq3l(XB(j + 1, l), XB(j, l));
    for (int32_t l = 0; l < N; ++l)
        for (int32_t l2 = 0; l2 < N; ++l2) {
            long double dv[3];
            orc_link_vec(XB(0, l2), XB(P - 1, l), box, dv);
            link[(size_t)l * N + l2] = ks * (dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
        }
    /* E[n][k]: ring through particles n-k .. n-1 (0-based), in order, closed
     * from n-1 back to n-k */
    for (int32_t n = 1; n <= N; ++n)
        for (int32_t k = 1; k <= n; ++k) {
            ld e = 0.0L;
            for (int32_t l = n - k; l < n; ++l) e += eint[l];
            for (int32_t l = n - k; l + 1 < n; ++l) e += link[(size_t)l * N + l + 1];
            e += link[(size_t)(n - 1) * N + (n - k)];
            E[(size_t)n * (N + 1) + k] = e;
        }
    V[0] = 0.0L;
    for (int32_t n = 1; n <= N; ++n) {
        ld lo = INFINITY;
        for (int32_t k = 1; k <= n; ++k) {
            const ld a = E[(size_t)n * (N + 1) + k] + V[n - k];
            if (a < lo) lo = a;
        }
        ld s = 0.0L;
        for (int32_t k = 1; k <= n; ++k)
            s += expl(-bn * (E[(size_t)n * (N + 1) + k] + V[n - k] - lo));
        V[n] = lo - logl(s / (ld)n) / bn;
        for (int32_t k = 1; k <= n; ++k)
            w[(size_t)n * (N + 1) + k] =
                expl(-bn * (E[(size_t)n * (N + 1) + k] + V[n - k] - V[n])) / (ld)n;
    }
    /* the weighted ring energy of the primitive estimator */
    if (ev) {
        ld *EV = (ld *)calloc((size_t)(N + 1), sizeof(ld));
        for (int32_t n = 1; n <= N; ++n)
            for (int32_t k = 1; k <= n; ++k)
                EV[n] += w[(size_t)n * (N + 1) + k] * (E[(size_t)n * (N + 1) + k] + EV[n - k]);
        *ev = (double)EV[N];
        free(EV);
    }
    /* adjoints: adj[n] = dV[N]/dV[n]; dV[N]/dE[n][k] = adj[n] w[n][k] */
    adj[N] = 1.0L;
    for (int32_t n = N; n >= 1; --n)
        for (int32_t k = 1; k <= n; ++k) adj[n - k] += adj[n] * w[(size_t)n * (N + 1) + k];
    /* link probabilities: the weight every E[n][k] gives each of its links */
    for (int32_t n = 1; n <= N; ++n)
        for (int32_t k = 1; k <= n; ++k) {
            const ld q = adj[n] * w[(size_t)n * (N + 1) + k];
            for (int32_t l = n - k; l + 1 < n; ++l) pl[(size_t)l * N + l + 1] += q;
            pl[(size_t)(n - 1) * N + (n - k)] += q;
        }
    if (prob)
        for (size_t e = 0; e < (size_t)N * N; ++e) prob[e] = (double)pl[e];
    if (f) {
        ld *fl = (ld *)calloc((size_t)P * N * 3, sizeof(ld));
        /* springs inside every ring: weight one (each particle lies on one cycle) */
        for (int32_t l = 0; l < N; ++l)
            for (int32_t j = 0; j + 1 < P; ++j)
                for (int d = 0; d < 3; ++d) {
                    const ld g = 2.0L * ks * ((ld)XB(j + 1, l)[d] - (ld)XB(j, l)[d]);
                    fl[((size_t)(j + 1) * N + l) * 3 + d] -= g;
                    fl[((size_t)j * N + l) * 3 + d] += g;
                }
        /* links, weighted by their probabilities */
        for (int32_t l = 0; l < N; ++l)
            for (int32_t l2 = 0; l2 < N; ++l2) {
                const ld q = pl[(size_t)l * N + l2];
                if (q == 0.0L) continue;
                long double dv[3];
                orc_link_vec(XB(0, l2), XB(P - 1, l), box, dv);
                for (int d = 0; d < 3; ++d) {
                    const ld g = 2.0L * ks * q * dv[d];
                    fl[((size_t)0 * N + l2) * 3 + d] -= g;
                    fl[((size_t)(P - 1) * N + l) * 3 + d] += g;
                }
            }
        for (size_t e = 0; e < (size_t)P * N * 3; ++e) f[e] = (double)fl[e];
        free(fl);
    }
    const double vb = (double)V[N];
    free(eint); free(link); free(E); free(V); free(w); free(adj); free(pl);
#undef XB
    return vb;
}

/* ------------------------------------------------------------------------
 * The bosonic step in Cartesian coordinates (see the header).
 * --------------------------------------------------------------------- */
double orc_boson_forces(const orc_system *sys, const double *x, double *f, double *U)
{
    const int32_t P = sys->n_beads, N = sys->n_atoms;
    const size_t n = (size_t)P * N * 3;
    const double kT = sys->kB * sys->temp;
    const double wn = omega_n(sys);
    const double ks = 0.5 * sys->mass[0] * sys->mvv2e * wn * wn;
    double *fs = (double *)malloc(sizeof(double) * n);
    orc_forces(sys, x, f, U);
    const double vb = orc_boson_spring(N, P, ks, 1.0 / ((double)P * kT), x, sys->box, fs, NULL, NULL);
    for (size_t e = 0; e < n; ++e) f[e] += fs[e];
    free(fs);
    return vb;
}

void orc_boson_step(const orc_system *sys, double *x, double *v, double *f, double *U, double *vb,
                    uint64_t *step, int32_t nsteps)
{
    const int32_t P = sys->n_beads, N = sys->n_atoms;
    const double h = 0.5 * sys->dt;
    const double kT = sys->kB * sys->temp;
    const int obabo = sys->integrator == 1;
    /* each O step lasts dt (BAOAB) or dt/2 (OBABO) */
    const double to = obabo ? 0.5 * sys->dt : sys->dt;
    const double c1 = sys->nve ? 1.0 : exp(-to / sys->tau), c2 = sqrt(1.0 - c1 * c1);
    /* O acts on every bead velocity with the noise of counter (atom, bead, s, q) */
    for (int32_t it = 0; it < nsteps; ++it) {
        const uint64_t s = *step;
        for (int32_t j = 0; j < P; ++j)
            for (int32_t i = 0; i < N; ++i) {
                const double im = 1.0 / (sys->mass[i] * sys->mvv2e);
                const double sigma = sqrt((double)P * kT * im);
                const uint64_t id = sys->atom_id ? (uint64_t)sys->atom_id[i] : (uint64_t)i;
                double z[3] = {0.0, 0.0, 0.0};
                if (!sys->nve) orc_gaussians_q(sys->seed, (uint32_t)id, (uint32_t)j, s, 0, z);
                for (int d = 0; d < 3; ++d) {
                    const size_t e = ((size_t)j * N + i) * 3 + d;
                    if (obabo) {
                        v[e] = c1 * v[e] + c2 * sigma * z[d];  /* O(dt/2) */
                        v[e] += h * f[e] * im;                 /* B */
                        x[e] += h * v[e];                      /* A(dt) as A(dt/2) twice */
                        x[e] += h * v[e];
                    } else {
                        v[e] += h * f[e] * im;                 /* B */
                        x[e] += h * v[e];                      /* A */
                        v[e] = c1 * v[e] + c2 * sigma * z[d];  /* O */
                        x[e] += h * v[e];                      /* A */
                    }
                }
            }
        *vb = orc_boson_forces(sys, x, f, U);
        for (int32_t j = 0; j < P; ++j)
            for (int32_t i = 0; i < N; ++i) {
                const double im = 1.0 / (sys->mass[i] * sys->mvv2e);
                const double sigma = sqrt((double)P * kT * im);
                const uint64_t id = sys->atom_id ? (uint64_t)sys->atom_id[i] : (uint64_t)i;
                double z[3] = {0.0, 0.0, 0.0};
                if (obabo && !sys->nve) orc_gaussians_q(sys->seed, (uint32_t)id, (uint32_t)j, s, 1, z);
                for (int d = 0; d < 3; ++d) {
                    const size_t e = ((size_t)j * N + i) * 3 + d;
                    v[e] += h * f[e] * im;                 /* B */
                    if (obabo) v[e] = c1 * v[e] + c2 * sigma * z[d];  /* O(dt/2) */
                }
            }
        *step = s + 1;
    }
}

void orc_boson_estimators(const orc_system *sys, const double *x, const double *v, orc_est *out)
{
    const int32_t P = sys->n_beads, N = sys->n_atoms;
    const size_t n = (size_t)P * N * 3;
    const double kT = sys->kB * sys->temp;
    const double wn = omega_n(sys);
    const double ks = 0.5 * sys->mass[0] * sys->mvv2e * wn * wn;
    double *fp = (double *)malloc(sizeof(double) * n);
    double *U = (double *)malloc(sizeof(double) * (size_t)P);
    orc_forces(sys, x, fp, U);
    double ev = 0.0;
    const double vb = orc_boson_spring(N, P, ks, 1.0 / ((double)P * kT), x, sys->box, NULL, NULL, &ev);
    double ekin = 0.0, u = 0.0, rf = 0.0;
    for (int32_t j = 0; j < P; ++j)
        for (int32_t i = 0; i < N; ++i)
            for (int d = 0; d < 3; ++d) {
                const size_t e = ((size_t)j * N + i) * 3 + d;
                ekin += 0.5 * sys->mass[i] * sys->mvv2e * v[e] * v[e];
                rf += x[e] * fp[e];
            }
    for (int32_t j = 0; j < P; ++j) u += U[j];
    memset(out, 0, sizeof(*out));
    out->ekin = ekin;
    out->espring = vb;
    out->epot = u;
    out->etot = ekin + vb + u;
    out->kprim = 1.5 * (double)P * (double)N * kT - ev / (double)P;
    out->kcv = -rf / (2.0 * (double)P);
    out->temp = 2.0 * ekin / (3.0 * (double)N * (double)P * (double)P * sys->kB);
    free(fp);
    free(U);
}