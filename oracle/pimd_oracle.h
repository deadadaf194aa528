/*
 * pimd_oracle.h -- plain CPU FP64 reference ("oracle") for the ring-polymer
 * BAOAB step with the PILE-L Langevin thermostat, as described in
 * Li et al., "fix pimd/langevin: An Efficient Implementation of Path Integral
 * Molecular Dynamics in LAMMPS" (arXiv:2602.13553).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The GPU library shares
 * no code, header, table or helper with it.
 *
 * Everything is FP64, written for clarity and checked against the physics
 * (orthogonality, energy conservation, closed forms), not for speed.
 *
 * Layout: every per-bead array is [P][N][3] (bead k, atom i, Cartesian dim a),
 * i.e. element r_i^(k)_a lives at ((k*N)+i)*3+a.  Velocities in the state are
 * normal-mode velocities v~ (the paper keeps positions Cartesian and
 * velocities in normal-mode form, Sec. III.A).
 *
 * Units: the caller chooses a consistent unit system.  kB*temp is an energy,
 * hbar is energy*time, and mvv2e converts mass*velocity^2 to energy (1 in
 * reduced LJ units; 1/4.184e-4 for amu, Angstrom, fs, kcal/mol).
 *
 * Parity pins: see the per-function comments; every function here is pinned
 * by a test against a closed form, an invariant, a library routine or brute
 * force, except where a comment says "parity unpinned".
 */
#ifndef PIMD_ORACLE_H
#define PIMD_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_POT_NONE = 0, ORC_POT_HARMONIC = 1, ORC_POT_PAIR = 2 };

typedef struct orc_system {
    int32_t n_atoms;        /* N */
    int32_t n_beads;        /* P (the paper's n) */
    int32_t nve;            /* 1: no thermostat (c1 = 1, c2 = 0) */
    int32_t pot;            /* ORC_POT_* */
    double temp;            /* T */
    double kB;              /* Boltzmann constant, energy per temperature */
    double hbar;            /* reduced Planck constant (already scaled by sp) */
    double mvv2e;           /* energy = mvv2e * mass * velocity^2 */
    double dt;              /* time step */
    double tau;             /* centroid damping time tau_0 */
    double tau_scale;       /* multiplies the non-centroid damping times */
    double box[3];          /* periodic box lengths (pair potentials only) */
    uint64_t seed;          /* thermostat seed */
    double omega;           /* harmonic trap frequency (ORC_POT_HARMONIC) */
    double lj_eps, lj_sigma, lj_rc;   /* Lennard-Jones among lj_active atoms */
    double bond_k, bond_r0;           /* U = bond_k (r - r0)^2 per bond */
    const double *mass;     /* [N] */
    const int32_t *lj_active; /* [N] 0/1, or NULL = every atom */
    int32_t n_bonds;
    const int32_t *bonds;   /* [n_bonds][2] atom pairs */
    const int64_t *atom_id; /* [N] each atom's index in the noise counter, or NULL = its
                               position; lets a sample of a system of independent atoms
                               (trap, free) be stepped alone with its original noise */
    int32_t integrator;     /* 0: BAOAB; 1: OBABO (O(dt/2) B(dt/2) A(dt) B(dt/2) O(dt/2)) */
    int32_t fixcom;         /* 1: remove the centroids' center-of-mass velocity at the end
                               of every step */
    int32_t npt;            /* 1: isotropic BZP barostat (App. E) with either splitting; with
                               nve = 1 the barostat's thermostat is off too (NpH) */
    double p_ext;           /* target pressure (energy per volume) */
    double tau_p;           /* barostat time: W = 3 P N kB T tau_p^2 */
    int32_t aniso;          /* 1: anisotropic barostat (one v_W per dimension, App. E) */
} orc_system;

typedef struct orc_est {
    double ekin;    /* sum_k K^(k), App. A item 1 (normal-mode form) */
    double espring; /* sum_k S^(k), Eq. 1 spring term (read with omega_n^2) */
    double epot;    /* sum_k U^(k), App. A item 3 */
    double etot;    /* H, Eq. A4 */
    double kprim;   /* K_PR, Eq. A5 (read with 1/n and omega_n^2) */
    double kcv;     /* K_CV, Eq. A7 */
    double temp;    /* ring-polymer temperature divided by P (Sec. III.A) */
    double pcv;     /* P_CV, App. A (centroid-virial pressure); 0 without a periodic box */
    double ppr;     /* P_PR, App. A (primitive pressure, read with the virial and 1/P); 0 likewise */
    double pmd;     /* P_MD, App. A (pressure of the extended classical system); 0 likewise */
} orc_est;

/* --- normal modes (App. B) --------------------------------------------- */
void orc_nm_matrix(int32_t P, double *M /* [P][P], row = mode */);
void orc_mode_lambda(int32_t P, double *lam /* [P] */);
/* a~ = M a for every atom and dim; a, at are [P][N][3].  M and the dot
 * products are evaluated in extended precision and rounded once. */
void orc_to_normal(int32_t P, int32_t N, const double *a, double *at);
/* a = M^T a~ */
void orc_from_normal(int32_t P, int32_t N, const double *at, double *a);

/* --- random numbers (App. D noise) ------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* three standard normal deviates for key seed and counter (i, k, s, 0) */
void orc_gaussians(uint64_t seed, uint32_t i, uint32_t k, uint64_t s, double z[3]);
/* The same for O step q of step s (0, or 1 for OBABO's second O). */
void orc_gaussians_q(uint64_t seed, uint32_t i, uint32_t k, uint64_t s, uint32_t q, double z[3]);

/* --- free ring-polymer propagator and thermostat coefficients ---------- */
/* A(h) for mode k: [[a00, a01], [a10, a11]] acting on (x~, v~) */
void orc_free_rp_matrix(const orc_system *sys, int32_t k, double h, double A[4]);
void orc_pile_coeffs(const orc_system *sys, int32_t k, double *c1, double *c2);

/* --- forces, per bead independently ----------------------------------- */
/* x, f: [N][3] of one bead; returns U^(k) */
double orc_forces_bead(const orc_system *sys, const double *xk, double *fk);
/* The cell virial Tr Xi of one bead (App. A, under the primitive pressure
 * estimator): minus the derivative of U under a uniform scaling of the
 * positions and the box, i.e. the sum of r_ij . F_ij over interacting pairs
 * (every image) and bonds.  0 without a periodic box. */
double orc_virial_bead(const orc_system *sys, const double *xk);
/* The diagonal Xi_aa of one bead's cell virial tensor: minus the derivative
 * of U under the scaling of the a-components of the positions and of L_a
 * alone, i.e. the sum of (r_ij)_a (F_ij)_a over interacting pairs (every
 * image) and bonds.  Zeros without a periodic box. */
void orc_virial_bead_diag(const orc_system *sys, const double *xk, double w[3]);
/* x, f: [P][N][3]; U: [P] */
void orc_forces(const orc_system *sys, const double *x, double *f, double *U);

/* --- the integrator ---------------------------------------------------- */
/* Advances (x, v~, f) by nsteps BAOAB steps.  step is the thermostat step
 * counter s used in the noise counter; it is incremented once per step. */
void orc_step(const orc_system *sys, double *x, double *vt, double *f, double *U,
              uint64_t *step, int32_t nsteps);
/* The two parts of orc_step around the force call, for forces supplied by
 * the caller: B A O A to the new positions (advancing the step counter),
 * then the closing B with the new positions' forces. */
void orc_step_positions(const orc_system *sys, double *x, double *vt, const double *f,
                        uint64_t *step);
void orc_step_kick(const orc_system *sys, double *vt, const double *f, uint64_t s);

/* --- BZP barostat (App. E, isotropic) ---------------------------------- */
typedef struct orc_baro {
    double vw;              /* barostat velocity v_W (isotropic) */
    double box[3];          /* current box lengths */
    double vwa[3];          /* the per-dimension velocities v_Wx, v_Wy, v_Wz (anisotropic) */
} orc_baro;
/* W = 3 P N kB T tau_p^2 (App. A) */
double orc_baro_mass(const orc_system *sys);
/* sinh(u)/u, by its Taylor series for |u| < 1e-3 */
double orc_sinhc(double u);
/* The barostat's share of a kick of length h: v_W advances along the exact
 * flow of the kick (forces, positions and box fixed, v~ += h f~/m), from the
 * momenta at the start of the kick.  vt and f as for orc_step. */
void orc_baro_kick(const orc_system *sys, orc_baro *b, const double *x, const double *vt,
                   const double *f, double h);
/* The centroid mode's flow under the barostat over a time t (App. E):
 * (x~0, v~0) -> (e x~0 + t sinhc(t v_W) v~0, v~0 / e), e = exp(t v_W). */
void orc_baro_centroid_flow(double vw, double t, double *xt0, double *vt0);
/* nsteps NpT (or NpH) steps: O, B, A, forces, B, O with the barostat; the box
 * in b moves with the centroids, and f, U are those of the new box. */
void orc_npt_step(const orc_system *sys, orc_baro *b, double *x, double *vt, double *f,
                  double *U, uint64_t *step, int32_t nsteps);
/* Barostat terms of App. A at box b: out = {V, K_W, U_W, J_W, enthalpy}, the
 * enthalpy H + K_W + U_W + J_W with H = etot. */
void orc_baro_energies(const orc_system *sys, const orc_baro *b, double etot, double out[5]);

/* --- bosonic exchange (Sec. III.C's fix pimd/langevin/bosonic; the
 * exchange potential of Hirshberg et al. 2019 as evaluated in quadratic time by
 * Feldman and Hirshberg 2023, both cited by the paper) ----------------------
 * N identical particles of one mass, P beads, Cartesian positions x [P][N][3]
 * (no box).  The springs inside each particle's ring (beads 0..P-1) are the
 * distinguishable ones; the link from bead P-1 of one particle to bead 0 of
 * the next is summed over permutations:
 *   exp(-beta_n V_B) = (1/N!) sum_sigma exp(-beta_n E_sigma),
 * E_sigma = sum_l E_int(l) + sum_l link(l, sigma(l)), with
 * link(l, l') = kspring |x_l'^0 - x_l^(P-1)|^2 and kspring = m omega_n^2 / 2.
 * box (may be NULL; [3], 0 = not periodic in that dimension): each link's
 * vector is taken under the minimum image (the springs inside a particle's
 * ring use its unwrapped coordinates).
 * The recursion over cycles: V[0] = 0,
 *   exp(-beta_n V[n]) = (1/n) sum_{k=1..n} exp(-beta_n (E[n,k] + V[n-k])),
 * E[n,k] the energy of the single ring through particles n-k+1..n (1-based).
 * Returns V_B = V[N]; f (may be NULL) receives -dV_B/dx for every bead; prob
 * (may be NULL, [N][N]) the probability that bead P-1 of particle l links to
 * bead 0 of particle l'; ev (may be NULL) the ring energy averaged over the
 * recursion's terms with their weights,
 *   EV[0] = 0,  EV[n] = sum_{k=1..n} w[n,k] (E[n,k] + EV[n-k]),  *ev = EV[N],
 * w[n,k] = exp(-beta_n (E[n,k] + V[n-k] - V[n])) / n: the spring energy that
 * the bosonic primitive kinetic energy estimator (App. A's bosonic list, item
 * 5) subtracts, K_PR = 3 P N kB T / 2 - EV[N] / P (with the 1/P of the
 * distinguishable K_PR; EV[N] = d(beta_n V_B)/d(beta_n) at fixed positions). */
double orc_boson_spring(int32_t N, int32_t P, double kspring, double beta_n, const double *x,
                        const double *box, double *f, double *prob, double *ev);
/* The bosonic fix's step (Sec. III.C: Cartesian coordinates, since the normal
 * modes change under exchange; the thermostat of Eq. D3) in Cartesian bead
 * velocities v [P][N][3], with the forces of the potential plus the exchange
 * springs' (orc_boson_spring, kspring = m mvv2e omega_n^2 / 2, beta_n =
 * 1/(P kB T), masses all equal to mass[0], links under the minimum image of
 * sys->box).  BAOAB (integrator 0): B(dt/2); A(dt/2) drift; O(dt)
 * v <- c1 v + c2 sigma z with c1 = exp(-dt/tau) for every bead, sigma =
 * sqrt(P kB T / (m mvv2e)), z from counter (atom, bead, step, 0); A(dt/2);
 * forces; B(dt/2).  OBABO (integrator 1): O(dt/2) (c1 = exp(-dt/(2 tau)),
 * counter (atom, bead, step, 0)); B(dt/2); A(dt) as two drifts of dt/2;
 * forces; B(dt/2); O(dt/2) (counter (atom, bead, step, 1)).  f holds the
 * total forces of x, U the beads' potential energies, *vb the exchange spring
 * energy; all are those of the new x. */
void orc_boson_step(const orc_system *sys, double *x, double *v, double *f, double *U, double *vb,
                    uint64_t *step, int32_t nsteps);
/* Total forces (potential + exchange springs), U per bead, returns V_B. */
double orc_boson_forces(const orc_system *sys, const double *x, double *f, double *U);
/* The bosonic fix's outputs (App. A's bosonic list) at a synchronized state
 * x, v (Cartesian bead velocities): ekin = sum_k K^(k) (item 1, Cartesian);
 * espring = V_B, the exchange spring energy: bead 0 carries the links summed
 * over exchange cycles and beads 1..P-1 their springs inside the rings
 * (item 2), so sum_k S^(k) = V_B; epot = sum_k U^(k) (item 3); etot = H
 * (item 4); kprim = 3 P N kB T / 2 - EV_B / P, the bosonic primitive
 * estimator (item 5), EV_B from orc_boson_spring; kcv holds the virial
 * estimator K_VR = -(1/2P) sum_k sum_i r_i^k . F_i^k (item 6) with the
 * potential's forces alone; temp as for distinguishable particles; the
 * pressures are 0. */
void orc_boson_estimators(const orc_system *sys, const double *x, const double *v, orc_est *out);

/* --- estimators (App. A) ----------------------------------------------- */
/* At a synchronized state.  U is [P] from orc_forces. */
void orc_estimators(const orc_system *sys, const double *x, const double *vt,
                    const double *f, const double *U, orc_est *out);
/* Spring energy in the normal-mode form of App. A item 2 (for the pin that
 * it equals the bead form of Eq. 1). */
double orc_spring_energy_nm(const orc_system *sys, const double *x);
/* K_CV written through normal modes: 3NkT/2 - (1/2P) sum_{k>=1} x~.f~ */
double orc_kcv_nm(const orc_system *sys, const double *x, const double *f);

#ifdef __cplusplus
}
#endif
#endif
