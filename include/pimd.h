/*
 * pimd.h -- C ABI of libpimd.so: the ring-polymer BAOAB (or OBABO) step with
 * the PILE-L Langevin thermostat on one MI355X (gfx950), all P beads of all N
 * atoms resident in HBM.
 *
 * Method: Li et al., "fix pimd/langevin: An Efficient Implementation of Path
 * Integral Molecular Dynamics in LAMMPS", arXiv:2602.13553.
 *   - ring-polymer Hamiltonian and spring frequency: Sec. II, Eqs. 1-2
 *   - normal-mode transform and its inverse: App. B, Eqs. B1-B3
 *   - BAOAB splitting in normal modes, thermostat at P*T: Sec. III.C, IV.A
 *     (OBABO, the splitting of the paper's example input: Sec. III.C)
 *   - PILE-L O step and damping times: App. D, Eqs. D1-D2
 *   - unwrapped coordinates for transforms and estimators: Sec. IV.B
 *   - estimators K, S, U, H, K_PR, K_CV: App. A, Eqs. A4, A5, A7; the
 *     pressures P_CV, P_PR, P_MD and the barostat's enthalpy: App. A
 *   - BZP barostat, isotropic or anisotropic (NpT, NpH): Sec. IV.A, App. E
 *
 * Conventions for every entry point:
 *   - Return 0 (PIMD_OK) or a negative PIMD_ERR_* code.  On error, out
 *     parameters are left untouched and pimd_last_error() describes it.  No
 *     C++ exception crosses this boundary.
 *   - Host pointers are borrowed for the duration of the call only
 *     (copy-in / copy-out).  Only pimd_get_positions and pimd_set_forces
 *     take device pointers.  Device state is owned by the context, or lives
 *     in a caller-provided device workspace (see pimd_create).
 *   - A context is used by one host thread at a time.
 *   - Host-side bead arrays use the layout [P][N][3] (bead k, atom i,
 *     Cartesian dim), FP64, atoms in the caller's order.  The device layout
 *     is private to the library.
 *   - Units are the caller's: kB*temp is an energy, hbar an energy*time, and
 *     mvv2e converts mass*velocity^2 to energy (1 in reduced LJ units,
 *     2390.0573... for amu, Angstrom, fs and kcal/mol).
 */
#ifndef PIMD_H
#define PIMD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PIMD_OK 0
#define PIMD_ERR_ARG (-1)         /* invalid argument or parameter */
#define PIMD_ERR_OOM (-2)         /* device allocation failed / workspace too small */
#define PIMD_ERR_DEVICE (-3)      /* HIP runtime error */
#define PIMD_ERR_STATE (-4)       /* call out of order (e.g. step before set_state) */
#define PIMD_ERR_NONFINITE (-5)   /* a position or velocity became NaN/Inf */
#define PIMD_ERR_UNSUPPORTED (-6) /* valid but not supported by the library */
#define PIMD_ERR_OVERFLOW (-7)    /* neighbor-list capacity exceeded */

/* ensemble (Sec. III.C): NVT = PILE-L thermostat at P*T, NVE = no thermostat;
 * NPT = PILE-L and the BZP barostat (Sec. IV.A, App. E) with a
 * thermostat on its velocity, NPH = the barostat with neither thermostat.
 * NPT and NPH need PIMD_POT_LJ or PIMD_POT_WATER and fixcom = 0; they are not
 * batched. */
#define PIMD_NVT 0
#define PIMD_NVE 1
#define PIMD_NPT 2
#define PIMD_NPH 3

/* potential U of one bead (the U(r^(k)) term of Eq. 1); every bead is an
 * independent copy of the physical system */
#define PIMD_POT_NONE 0      /* U = 0: free ring polymers */
#define PIMD_POT_HARMONIC 1  /* U = sum_i 1/2 m_i omega^2 |r_i|^2 (trap at the origin) */
#define PIMD_POT_LJ 2        /* 12-6 Lennard-Jones among all atoms, periodic box */
#define PIMD_POT_WATER 3     /* LJ among topology-active atoms + harmonic bonds */
#define PIMD_POT_EXTERNAL 4  /* forces from the caller (pimd_set_forces), e.g. a machine-learned
                                potential evaluated on each bead (Sec. II: the force on bead k is
                                minus the gradient of U at replica k; Sec. IV.A: one force call
                                per replica per step) */

typedef struct pimd_params {
    int32_t n_atoms;    /* N >= 1 */
    int32_t n_beads;    /* P >= 1 (the paper's n); the library supports P <= 128 */
    int32_t ensemble;   /* PIMD_NVT, PIMD_NVE, PIMD_NPT or PIMD_NPH */
    int32_t potential;  /* PIMD_POT_* */
    double temp;        /* T > 0; the thermostat acts at P*T (Sec. IV.A) */
    double kB;          /* Boltzmann constant (energy per temperature) > 0 */
    double hbar;        /* reduced Planck constant, already scaled by sp (Sec. III.C) > 0 */
    double mvv2e;       /* energy per mass*velocity^2 > 0 */
    double dt;          /* time step > 0 */
    double tau;         /* centroid damping time tau_0 (> 0 for NVT) */
    double tau_scale;   /* scale on tau_k = 1/(2 omega_k), k >= 1 (Eq. D1) (> 0 for NVT) */
    double box[3];      /* periodic box lengths; required (> 0) for LJ and WATER */
    uint64_t seed;      /* thermostat seed */
    double omega;       /* trap frequency (HARMONIC) */
    double lj_eps;      /* LJ epsilon */
    double lj_sigma;    /* LJ sigma > 0 */
    double lj_rc;       /* LJ cutoff > 0; energy shifted to 0 at rc, force not shifted */
    double skin;        /* neighbor-list skin >= 0 (LJ, WATER) */
    double bond_k;      /* bond U = bond_k (r - bond_r0)^2 (WATER) */
    double bond_r0;
    int32_t nbr_capacity; /* neighbors per atom; 0 = sized from the density */
    int32_t flags;        /* PIMD_FLAG_* (0 = defaults) */
    int32_t integrator;   /* PIMD_BAOAB (0) or PIMD_OBABO (1) */
    int32_t fixcom;       /* 1: remove the centroids' center-of-mass velocity at the end
                             of every step (Sec. III.C's fixcom keyword); not in a batch */
    double p_ext;         /* NPT, NPH: target pressure, energy per volume (finite); the
                             default neighbor capacity allows twice the starting density
                             (set nbr_capacity for more) */
    double tau_p;         /* NPT, NPH: barostat time > 0; mass W = 3 P N kB T tau_p^2 */
    int32_t bosonic;      /* 1: identical bosons with exchange (the bosonic fix; see below) */
    int32_t baro_aniso;   /* NPT, NPH: 1 = anisotropic barostat (one v_W per dimension;
                             see below), 0 = isotropic; must be 0 otherwise */
} pimd_params;

/* bosonic = 1: the bosonic fix of Sec. III.C.  The N atoms are identical
 * bosons (all masses equal), integrated in Cartesian coordinates (the normal
 * modes change under exchange): bead velocities v (Cartesian), forces of the
 * potential plus the springs, the springs inside each particle's ring and
 * the links from bead P-1 of one particle to bead 0 of another summed over
 * exchange cycles (the potential of pimd_boson_spring; links under the
 * minimum image of params.box where box > 0).  The step is BAOAB (B(dt/2)
 * A(dt/2) O(dt) A(dt/2) B(dt/2)) or OBABO (O(dt/2) B(dt/2) A(dt) B(dt/2)
 * O(dt/2), A(dt) as two drifts of dt/2), each O the Cartesian PILE of App. D
 * on every bead velocity: v <- c1 v + c2 sqrt(P kB T / (m mvv2e)) z,
 * c1 = exp(-t/tau) over the O step's length t, one damping time tau for all
 * beads (App. D's default for Cartesian coordinates is tau = 1/(2 omega_n),
 * omega_n = P kB T / hbar; tau_scale is unused), z of counter (atom, bead,
 * step, q) with q as for distinguishable particles.  Ensembles NVT and NVE;
 * potentials NONE, HARMONIC, LJ and EXTERNAL; N <= 1024; no fixcom, no
 * barostat, not in a batch.  The estimators become App. A's bosonic outputs:
 * espring = V_B (bead 0's exchange links plus the springs inside the rings),
 * kprim the bosonic primitive estimator 3 P N kB T / 2 - EV_B / P (EV_B as in
 * pimd_boson_spring), and the kcv slot holds the virial estimator K_VR =
 * -(1/2P) sum_k sum_i r_i^k . F_i^k with the potential's forces; the
 * pressures are 0.  pimd_get_state returns the Cartesian momenta m v. */

/* The barostat (NPT, NPH; App. E).  An OBABO step: O(dt/2) on the
 * beads and on v_W; B(dt/2) on v_W and the beads together; A(dt) with the
 * centroid modes under the barostat, x~0 <- e x~0 + t sinh(u)/u v~0,
 * v~0 <- v~0 / e (t = dt, u = t v_W, e = exp(u)), the other modes by the free
 * flow, and the box L <- e L; the forces in the new box; B(dt/2); O(dt/2) on
 * v_W and the beads.  A BAOAB step: B(dt/2); A(dt/2) as above with t = dt/2;
 * O(dt) on the beads and on v_W; A(dt/2) with the new v_W; forces; B(dt/2).
 * v_W's force is (3/W)[P V (P_CV - p_ext) + P kB T] (the value for which the
 * enthalpy H + K_W + U_W + J_W of App. A is conserved in NPH; J_W =
 * -P kB T ln V); its kick integrates the centroid kinetic term along the
 * beads' kick (App. E's h^2 and h^3 terms, from the momenta at the kick's
 * start).  Its O step: v_W <- c1 v_W + c2 sqrt(P kB T / W) z, c1 =
 * exp(-t/tau) over the O step's length t, z the first Gaussian of counter
 * (2^64 - 1, 0, step, q) (q as for the beads' O steps).
 * pimd_set_state starts the box at params.box with v_W = 0, or at the values
 * given to pimd_set_barostat before it (a restart). */

/* baro_aniso = 1: App. E's anisotropic barostat.  Each dimension a has its
 * own v_Wa (same mass W), moves the centroid modes' component a and the box
 * length L_a alone (u = t v_Wa in the flow above, L_a <- exp(t v_Wa) L_a),
 * and is driven by that dimension's diagonal element of the centroid-virial
 * stress tensor: force (1/W)[P V (P_CV^aa - p_ext) + P kB T], with
 * P V P_CV^aa = sum_i m_i |v~0_ia|^2 - sum_k sum_i (x_ia^k - c_ia) F_ia^k +
 * sum_k W_aa^k (W_aa^k bead k's pair virial along a), and the kick's h^2 and
 * h^3 terms from that dimension's sums.  Its O step uses the three Gaussians
 * of v_W's counter, one per dimension.  The box keeps no aspect ratio; the
 * neighbor lists are rebuilt against the smallest scaling of any dimension;
 * K_W = W sum_a v_Wa^2 / 2. */

/* fixcom = 1: at the end of every step (after the closing B, and OBABO's
 * second O) the mass-weighted mean u = sum_i m_i v~0_i / sum_i m_i of the
 * centroid-mode velocities is subtracted from every atom's centroid mode, i.e.
 * the centroids' center-of-mass velocity u / sqrt(P) is removed from every
 * bead; the estimators are those of the state after the removal.  With the
 * pair potentials the closing half-kick then runs in a pass of its own
 * before each step. */

/* integrator: the Trotter splitting of one step (Sec. III.C; the paper's
 * example input uses OBABO).
 *   PIMD_BAOAB  B(dt/2) A(dt/2) O(dt) A(dt/2) B(dt/2); one noise draw per step,
 *               counter (atom, mode, step, 0)
 *   PIMD_OBABO  O(dt/2) B(dt/2) A(dt) B(dt/2) O(dt/2); A(dt) is A(dt/2) twice;
 *               the two half-step O use counters (atom, mode, step, 0) and
 *               (atom, mode, step, 1), with c1 = exp(-dt/(2 tau_k))
 * In both the estimators are taken at the end of the step. */
#define PIMD_BAOAB 0
#define PIMD_OBABO 1

/* flags.  By default the launch shapes come from the library's tuning table
 * (measured on MI355X by paper_2602_13553_amd/autotune.py): the step pass
 * runs its normal-mode transforms on the FP64 matrix cores (MFMA) for
 * P = 16, 32, 64 once N*P reaches the tuned size for that P, and on the FP64
 * vector ALUs otherwise; the force pass shares each atom's list among the
 * tuned number of lane sub-groups.  The flags override the table:
 *   PIMD_FLAG_VALU_TRANSFORMS   vector-ALU transforms at every size
 *   PIMD_FLAG_MFMA_TRANSFORMS   matrix-core transforms wherever P allows
 *                               (with both set, VALU wins)
 *   PIMD_PAIR_SUBGROUPS(S)      S = 1, 2, 4, 8 or 16 sub-groups of P lanes
 *                               per atom in the force pass (S*P <= 256)
 *   PIMD_FLAG_CLUSTER_PAIRS     force pass on cluster lists: the 256/P
 *                               consecutive atoms of a block share one list,
 *                               and each neighbor's bead rows are staged once
 *                               per block (P >= 8; blocks whose cluster is too
 *                               wide for the box fall back to per-atom lists)
 *   PIMD_FLAG_ATOM_PAIRS        force pass on per-atom lists only
 *   PIMD_FLAG_NO_GRAPHS         pimd_step launches every step's kernels one
 *                               by one instead of replaying a captured
 *                               hipGraph (for callers that capture the stream
 *                               themselves); this is also the path a context
 *                               takes when the capture fails
 * Results do not depend on the launch shape beyond the rounding of the
 * transforms (MFMA and VALU sum in different orders). */
#define PIMD_FLAG_VALU_TRANSFORMS 1
#define PIMD_FLAG_MFMA_TRANSFORMS 2
#define PIMD_FLAG_CLUSTER_PAIRS 4
#define PIMD_FLAG_ATOM_PAIRS 8
#define PIMD_FLAG_NO_GRAPHS 16
#define PIMD_PAIR_SUBGROUPS_SHIFT 8
#define PIMD_PAIR_SUBGROUPS_MASK (0xF << PIMD_PAIR_SUBGROUPS_SHIFT)
#define PIMD_PAIR_SUBGROUPS(S)                                                   \
    ((S) == 1 ? 1 << PIMD_PAIR_SUBGROUPS_SHIFT                                   \
     : (S) == 2 ? 2 << PIMD_PAIR_SUBGROUPS_SHIFT                                 \
     : (S) == 4 ? 3 << PIMD_PAIR_SUBGROUPS_SHIFT                                 \
     : (S) == 8 ? 4 << PIMD_PAIR_SUBGROUPS_SHIFT                                 \
     : (S) == 16 ? 5 << PIMD_PAIR_SUBGROUPS_SHIFT : 0)

typedef struct pimd_topology {
    const int32_t *lj_active; /* [N] 1 = takes part in LJ; NULL = every atom */
    int32_t n_bonds;          /* harmonic bonds, at most 4 per atom */
    const int32_t *bonds;     /* [n_bonds][2] atom indices (caller's order) */
} pimd_topology;

/* Instantaneous estimators at the state's step, and running sums over every
 * step completed by pimd_step since the last pimd_reset_averages. */
#define PIMD_NEST 10
typedef struct pimd_estimators {
    uint64_t step;     /* thermostat step counter of the state */
    /* order of the arrays below: ekin, espring, epot, etot, kprim, kcv, temp, pcv, ppr, pmd */
    double value[PIMD_NEST];
    uint64_t count;    /* number of steps in the running sums */
    double sum[PIMD_NEST];
    double sumsq[PIMD_NEST];
    int32_t nonfinite; /* 1 if a NaN/Inf position or velocity was seen */
    int32_t overflow;  /* 1 if a neighbor list ran out of capacity */
    uint64_t n_rebuilds; /* neighbor-list builds since set_state (LJ, WATER) */
    double rlist;        /* centroid cutoff of the current neighbor lists */
    /* NPT, NPH (0 otherwise), at the state's step: */
    double volume;       /* V of the current box */
    double vw;           /* barostat velocity v_W (anisotropic: the mean of the three, the
                            isotropic v_W with the same volume rate) */
    double enthalpy;     /* H + K_W + U_W + J_W (App. A): K_W = W v_W^2 / 2, U_W = P p_ext V,
                            J_W = -P kB T ln V */
    double vwa[3];       /* anisotropic barostat: v_W of each dimension (0 otherwise) */
} pimd_estimators;
/* ekin    = sum_k sum_i 1/2 m_i |v~_i^(k)|^2 (App. A item 1)
 * espring = sum_k sum_i 1/2 m_i omega_n^2 lambda_k |x~_i^(k)|^2 (App. A item 2,
 *           read with omega_n^2)
 * epot    = sum_k U^(k) (App. A item 3)
 * etot    = H = ekin + espring + epot (Eq. A4)
 * kprim   = K_PR = 3 P N kB T / 2 - espring / P (Eq. A5, read with the 1/P)
 * kcv     = K_CV = 3 N kB T / 2 - (1/2P) sum_k sum_i (r_i^k - r_i^c).F_i^k (Eq. A7)
 * temp    = 2 ekin / (3 N P^2 kB): the ring-polymer temperature over P (Sec. III.A)
 * pcv     = P_CV, the centroid-virial pressure (App. A):
 *           [sum_i m_i |v~_i^(0)|^2 - sum_k sum_i (r_i^k - r_i^c).F_i^k
 *            + sum_k Tr Xi^k] / (3 P V), with V the box volume and Tr Xi^k the
 *           cell virial of bead k (the sum of r_ij.F_ij over interacting pairs,
 *           every periodic image, and bonds; equal to minus the derivative of
 *           U^(k) under a uniform scaling of positions and box).  Computed for
 *           PIMD_POT_LJ and PIMD_POT_WATER; 0 for every other potential, whose
 *           forces carry no cell virial here.  With fixcom the centroid term is
 *           taken after the center-of-mass velocity is removed.
 * ppr     = P_PR, the primitive pressure (App. A), read with the virial and the
 *           1/P that the printed formula lacks (kB T times the volume derivative
 *           of the log of the ring polymer's Boltzmann weight):
 *           [3 P N kB T - (2 espring - sum_k Tr Xi^k) / P] / (3V); 0 likewise
 * pmd     = P_MD, the pressure of the extended classical system (App. A):
 *           [2 ekin + sum_k Tr Xi^k] / (3V); 0 likewise */

typedef struct pimd_ctx pimd_ctx;

/* Device bytes one context needs for these parameters (for admission by HBM
 * budget).  mass [N] is required for LJ and WATER unless nbr_capacity > 0
 * (the neighbor-list size is bounded from the lightest active atom's thermal
 * wavelength); topo may be NULL.  Errors: PIMD_ERR_ARG, PIMD_ERR_UNSUPPORTED. */
int pimd_workspace_bytes(const pimd_params *p, const double *mass, const pimd_topology *topo,
                         size_t *bytes);

/* Create a context on the current HIP device.
 *   p         parameters (copied)
 *   mass      [N] host masses > 0 (copied)
 *   topo      WATER: active-LJ flags and bonds; LJ: may be NULL; else ignored
 *   workspace device buffer of at least pimd_workspace_bytes() bytes owned by
 *             the caller and kept alive until pimd_destroy, or NULL to let the
 *             library allocate (hipMalloc) its own
 *   stream    hipStream_t to enqueue on (borrowed; must not be the legacy
 *             null stream), or NULL for a stream owned by the context
 * Errors: ARG (bad parameter), UNSUPPORTED (P > 128, pair potential without a
 * periodic box), OOM, DEVICE. */
int pimd_create(const pimd_params *p, const double *mass, const pimd_topology *topo,
                void *workspace, size_t workspace_bytes, void *stream, pimd_ctx **out);

/* Load a state (Sec. IV.A: Cartesian positions, velocities turned into normal
 * modes v~ = M v).  x and v are [P][N][3] host arrays; x is taken as
 * unwrapped (all beads of an atom in the same periodic image, Sec. IV.B).
 * Computes f(x), the neighbor lists and the estimators of this state (with
 * external forces: neither; they follow pimd_set_forces), and sets the
 * thermostat step counter to `step`.  Synchronizes.
 * Errors: ARG (NULL or non-finite input, step >= 2^63), DEVICE. */
int pimd_set_state(pimd_ctx *ctx, const double *x, const double *v, uint64_t step);

/* Enqueue nsteps >= 0 steps on the context's stream and return without
 * waiting.  Each BAOAB step: B(dt/2), A(dt/2), O(dt), A(dt/2), forces,
 * B(dt/2), in normal modes (OBABO: see the integrator field); the noise for
 * mode k, atom i (the caller's index), dim a at step s is the Philox4x32-10
 * stream keyed by (seed mod 2^32, seed / 2^32) at counter (i, k, s mod 2^32,
 * s / 2^32) (with 2^31 added to the last word for OBABO's second O), through
 * Box-Muller; steps below 2^63.
 * After the call's work completes the state is synchronized (full-step
 * velocities) and the estimators of every step are in the running sums.
 * External forces take one step per call (see pimd_set_forces).
 * Errors: STATE (no set_state yet; external forces not set), ARG (nsteps < 0;
 * external forces and nsteps > 1), DEVICE. */
int pimd_step(pimd_ctx *ctx, int64_t nsteps);

/* Wait for the stream, then copy out the estimators.  Returns
 * PIMD_ERR_NONFINITE / PIMD_ERR_OVERFLOW (after filling *out) if the device
 * flagged either condition.  Errors: STATE, DEVICE. */
int pimd_get_estimators(pimd_ctx *ctx, pimd_estimators *out);

/* Wait for the stream, then copy out Cartesian positions x (unwrapped) and
 * momenta p = m M^T v~, both [P][N][3] host arrays (either may be NULL), and
 * the step counter (may be NULL).  Errors: STATE, DEVICE. */
int pimd_get_state(pimd_ctx *ctx, double *x, double *p, uint64_t *step);

/* NPT, NPH: wait for the stream, then copy out the current box lengths
 * (box[3], may be NULL) and the barostat velocity (vw, may be NULL: one
 * double, or with baro_aniso the three v_Wa).
 * Errors: STATE, UNSUPPORTED (no barostat), DEVICE. */
int pimd_get_barostat(pimd_ctx *ctx, double *box, double *vw);

/* NPT, NPH: the box lengths (box[3], > 0; isotropic: in the aspect ratio of
 * params.box, which that barostat keeps) and barostat velocity (vw: one
 * double, or with baro_aniso three) that the next pimd_set_state starts
 * from, e.g. those pimd_get_barostat returned with the state being restored;
 * the state's forces and estimators are then those of this box.  Host-side
 * only (no device work).  Errors: ARG (bad box, NULL or non-finite vw),
 * UNSUPPORTED (no barostat). */
int pimd_set_barostat(pimd_ctx *ctx, const double *box, const double *vw);

/* Bosonic exchange springs (the bosonic fix of Sec. III.C; the exchange
 * potential of Hirshberg et al. 2019, evaluated in quadratic time as in
 * Feldman and Hirshberg 2023, both cited by the paper).  N identical
 * particles of P beads, x [P][N][3] (bead, particle, dim; device memory).
 * Springs kspring |r - r'|^2 (kspring = m omega_n^2 / 2) join bead j to j+1
 * inside each particle's ring; the link from bead P-1 of a particle to bead 0
 * of the next is summed over exchange cycles:
 *   exp(-beta_n V[n]) = (1/n) sum_{k=1..n} exp(-beta_n (E[n,k] + V[n-k])),
 * V[0] = 0, E[n,k] the single ring through particles n-k..n-1 (0-based),
 * V_B = V[N].  box (host, [3]; NULL = no box): periodic lengths, 0 = not
 * periodic in that dimension; each link's vector is then taken under the
 * minimum image, while a particle's own springs use its unwrapped
 * coordinates.
 * Writes to out (device, two doubles) V_B and EV_B = sum_k w[n,k] (E[n,k] +
 * EV[n-k]) at n = N (w the recursion's weights, EV[0] = 0), the ring energy
 * that App. A's bosonic primitive kinetic energy estimator subtracts:
 * K_PR = 3 P N kB T / 2 - EV_B / P.  f ([P][N][3], device, overwritten)
 * receives the spring forces -dV_B/dx; prob ([N][N], device, or NULL) the
 * probability that bead P-1 of particle l links to bead 0 of particle l'.
 * Work is enqueued on stream (a hipStream_t; NULL = the null stream); the
 * call allocates its scratch (about 8 N^2 bytes), waits for the stream and
 * frees it before it returns.
 * Errors: ARG (NULL x, f or out, N < 1, P < 1, kspring < 0 or not finite,
 * beta_n <= 0, a negative or non-finite box length), UNSUPPORTED (N > 1024,
 * P > 128), OOM (scratch), DEVICE. */
int pimd_boson_spring(const double *x, int32_t N, int32_t P, double kspring, double beta_n,
                      const double *box, double *f, double *prob, double *out, void *stream);

/* pimd_boson_spring without any allocation, for callers that cannot allocate
 * device memory: code under hipGraph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same arguments, results and errors as
 * pimd_boson_spring, for N <= 512 (UNSUPPORTED above).  Its scratch is a
 * static device array of 2.1 MB per device, held until the process ends and
 * looked up (hipGetSymbolAddress) at the first call on each device.  The call
 * enqueues its kernels on stream and returns without waiting.  All calls on a
 * device share that device's scratch, which keeps the last call's contents
 * (every value a call reads is written earlier in the same call, so nothing is
 * cleared): calls that overlap on one device, on different streams or from
 * different host threads, race and give wrong results. */
int pimd_boson_spring_noalloc(const double *x, int32_t N, int32_t P, double kspring,
                              double beta_n, const double *box, double *f, double *prob,
                              double *out, void *stream);

/* Clear the running sums (enqueued on the stream).  Errors: STATE, DEVICE. */
int pimd_reset_averages(pimd_ctx *ctx);

/* External forces (PIMD_POT_EXTERNAL).  The library computes no forces; the
 * caller evaluates its potential on the P replicas of the current positions
 * and hands back the forces, once per step (Sec. IV.A: the force call of the
 * step, made by the caller instead of the library):
 *
 *   pimd_set_state(ctx, x, v, s0);
 *   loop: pimd_get_positions(ctx, xd);  f = -dU/dx at xd (caller);
 *         pimd_set_forces(ctx, fd, U);  pimd_step(ctx, 1);
 *
 * pimd_set_forces completes the pending closing half-kick of the last step
 * (or, right after pimd_set_state, nothing) and records the estimators of the
 * state with these forces, as pimd_step does for the library's potentials.
 * pimd_step then takes exactly one step; pimd_get_estimators and the momenta
 * of pimd_get_state need the forces of the current positions (STATE
 * otherwise).  Not available in a batch. */

/* Enqueue a copy of the Cartesian positions (unwrapped) into x, a [P][N][3]
 * DEVICE array on the context's device (caller's atom order), on the
 * context's stream; order the caller's reads after it on that stream.  Any
 * potential.  Errors: ARG (NULL), STATE (no set_state yet), DEVICE. */
int pimd_get_positions(pimd_ctx *ctx, double *x);

/* Forces on the current positions, f [P][N][3] DEVICE array (caller's atom
 * order; read on the context's stream, so the caller may reuse it once that
 * stream has passed this call), and their total potential energy
 * epot = sum_k U^(k) (App. A, item 3).  Enqueued; returns without waiting.
 * Errors: STATE (potential not PIMD_POT_EXTERNAL, or no set_state yet),
 * ARG (NULL f or non-finite epot), DEVICE. */
int pimd_set_forces(pimd_ctx *ctx, const double *f, double epot);

/* Per-kernel timing.  Between pimd_profile_begin and pimd_profile_end,
 * pimd_step launches its kernels directly (no graph) and brackets each one
 * with HIP events on the context's stream; pimd_profile_end waits for the
 * stream and returns, per kernel kind, the number of launches and the summed
 * event-measured durations.  Kinds: PIMD_KERNEL_FUSED (the step pass),
 * PIMD_KERNEL_PAIR (forces), PIMD_KERNEL_CLOSE (closing B at the end of a
 * pimd_step call), PIMD_KERNEL_FINALIZE (the one-block reduction after each
 * fused or closing pass).  Errors: STATE (end without begin), DEVICE. */
#define PIMD_NKERNEL 4
#define PIMD_KERNEL_FUSED 0
#define PIMD_KERNEL_PAIR 1
#define PIMD_KERNEL_CLOSE 2
#define PIMD_KERNEL_FINALIZE 3
typedef struct pimd_profile {
    uint64_t launches[PIMD_NKERNEL];
    double ms[PIMD_NKERNEL];
} pimd_profile;
int pimd_profile_begin(pimd_ctx *ctx);
int pimd_profile_end(pimd_ctx *ctx, pimd_profile *out);

/* Launch shapes the context uses (chosen at pimd_create from the tuning
 * table and the flags; fixed for the context's life).  transforms: 1 = FP64
 * matrix cores, 0 = FP64 vector ALUs in the step pass; fused_blocks: blocks
 * of the step pass; pair_subgroups, pair_blocks: lane sub-groups per atom and
 * blocks of the force pass (0 without pair forces); cells: centroid cells of
 * the list build (0 = all-pairs scan); cluster_pairs: 1 when the force pass
 * runs on cluster lists; bead_pairs: 1 when its lanes take two consecutive
 * beads each (even P, per-atom lists; the pair_subgroups sub-groups of P
 * lanes then work as twice as many of P/2 lanes).  Errors: ARG. */
typedef struct pimd_launch_info {
    int32_t transforms;
    int32_t fused_blocks;
    int32_t pair_subgroups;
    int32_t pair_blocks;
    int32_t cells;
    int32_t cluster_pairs;
    int32_t bead_pairs;
} pimd_launch_info;
int pimd_get_launch_info(const pimd_ctx *ctx, pimd_launch_info *out);

/* ---- Batched execution ------------------------------------------------
 * Many independent systems (each with its own N, P, T, potential, seed, ...)
 * advanced together: one step of the whole batch is a fixed handful of
 * launches (the fused pass per bead-count group, one finalize pass with a
 * block per system, the force pass for the systems with even and with odd
 * P), whatever the number of systems, and
 * chunks of steps are captured in a hipGraph.  Every system behaves exactly
 * as a pimd_ctx with the same parameters (same kernels, same noise stream);
 * its arithmetic does not depend on the other systems in the batch.
 * A system id stays valid until pimd_batch_remove.  Batch calls are made by
 * one host thread at a time. */
typedef struct pimd_batch pimd_batch;

/* Empty batch on the current device.  stream: hipStream_t (borrowed, not the
 * legacy null stream) or NULL for a stream owned by the batch.
 * Errors: ARG, DEVICE. */
int pimd_batch_create(void *stream, pimd_batch **out);

/* Add a system (arguments as in pimd_create; the library allocates its
 * device memory, pimd_workspace_bytes() of it).  The system takes part in
 * pimd_batch_step once pimd_batch_set_state has been called for it.
 * Errors: ARG, UNSUPPORTED, OOM, DEVICE. */
int pimd_batch_add(pimd_batch *b, const pimd_params *p, const double *mass,
                   const pimd_topology *topo, int32_t *sys);

/* Remove a system and free its device memory (waits for the stream).
 * Errors: ARG (unknown id). */
int pimd_batch_remove(pimd_batch *b, int32_t sys);

/* As pimd_set_state for one system of the batch; activates it.  Its step
 * budget becomes unlimited.  Errors: ARG, DEVICE. */
int pimd_batch_set_state(pimd_batch *b, int32_t sys, const double *x, const double *v,
                         uint64_t step);

/* Let the system take at most `steps` more steps (-1 = unlimited).  Systems
 * whose budget is spent sit out the remaining steps of a pimd_batch_step call
 * (their state is synchronized at the end of the call).  Enqueued on the
 * stream.  Errors: ARG, STATE (no state yet). */
int pimd_batch_set_budget(pimd_batch *b, int32_t sys, int64_t steps);

/* Enqueue nsteps steps for every active system with budget left, then the
 * closing B; returns without waiting.  Errors: ARG, DEVICE. */
int pimd_batch_step(pimd_batch *b, int64_t nsteps);

/* As pimd_get_estimators / pimd_get_state for one system (wait for the
 * stream).  Errors: ARG, STATE, NONFINITE, OVERFLOW, DEVICE. */
int pimd_batch_get_estimators(pimd_batch *b, int32_t sys, pimd_estimators *out);
int pimd_batch_get_state(pimd_batch *b, int32_t sys, double *x, double *p, uint64_t *step);

/* Wait for the stream, free every system and the batch.  NULL is a no-op. */
void pimd_batch_destroy(pimd_batch *b);

/* Message of the last error on the batch (never NULL). */
const char *pimd_batch_last_error(const pimd_batch *b);

/* Free the context and everything the library allocated for it (waits for
 * the stream first).  NULL is a no-op. */
void pimd_destroy(pimd_ctx *ctx);

/* Message of the last error on ctx (or of the last failed pimd_create when
 * ctx is NULL).  Never NULL; valid until the next call on the context. */
const char *pimd_last_error(const pimd_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* PIMD_H */
