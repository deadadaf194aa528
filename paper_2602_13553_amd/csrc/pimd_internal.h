// Internal declarations of libpimd.so shared by its host (pimd_api.hip) and
// device (pimd_kernels.hip) translation units.  Not installed, not part of the
// C ABI.
//
// Device layout of every per-bead array: [N][3][P] in the library's internal
// atom order (LJ-active atoms first), i.e. element (atom i, dim a, bead or
// mode k) at (i*3 + a)*P + k.  The P beads (or modes) of one atom-dim are
// contiguous, so a group of P lanes reads them in one coalesced segment, and
// neighbor gathers in the force kernel fetch whole bead rows.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pimd {

constexpr int kBlock = 256;      // threads per block for the step kernels
constexpr int kMaxBeads = 128;   // P limit of the library (LDS-resident M)
constexpr int kMaxBonds = 4;     // bonds per atom
constexpr int kNumEst = 10;      // ekin, espring, epot, etot, kprim, kcv, temp, pcv, ppr, pmd
constexpr int kCellCapMax = 4096;  // atoms per centroid cell, at most
constexpr int kMaxCells = 3072;    // centroid cells per system, at most (LDS counts, 4 per cell)
constexpr int kPairStage = 2048;        // neighbor-list entries staged in LDS per force-pass block
constexpr int kClusterMax = 512;         // union-list entries per force-pass cluster (LDS)
constexpr int kClusterRows = 1536;       // doubles per staged chunk of neighbor bead rows
constexpr int kClusterSmem = 8 * 2 * kClusterRows + 16 * kClusterMax;   // dynamic LDS bytes

// Per-block partial slots written by the fused kernel.
// PF_PX..PF_PZ: sum of hm * v~0 over the block's atoms (fixcom momentum)
// PF_K0: sum of hm |v~0|^2 over the block's atoms (centroid-virial pressure)
enum { PF_EKIN = 0, PF_ESPRING, PF_VIR, PF_UEXT, PF_EMAX, PF_DMAX, PF_NONFINITE, PF_K0, PF_PX, PF_PY,
       PF_PZ, PF_COUNT };

// Fused-kernel modes.
enum FusedMode : int {
    FUSED_STEP = 0,   // (pending closing B + estimators) opening B, A, O, A, inverse transform
    FUSED_CLOSE = 1,  // pending closing B + estimators only
    FUSED_EST = 2,    // estimators of a synchronized state (after set_state)
    FUSED_PREP = 3,   // v~ = M v, centroids, excursion; requests a neighbor build
};

// Device-resident control block.  Written by k_finalize (one block, after
// each fused pass) and by small host-enqueued kernels; read at kernel start.
struct Ctl {
    unsigned long long step;   // thermostat step counter s
    int synced;                // 1: velocities are at the full step
    int rebuild;               // 1: the coming force pass rebuilds the lists
    double rlist;              // centroid cutoff of the current lists
    double ebuild;             // max bead-centroid excursion at the last build
    int nonfinite;
    int overflow;
    unsigned long long n_rebuilds;
    long long budget;          // steps this system may still take (-1 = unlimited)
    int ran;                   // 1: the last fused pass did work (the force pass follows it)
    int pad1;
    unsigned long long est_step;
    double value[kNumEst];
    unsigned long long count;
    double sum[kNumEst];
    double sumsq[kNumEst];
    int cell_ok;               // 1: the coming rebuild may use the sorted cells
    int cell_R[3];             // stencil half-width in cells per dim for that rebuild
    double ucom[3];            // fixcom: centroid-mode velocity to subtract from every atom
    int ucom_pending;          // 1: ucom is still to be subtracted
    int pad2;
    // barostat (NpT, NpH): the box moves with v_W, so the passes read it here
    double box[3];             // current box lengths
    double box_build[3];       // box lengths at the last neighbor-list build
    double vw;                 // barostat velocity v_W
    double volume;             // V, K_W + U_W + J_W and the enthalpy at the estimator point
    double ebaro;
    double enthalpy;
    double vwa[3];             // anisotropic barostat: v_W per dimension (vw unused)
};

// One atom of a centroid cell as the list build reads it: its centroid, its
// index and the integer box index of the unwrapped centroid per dim.
struct __attribute__((aligned(16))) CellEntry {
    double c[3];
    int j;
    int nb[3];
    int pad;
};

struct FusedArgs {
    int N, P, n_active;
    int mode;                 // FusedMode
    int pair;                 // 1: forces come from array f (the pair kernel or the caller)
    int lists;                // 1: neighbor lists (rebuild decisions) exist
    int nvt;                  // 1: PILE-L O step
    int obabo;                // 1: OBABO splitting (O half steps around B A A B), 0: BAOAB
    int fixcom;               // 1: centroid COM velocity removed at the end of every step
    double inv_hsum;          // 1 / sum_i hm_i (fixcom)
    double inv_3v;            // 1 / (3 V) for periodic pair systems, else 0 (pressures)
    double hdt;               // dt / 2
    double omega2;            // external trap omega^2 (0 for none / pair)
    double skin;
    double rc;
    double kT15N;             // 3 N kB T / 2
    double kT15PN;            // 3 P N kB T / 2
    double temp_norm;         // 2 / (3 N P^2 kB)
    unsigned long long seed;
    double *x;                // [N][3][P] Cartesian, unwrapped
    double *yt;               // [N][3][P] y~ = M (x - x_bead0): the positions' modes, carried
    double *v;                // [N][3][P] normal-mode velocities
    const double *f;          // [N][3][P] Cartesian forces (pair) or nullptr
    const double *vin;        // PREP: [N][3][P] Cartesian velocities
    double *cent;             // [N][3] centroids (written)
    const double *cref;       // [N][3] centroids at the last list build
    const double *M;          // [P][P] normal-mode matrix, row = mode
    const double *MT;         // [P][P] its transpose, row = bead
    const double *modes;      // [P][8] per-mode constants
    const double *atoms;      // [N][4] per-atom constants
    const int *orig;          // [N] caller's atom index (noise counter)
    double *partials;         // [gridDim][PF_COUNT]
    const double *fpartials;  // [n_fpartials][2] force-pass (energy, cell virial) per block
    int n_fpartials;
    Ctl *ctl;
    // centroid cells (ncell = 0: no cell list, lists come from the all-pairs scan)
    int ncell, cell_cap;
    int nc[3];                // cells per dim, each >= 3
    double box[3];
    double icw[3];            // cells per unit length
    CellEntry *cell_ent;      // [ncell][cell_cap] the same, increasing index, with centroids
    int *cell_scnt;           // [ncell] atoms per cell
    int4 *cinfo;              // [N] (cell, image index per dim) of each active atom's centroid
    // bosonic exchange (the bosonic fix): Cartesian bead velocities in v, the
    // step pass of pimd_boson.hip, and the springs' forces and energies apart
    int boson;
    const double *fs;         // [N][3][P] spring forces (rings and exchange links)
    const double *bres;       // [2] V_B and EV_B of the current positions
};

// modes[k*8 + ...]
enum { MD_A00 = 0, MD_A01, MD_A10, MD_A11, MD_C1, MD_C2, MD_SPRING, MD_NONCENTROID };
// atoms[i*4 + ...]
enum { AT_HALF_M = 0, AT_INV_M, AT_SIGMA, AT_ACTIVE };

// bond_j entries with this bit set name a partner whose force the atom's
// bond writes (the partner has no lane of its own in the force pass)
constexpr int kBondOwned = 1 << 30;

struct PairArgs {
    int N, P, n_active, cap;
    int n_forced;             // atoms 0..n_forced-1 have lanes; the rest are bond-owned
    int S;                    // sub-groups of lanes sharing one atom's list
    int paired;               // 1: lanes take bead pairs (pair_lanes_paired)
    int n_active_tiles;       // tiles that hold LJ-active atoms (they come first)
    double box[3];
    double rc2;
    double lj_eps, lj_sig2, lj_ushift;
    double bond_k, bond_r0;
    const double *x;          // [N][3][P]
    double *f;                // [N][3][P]
    const double *cent;       // [N][3]
    double *cref;             // [N][3]
    int *nbr_count;           // [N]
    int2 *nbr;                // [N][cap] (j, packed image shift)
    const int *bond_j;        // [N][kMaxBonds] partner or -1
    double *fpartials;        // [gridDim][2]: (energy, cell virial) per block
    Ctl *ctl;
    int nc[3], cell_cap;      // centroid cells (see FusedArgs)
    const CellEntry *cell_ent;
    const int *cell_scnt;
    const int4 *cinfo;
    // cluster lists (n_clusters = 0: per-atom lists only).  Block b of the
    // force pass takes the kBlock/P consecutive atoms b*A ...; its active atoms
    // share one list of neighbors j with a mask of the atoms that use each.
    int n_clusters, ccap;
    int4 *clist;              // [n_clusters][ccap] (3P j, packed shift, atom mask, 0)
    int *ccount;              // [n_clusters]
    int *cframe;              // [n_active] packed box offset of each atom in its cluster's frame
    int *cmode;               // [n_clusters] 0: cluster list, 1: per-atom lists (fallback)
    double *fdiag;            // anisotropic barostat: [blocks][3] the diagonal of each
                              // block's cell virial (nullptr: not needed)
};

// Barostat passes (pimd_npt.hip).  A step is: NPT_STEP pass A (pending
// closing kick and O, estimators, opening O, the barostat's sums) -> its
// finalize (the barostat's kicks and O steps) -> pass B (kick, A with the
// centroid scaling, inverse transform) -> its finalize (box, rebuild) ->
// forces in the new box.
enum NptMode : int { NPT_STEP = 0, NPT_CLOSE = 1, NPT_EST = 2 };
// per-block partials of pass A
enum { NP_EKIN = 0, NP_ESPRING, NP_VIR, NP_K0, NP_K0A, NP_FVA, NP_F2, NP_K0B, NP_FVB, NP_BAD,
       NP_COUNT };
// the anisotropic barostat's per-dimension sums, after those (3 each)
enum { NP_K0A3 = NP_COUNT, NP_FVA3 = NP_COUNT + 3, NP_F23 = NP_COUNT + 6, NP_K0B3 = NP_COUNT + 9,
       NP_FVB3 = NP_COUNT + 12, NP_VIR3 = NP_COUNT + 15, NP_COUNT_ANISO = NP_COUNT + 18 };
struct NptArgs {
    FusedArgs f;              // the system (x, v, f, tables, control block, partials)
    double *ft;               // [N][3][P] f~ of the current forces (pass A -> pass B)
    double *part;             // [gridDim][NP_COUNT_ANISO] pass A partials; pass B: [gridDim][3]
    int aniso;                // 1: one v_W per dimension (App. E's anisotropic barostat)
    const double *fdiag;      // aniso: [force-pass blocks][3] diagonal of the cell virial
    double dt;
    double p_ext;
    double wmass;             // W = 3 P N kB T tau_p^2
    double bc1, bc2, bsig;    // v_W's O step over dt/2: c1, c2, sqrt(P kB T / W)
    double kTP;               // P kB T
};
int npt_grid(int N, int P);
// vw: the isotropic v_W in [0]; anisotropic, the three v_Wa
void launch_npt_init(Ctl *ctl, const double box[3], const double vw[3], hipStream_t s);
void launch_npt_a(const NptArgs &a, int mode, hipStream_t s);
void launch_npt_b(const NptArgs &a, hipStream_t s);
void launch_pair_npt(const PairArgs &a, int grid, hipStream_t s);

// Bosonic exchange springs (pimd_boson.hip).  Scratch (doubles): the ring
// weights w[n,k] and their probabilities' suffix sums T[n,k] (rows n = 1..N
// of n entries each, row n at n(n-1)/2), the adjoints adj[0..N] and the
// particles' inner spring energies eint[N].
constexpr int kBosonMaxN = 1024;   // particles (the sequential kernel's LDS)
constexpr __host__ __device__ inline size_t boson_scr_tri(int N) { return (size_t)N * (size_t)(N + 1) / 2; }
constexpr __host__ __device__ inline size_t boson_scr_adj(int N) { return 2 * boson_scr_tri(N); }
constexpr __host__ __device__ inline size_t boson_scr_eint(int N) { return boson_scr_adj(N) + (size_t)N + 1; }
constexpr __host__ __device__ inline size_t boson_scr_doubles(int N) { return boson_scr_eint(N) + (size_t)N; }
struct BosonArgs {
    const double *x;     // positions
    int N, P;
    int layout;          // 0: [P][N][3] (bead, particle, dim); 1: [N][3][P]
    double ks;           // kspring: m omega_n^2 / 2 (in energy units)
    double bn;           // beta_n = 1 / (P kB T)
    double box[3];       // periodic lengths of the links' minimum image (0: none)
    double *f;           // spring forces, same layout as x (overwritten)
    double *prob;        // [N][N] link probabilities, or nullptr
    double *scr;         // boson_scr_doubles(N)
    double *res;         // [2]: V_B, EV_B (the primitive estimator's weighted ring energy)
};
void launch_boson_springs(const BosonArgs &a, hipStream_t st);

// The bosonic step pass (all FusedModes) and the harmonic trap's forces on
// Cartesian beads, with per-block energies in fpartials (pimd_boson.hip).
int boson_pass_grid(int N, int P);
void launch_boson_pass(const FusedArgs &a, int grid, hipStream_t st);
int boson_trap_grid(int N, int P);
void launch_boson_trap(const FusedArgs &a, double *f, double *fpartials, hipStream_t st);

// Records the message that pimd_last_error(NULL) returns (pimd_api.hip).
int report_error(int code, const char *msg);

// Launchers (pimd_kernels.hip).
int fused_smem_bytes(int P);
int fused_grid(int N, int P);
void launch_fused(const FusedArgs &a, int grid, hipStream_t s);
void launch_finalize(const FusedArgs &a, int fused_blocks, hipStream_t s);
bool fused_mfma_supported(int P);
int fused_mfma_grid(int N, int P);
void launch_fused_mfma(const FusedArgs &a, int grid, hipStream_t s);
// batched launches: items are (system index, tile) pairs grouped by system
int mfma_block_tiles(int N, int P);
void set_mfma_batch_smem();
void launch_fused_mfma_batch(int P, bool obabo, const FusedArgs *table, const int2 *items,
                             int n_items, int grid, hipStream_t s);
void launch_fused_batch(const FusedArgs *table, const int2 *items, int n_items, int mode,
                        int smem_bytes, int grid, hipStream_t s);
void set_batch_smem(int smem_bytes);
void launch_finalize_batch(const FusedArgs *table, const int *nparts, int n_sys, int mode,
                           hipStream_t s);
void set_pair_smem();
void launch_pair_batch(const PairArgs *table, const int2 *items, int n_items, int grid,
                       bool clusters, bool paired, hipStream_t s);
int pair_subgroups(int N, int P);
int pair_grid(int N, int P, int S);
int pair_active_tiles(int n_active, int P, int S);
// The force pass gives each lane two consecutive beads (16-byte gathers) when
// P is even and the position array fits 32-bit buffer offsets; the rule is
// the same for a system alone and in a batch, so both sum in the same order.
inline bool pair_lanes_paired(int N, int P)
{
    return P % 2 == 0 && (long long)N * 3 * P * 8 < (1LL << 31);
}
void launch_pair(const PairArgs &a, int grid, hipStream_t s);
void launch_import(const double *src, double *dst, const int *orig, int N, int P, hipStream_t s);
void launch_export(const double *x, const double *v, const double *atoms_mass, const double *M,
                   const int *orig, double *xdst, double *pdst, int N, int P, hipStream_t s);
void launch_ctl_reset_sums(Ctl *ctl, hipStream_t s);
void launch_store_energy(double *dst, double v, hipStream_t s);
void launch_apply_ucom(const FusedArgs &a, hipStream_t s);
void launch_ctl_init(Ctl *ctl, unsigned long long step, hipStream_t s);
void launch_ctl_set_budget(Ctl *ctl, long long budget, hipStream_t s);

}  // namespace pimd
