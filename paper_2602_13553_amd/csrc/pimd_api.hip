// Host side of libpimd.so: parameter validation, the library's tables
// (normal-mode matrix, per-mode propagator and thermostat constants, per-atom
// constants), the device workspace, and the C ABI declared in include/pimd.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/pimd.h"
#include "pimd_internal.h"
#include "pimd_tuning.h"

using namespace pimd;

namespace {

thread_local std::string g_create_error = "no error";

constexpr int kGraphChunk = 32;   // steps per captured graph

struct Layout {
    size_t x, yt, v, f, stage, cent, cref, M, MT, modes, atoms, mass, orig, bond_j, nbr_count, nbr,
        partials, fpartials, ctl, cell_ent, cell_scnt, cinfo, total;
    int cap, fused_grid, mfma_grid, pair_grid, pair_S, pair_active_tiles, n_active;
    int n_forced;                 // atoms with lanes in the force pass (bond-owned ones last)
    int valu_tiles, mfma_tiles;
    int ncell, cell_cap, nc[3];   // centroid cells (ncell = 0: none)
    bool clusters;                // force pass on cluster lists
    int n_clusters;
    size_t clist, ccount, cframe, cmode;
    int npt_grid;                 // barostat passes' blocks (0: no barostat)
    size_t nft, npart;            // barostat: f~ and pass partials
    size_t fdiag;                 // anisotropic barostat: per force-pass block, the cell virial's diagonal
    size_t fs, bscr, bres;        // bosons: spring forces, exchange scratch, (V_B, EV_B)
    int trap_grid;                // bosons in a trap: the trap kernel's blocks
};

size_t align_up(size_t v) { return (v + 255) & ~size_t(255); }

bool is_pair(int pot) { return pot == PIMD_POT_LJ || pot == PIMD_POT_WATER; }
// the BZP barostat moves the box
bool is_npt(const pimd_params *p) { return p->ensemble == PIMD_NPT || p->ensemble == PIMD_NPH; }
// a PILE-L thermostat on the beads
bool thermostatted(const pimd_params *p) { return p->ensemble == PIMD_NVT || p->ensemble == PIMD_NPT; }
// forces from an array (the force pass or the caller) rather than in the step pass
bool forces_in_array(int pot) { return is_pair(pot) || pot == PIMD_POT_EXTERNAL; }
bool forces_in_array(const pimd_params *p) { return p->bosonic || forces_in_array(p->potential); }

}  // namespace

struct pimd_ctx {
    pimd_params p;
    Layout lay;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    char *ws = nullptr;
    bool own_ws = false;
    bool have_state = false;
    // external forces: the forces in d_f belong to the current positions, and
    // the velocities are at the full step (no closing kick pending)
    bool forces_current = true;
    bool synced = true;
    double *d_x, *d_v, *d_f, *d_stage, *d_cent, *d_cref, *d_M, *d_MT, *d_modes, *d_atoms, *d_mass;
    double *d_partials, *d_fpartials;
    int *d_orig, *d_bond_j, *d_nbr_count;
    int2 *d_nbr;
    Ctl *d_ctl;
    std::vector<int> orig;          // internal -> caller index
    FusedArgs fa;
    PairArgs pa;
    NptArgs na;                     // the barostat's passes (NPT, NPH)
    BosonArgs ba;                   // the exchange springs (bosonic)
    double start_box[3] = {0.0, 0.0, 0.0};   // the box and v_W the next set_state starts from
    double start_vw[3] = {0.0, 0.0, 0.0};   // isotropic: [0]; anisotropic: per dimension
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    bool graph_failed = false;
    // profiling: event pairs around every launch while enabled
    bool profiling = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<int, size_t>> ev_used;   // (kernel kind, first event index)
    std::string err = "no error";
};

namespace {

int fail(pimd_ctx *c, int code, const std::string &msg)
{
    if (c)
        c->err = msg;
    else
        g_create_error = msg;
    return code;
}

}  // namespace

int pimd::report_error(int code, const char *msg)
{
    g_create_error = msg;
    return code;
}

namespace {

int hip_fail(pimd_ctx *c, hipError_t e, const char *where)
{
    return fail(c, PIMD_ERR_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(ctx, expr)                                          \
    do {                                                            \
        hipError_t e_ = (expr);                                     \
        if (e_ != hipSuccess) return hip_fail((ctx), e_, #expr);    \
    } while (0)

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

int validate(const pimd_params *p, const pimd_topology *topo, std::string &why)
{
    if (!p) { why = "params is NULL"; return PIMD_ERR_ARG; }
    if (p->n_atoms < 1) { why = "n_atoms must be >= 1"; return PIMD_ERR_ARG; }
    if (p->n_beads < 1) { why = "n_beads must be >= 1"; return PIMD_ERR_ARG; }
    if (p->n_beads > kMaxBeads) { why = "n_beads > 128 is not supported"; return PIMD_ERR_UNSUPPORTED; }
    if ((long long)p->n_atoms * 3 * p->n_beads >= (1LL << 31)) {
        why = "n_atoms * 3 * n_beads must stay below 2^31";
        return PIMD_ERR_UNSUPPORTED;
    }
    {
        const int known = PIMD_FLAG_VALU_TRANSFORMS | PIMD_FLAG_MFMA_TRANSFORMS | PIMD_PAIR_SUBGROUPS_MASK |
                          PIMD_FLAG_CLUSTER_PAIRS | PIMD_FLAG_ATOM_PAIRS | PIMD_FLAG_NO_GRAPHS;
        const int code = (p->flags & PIMD_PAIR_SUBGROUPS_MASK) >> PIMD_PAIR_SUBGROUPS_SHIFT;
        if (p->flags & ~known) { why = "unknown bits in flags"; return PIMD_ERR_ARG; }
        if (code > 5 || (code > 0 && (1 << (code - 1)) * p->n_beads > kBlock)) {
            why = "PIMD_PAIR_SUBGROUPS(S) needs S in {1, 2, 4, 8, 16} and S * n_beads <= 256";
            return PIMD_ERR_ARG;
        }
    }
    if (p->ensemble < PIMD_NVT || p->ensemble > PIMD_NPH) { why = "bad ensemble"; return PIMD_ERR_ARG; }
    if (p->integrator != PIMD_BAOAB && p->integrator != PIMD_OBABO) { why = "bad integrator"; return PIMD_ERR_ARG; }
    if (p->fixcom != 0 && p->fixcom != 1) { why = "fixcom must be 0 or 1"; return PIMD_ERR_ARG; }
    if (p->potential < PIMD_POT_NONE || p->potential > PIMD_POT_EXTERNAL) { why = "bad potential"; return PIMD_ERR_ARG; }
    if (!finite_pos(p->temp) || !finite_pos(p->kB) || !finite_pos(p->hbar) || !finite_pos(p->mvv2e) ||
        !finite_pos(p->dt)) {
        why = "temp, kB, hbar, mvv2e and dt must be finite and > 0";
        return PIMD_ERR_ARG;
    }
    if (thermostatted(p) && (!finite_pos(p->tau) || !finite_pos(p->tau_scale))) {
        why = "tau and tau_scale must be finite and > 0 for NVT and NPT";
        return PIMD_ERR_ARG;
    }
    if (is_npt(p)) {
        if (!finite_pos(p->tau_p) || !std::isfinite(p->p_ext)) {
            why = "the barostat needs tau_p > 0 and a finite p_ext";
            return PIMD_ERR_ARG;
        }
        if (!is_pair(p->potential) || p->fixcom) {
            why = "the barostat runs with PIMD_POT_LJ or PIMD_POT_WATER, and fixcom = 0";
            return PIMD_ERR_UNSUPPORTED;
        }
        if (p->flags & (PIMD_FLAG_MFMA_TRANSFORMS | PIMD_FLAG_CLUSTER_PAIRS)) {
            why = "the barostat's passes use the vector-ALU transforms and per-atom lists";
            return PIMD_ERR_UNSUPPORTED;
        }
    }
    if (p->baro_aniso != 0 && (p->baro_aniso != 1 || !is_npt(p))) {
        why = "baro_aniso must be 0, or 1 with NPT or NPH";
        return PIMD_ERR_ARG;
    }
    if (p->bosonic != 0 && p->bosonic != 1) { why = "bosonic must be 0 or 1"; return PIMD_ERR_ARG; }
    if (p->bosonic) {
        if (p->ensemble != PIMD_NVT && p->ensemble != PIMD_NVE) {
            why = "bosons run in NVT or NVE";
            return PIMD_ERR_UNSUPPORTED;
        }
        if (p->potential == PIMD_POT_WATER || p->fixcom) {
            why = "bosons run with PIMD_POT_NONE, HARMONIC, LJ or EXTERNAL, and fixcom = 0";
            return PIMD_ERR_UNSUPPORTED;
        }
        if (p->n_atoms > kBosonMaxN) { why = "more than 1024 bosons"; return PIMD_ERR_UNSUPPORTED; }
        if (p->flags & PIMD_FLAG_CLUSTER_PAIRS) {
            why = "bosons use per-atom neighbor lists";
            return PIMD_ERR_UNSUPPORTED;
        }
        for (int d = 0; d < 3; ++d)
            if (!(p->box[d] >= 0.0) || !std::isfinite(p->box[d])) {
                why = "box lengths must be finite and >= 0";
                return PIMD_ERR_ARG;
            }
    }
    if (p->potential == PIMD_POT_HARMONIC && !std::isfinite(p->omega)) { why = "bad omega"; return PIMD_ERR_ARG; }
    if (is_pair(p->potential)) {
        for (int d = 0; d < 3; ++d)
            if (!finite_pos(p->box[d])) {
                why = "pair potentials need a periodic box with all lengths > 0";
                return PIMD_ERR_UNSUPPORTED;
            }
        if (!finite_pos(p->lj_rc) || !finite_pos(p->lj_sigma) || !std::isfinite(p->lj_eps) ||
            !(p->skin >= 0.0) || !std::isfinite(p->skin)) {
            why = "lj_rc, lj_sigma > 0, finite lj_eps and skin >= 0 required";
            return PIMD_ERR_ARG;
        }
        if (p->nbr_capacity < 0) { why = "nbr_capacity must be >= 0"; return PIMD_ERR_ARG; }
    }
    if (p->potential == PIMD_POT_WATER && topo) {
        if (topo->n_bonds < 0 || (topo->n_bonds > 0 && !topo->bonds)) { why = "bad bond list"; return PIMD_ERR_ARG; }
        if (!std::isfinite(p->bond_k) || !std::isfinite(p->bond_r0)) { why = "bad bond parameters"; return PIMD_ERR_ARG; }
        std::vector<int> deg(p->n_atoms, 0);
        for (int b = 0; b < topo->n_bonds; ++b) {
            const int i = topo->bonds[2 * b], j = topo->bonds[2 * b + 1];
            if (i < 0 || j < 0 || i >= p->n_atoms || j >= p->n_atoms || i == j) {
                why = "bond index out of range";
                return PIMD_ERR_ARG;
            }
            if (++deg[i] > kMaxBonds || ++deg[j] > kMaxBonds) {
                why = "more than 4 bonds on one atom";
                return PIMD_ERR_UNSUPPORTED;
            }
        }
    }
    return PIMD_OK;
}

// Atoms (caller index) outside the LJ whose only bond goes to an LJ-active
// atom (water-shaped potential with a topology; none otherwise).
std::vector<int> bond_owned(const pimd_params *p, const pimd_topology *topo)
{
    std::vector<int> owned(p->n_atoms, 0);
    if (p->potential != PIMD_POT_WATER || !topo || !topo->lj_active) return owned;
    std::vector<int> deg(p->n_atoms, 0), partner(p->n_atoms, -1);
    for (int b = 0; b < topo->n_bonds; ++b) {
        const int i = topo->bonds[2 * b], j = topo->bonds[2 * b + 1];
        ++deg[i]; ++deg[j];
        partner[i] = j; partner[j] = i;
    }
    for (int i = 0; i < p->n_atoms; ++i)
        owned[i] = (!topo->lj_active[i] && deg[i] == 1 && topo->lj_active[partner[i]]) ? 1 : 0;
    return owned;
}

// Internal order; orig[internal] = caller index.  LJ-active atoms first, then
// the other atoms that need lanes of their own in the force pass, then the
// bond-owned atoms: atoms outside the LJ with a single bond, to an LJ-active
// atom, whose force the active atom's bond writes (the H atoms of the
// water-shaped system).  Each group keeps the caller's order.  *n_forced is
// the number of atoms before the bond-owned ones.
std::vector<int> internal_order(const pimd_params *p, const pimd_topology *topo, int *n_active,
                                int *n_forced)
{
    std::vector<int> orig;
    orig.reserve(p->n_atoms);
    const int32_t *act = (p->potential == PIMD_POT_WATER && topo) ? topo->lj_active : nullptr;
    if (!is_pair(p->potential)) act = nullptr;
    for (int i = 0; i < p->n_atoms; ++i)
        if (!act || act[i]) orig.push_back(i);
    *n_active = is_pair(p->potential) ? (int)orig.size() : 0;
    *n_forced = (int)orig.size();
    if (act) {
        std::vector<int> owned = bond_owned(p, topo);
        for (int i = 0; i < p->n_atoms; ++i)
            if (!act[i] && !owned[i]) orig.push_back(i);
        *n_forced = (int)orig.size();
        for (int i = 0; i < p->n_atoms; ++i)
            if (!act[i] && owned[i]) orig.push_back(i);
    }
    return orig;
}

// Generous bound on the bead-centroid excursion of the lightest active atom:
// three thermal wavelengths hbar / sqrt(m kB T mvv2e).  Zero when the caller
// fixes the list capacity (the masses are then optional for sizing).
double excursion_guess(const pimd_params *p, const double *mass, const std::vector<int> &orig,
                       int n_active)
{
    if (p->nbr_capacity > 0 || n_active == 0 || p->n_beads < 2 || !mass) return 0.0;
    double mmin = 1e300;
    for (int q = 0; q < n_active; ++q) mmin = std::min(mmin, mass[orig[q]]);
    const double lam = p->hbar / std::sqrt(mmin * p->kB * p->temp * p->mvv2e);
    return 3.0 * lam;
}

int neighbor_capacity(const pimd_params *p, const double *mass, const std::vector<int> &orig,
                      int n_active)
{
    if (p->nbr_capacity > 0) return p->nbr_capacity;
    if (n_active == 0) return 1;
    const double e_guess = excursion_guess(p, mass, orig, n_active);
    const double r = p->lj_rc + p->skin + 2.0 * e_guess;
    const double vol = p->box[0] * p->box[1] * p->box[2];
    const double nb = (double)n_active / vol * (4.0 / 3.0) * M_PI * r * r * r;
    // a barostat may compress the box: room for twice the starting density
    return (int)std::ceil((is_npt(p) ? 2.8 : 1.4) * nb) + 32;
}

// Centroid cells of width >= the expected list cutoff rc + skin + 2 E, so that
// a rebuild normally scans 3 x 3 x 3 cells; none when a dim holds fewer than
// three cells (small boxes use the all-pairs scan with periodic images) or
// when the grid would be much sparser than the atoms.
void cell_grid(const pimd_params *p, int n_active, double e_guess, Layout &L)
{
    L.ncell = 0;
    L.cell_cap = 0;
    L.nc[0] = L.nc[1] = L.nc[2] = 0;
    if (!is_pair(p->potential) || n_active == 0) return;
    // Under a barostat the grid keeps its cell count while the box moves:
    // cells 25% wider than the cutoff leave room for the box to shrink (a
    // rebuild whose stencil no longer fits falls back to the all-pairs scan),
    // and the cell capacity allows twice the starting density.
    const bool npt = is_npt(p);
    const double w = (p->lj_rc + p->skin + 2.0 * e_guess) * (npt ? 1.25 : 1.0);
    long long ncell = 1;
    int nc[3];
    for (int d = 0; d < 3; ++d) {
        const double q = std::floor(p->box[d] / w);
        if (!(q >= 3.0)) return;
        nc[d] = (int)std::min(q, 1024.0);
        ncell *= nc[d];
    }
    if (ncell > 8LL * n_active + 64) return;
    const double mean = (double)n_active / (double)ncell;
    const int cap = ((int)std::ceil((npt ? 4.0 : 2.0) * mean) + 16 + 3) & ~3;   // rows of whole int4
    if (cap > kCellCapMax || ncell > kMaxCells) return;
    L.ncell = (int)ncell;
    L.cell_cap = cap;
    for (int d = 0; d < 3; ++d) L.nc[d] = nc[d];
}

// Transform variant of the step pass: the flags, else the tuned size at which
// the matrix cores overtake the vector ALUs for this P.
bool use_mfma(const pimd_params *p)
{
    const int P = p->n_beads;
    if (!fused_mfma_supported(P) || (p->flags & PIMD_FLAG_VALU_TRANSFORMS) || is_npt(p) || p->bosonic)
        return false;
    if (p->flags & PIMD_FLAG_MFMA_TRANSFORMS) return true;
    const int row = P == 16 ? 0 : (P == 32 ? 1 : 2);
    return (long long)p->n_atoms * P >= tuning::kMfmaMinBeadAtoms[row];
}

// Cluster lists in the force pass: the flags, else the tuning table.  They
// need a cluster of at most 32 atoms (P >= 8) and LJ-active atoms.
bool use_clusters(const pimd_params *p, int n_active)
{
    const int P = p->n_beads, N = p->n_atoms;
    if (!is_pair(p->potential) || n_active == 0 || P < 8 || kBlock / P > 32 || is_npt(p) || p->bosonic)
        return false;
    if (p->flags & PIMD_FLAG_ATOM_PAIRS) return false;
    if (p->flags & PIMD_FLAG_CLUSTER_PAIRS) return true;
    const int row = P == 8 ? 0 : P == 16 ? 1 : P == 32 ? 2 : P == 64 ? 3 : -1;
    if (row < 0) return false;
    int lg = 0;
    while ((2 << lg) <= N) ++lg;
    const int col = std::min(std::max(lg - 6, 0), 9);
    return tuning::kClusterPairs[row][col] != 0;
}

// Lane sub-groups per atom in the force pass: the flags, else the tuning
// table of the potential, else the occupancy heuristic.
int choose_pair_subgroups(const pimd_params *p)
{
    const int P = p->n_beads, N = p->n_atoms;
    const int code = (p->flags & PIMD_PAIR_SUBGROUPS_MASK) >> PIMD_PAIR_SUBGROUPS_SHIFT;
    if (code > 0) return 1 << (code - 1);
    const int row = P == 8 ? 0 : P == 16 ? 1 : P == 32 ? 2 : P == 64 ? 3 : -1;
    if (row >= 0) {
        int lg = 0;
        while ((2 << lg) <= N) ++lg;            // floor(log2 N)
        const int col = std::min(std::max(lg - 6, 0), 9);
        const int S = p->potential == PIMD_POT_WATER ? tuning::kPairSubgroupsWater[row][col]
                                                     : tuning::kPairSubgroups[row][col];
        if (S > 0 && S * P <= kBlock) return S;
    }
    return pair_subgroups(N, P);
}

Layout make_layout(const pimd_params *p, int n_active, int n_forced, int cap, double e_guess)
{
    Layout L{};
    cell_grid(p, n_active, e_guess, L);
    const size_t N = (size_t)p->n_atoms, P = (size_t)p->n_beads;
    const size_t arr = N * 3 * P * sizeof(double);
    const bool pair = is_pair(p->potential);
    L.cap = cap;
    L.n_active = n_active;
    L.fused_grid = fused_grid(p->n_atoms, p->n_beads);
    L.mfma_grid = use_mfma(p) ? fused_mfma_grid(p->n_atoms, p->n_beads) : 0;
    L.clusters = pair && use_clusters(p, n_active);
    L.pair_S = pair ? (L.clusters ? 1 : choose_pair_subgroups(p)) : 1;
    L.n_forced = n_forced;
    L.pair_grid = pair ? pair_grid(n_forced, p->n_beads, L.pair_S) : 0;
    L.pair_active_tiles = pair ? pair_active_tiles(n_active, p->n_beads, L.pair_S) : 0;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o += align_up(bytes); return r; };
    L.x = take(arr);
    L.yt = take(arr);
    L.v = take(arr);
    L.f = take(forces_in_array(p) ? arr : 0);
    L.stage = take(arr);
    L.cent = take(N * 3 * sizeof(double));
    L.cref = take(N * 3 * sizeof(double));
    L.M = take(P * P * sizeof(double));
    L.MT = take(P * P * sizeof(double));
    L.modes = take(P * 8 * sizeof(double));
    L.atoms = take(N * 4 * sizeof(double));
    L.mass = take(N * sizeof(double));
    L.orig = take(N * sizeof(int));
    L.bond_j = take(pair ? N * kMaxBonds * sizeof(int) : 0);
    L.nbr_count = take(pair ? N * sizeof(int) : 0);
    L.nbr = take(pair ? (size_t)n_active * cap * sizeof(int2) : 0);
    // partials: per block (single system) or per tile (batched execution)
    L.valu_tiles = (p->n_atoms + (kBlock / p->n_beads) - 1) / (kBlock / p->n_beads);
    L.mfma_tiles = fused_mfma_supported(p->n_beads) ? mfma_block_tiles(p->n_atoms, p->n_beads) : 0;
    const int nparts = std::max(std::max(L.fused_grid, L.mfma_grid), std::max(L.valu_tiles, L.mfma_tiles));
    L.partials = take((size_t)nparts * PF_COUNT * sizeof(double));
    L.trap_grid = (p->bosonic && p->potential == PIMD_POT_HARMONIC) ? boson_trap_grid(p->n_atoms, p->n_beads) : 0;
    L.fpartials = take((size_t)2 * std::max(std::max(L.pair_grid, L.trap_grid), 1) * sizeof(double));
    L.ctl = take(sizeof(Ctl));
    L.cell_ent = take((size_t)L.ncell * L.cell_cap * sizeof(CellEntry));
    L.cell_scnt = take((size_t)L.ncell * sizeof(int));
    L.cinfo = take(L.ncell ? N * sizeof(int4) : 0);
    L.n_clusters = L.clusters ? (n_active + (kBlock / p->n_beads) - 1) / (kBlock / p->n_beads) : 0;
    L.clist = take((size_t)L.n_clusters * kClusterMax * sizeof(int4));
    L.ccount = take((size_t)L.n_clusters * sizeof(int));
    L.cframe = take(L.clusters ? (size_t)n_active * sizeof(int) : 0);
    L.cmode = take((size_t)L.n_clusters * sizeof(int));
    L.npt_grid = is_npt(p) ? npt_grid(p->n_atoms, p->n_beads) : 0;
    L.nft = take(L.npt_grid ? arr : 0);
    L.npart = take((size_t)L.npt_grid * NP_COUNT_ANISO * sizeof(double));
    L.fdiag = take((L.npt_grid && p->baro_aniso) ? (size_t)L.pair_grid * 3 * sizeof(double) : 0);
    L.fs = take(p->bosonic ? arr : 0);
    L.bscr = take(p->bosonic ? boson_scr_doubles(p->n_atoms) * sizeof(double) : 0);
    L.bres = take(p->bosonic ? 2 * sizeof(double) : 0);
    L.total = o;
    return L;
}

// Normal-mode matrix of App. B (Eq. B1): row k = mode, column j = bead.
// Centroid row 1/sqrt(P); for even P the alternating row (-1)^j/sqrt(P) at
// k = P/2; cosine rows sqrt(2/P) cos(2 pi k j/P) for 1 <= k <= P/2; sine rows
// sqrt(2/P) sin(2 pi k j/P) above.  The phase k*j is reduced mod P first.
std::vector<double> nm_matrix(int P)
{
    std::vector<double> M((size_t)P * P);
    const double a0 = 1.0 / std::sqrt((double)P), a1 = std::sqrt(2.0 / (double)P);
    for (int k = 0; k < P; ++k) {
        const bool alt = (P % 2 == 0) && (2 * k == P);
        for (int j = 0; j < P; ++j) {
            const long long ph = ((long long)k * j) % P;
            const double ang = 2.0 * M_PI * (double)ph / (double)P;
            double m;
            if (k == 0)
                m = a0;
            else if (alt)
                m = (j & 1) ? -a0 : a0;
            else if (2 * k < P)
                m = a1 * std::cos(ang);
            else
                m = a1 * std::sin(ang);
            M[(size_t)k * P + j] = m;
        }
    }
    return M;
}

// Per-mode constants: exact free-ring-polymer flow over h = dt/2 for the
// spring frequency omega_k = 2 omega_n |sin(pi k / P)|, omega_n = P kB T / hbar
// (Eqs. 2, B2); PILE-L c1 = exp(-t/tau_k), c2 = sqrt(1 - c1^2) with tau_0 = tau
// and tau_k = tau_scale / (2 omega_k) (Eqs. D1, D2) for the O step's length t
// (dt in BAOAB, dt/2 for each of OBABO's two O steps); omega_k^2 for the spring
// energy.
std::vector<double> mode_table(const pimd_params *p)
{
    const int P = p->n_beads;
    std::vector<double> t((size_t)P * 8, 0.0);
    const double wn = (double)P * p->kB * p->temp / p->hbar;
    const double h = 0.5 * p->dt;
    for (int k = 0; k < P; ++k) {
        const double wk = (k == 0) ? 0.0 : 2.0 * wn * std::fabs(std::sin(M_PI * (double)k / (double)P));
        double *r = &t[(size_t)k * 8];
        if (wk == 0.0) {
            r[MD_A00] = 1.0; r[MD_A01] = h; r[MD_A10] = 0.0; r[MD_A11] = 1.0;
        } else {
            const double c = std::cos(wk * h), s = std::sin(wk * h);
            r[MD_A00] = c; r[MD_A01] = s / wk; r[MD_A10] = -wk * s; r[MD_A11] = c;
        }
        if (thermostatted(p)) {
            // bosons: Cartesian beads, one damping time for all (App. D)
            const double tau_k = (k == 0 || p->bosonic) ? p->tau : p->tau_scale / (2.0 * wk);
            const double to = (p->integrator == PIMD_OBABO) ? 0.5 * p->dt : p->dt;
            r[MD_C1] = std::exp(-to / tau_k);
            r[MD_C2] = std::sqrt(-std::expm1(-2.0 * to / tau_k));
        } else {
            r[MD_C1] = 1.0; r[MD_C2] = 0.0;
        }
        r[MD_SPRING] = wk * wk;
        r[MD_NONCENTROID] = (k == 0) ? 0.0 : 1.0;
    }
    return t;
}

int launch_error(pimd_ctx *c, const char *where)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(c, e, where);
    return PIMD_OK;
}

// Event pair around a launch when profiling (events are pooled and reused).
size_t prof_begin(pimd_ctx *c, int kind)
{
    if (!c->profiling) return 0;
    size_t first = c->ev_used.empty() ? 0 : c->ev_used.back().second + 2;
    while (c->ev_pool.size() < first + 2) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return 0;
        c->ev_pool.push_back(e);
    }
    c->ev_used.push_back({kind, first});
    (void)hipEventRecord(c->ev_pool[first], c->stream);
    return first;
}

void prof_end(pimd_ctx *c, size_t first)
{
    if (c->profiling) (void)hipEventRecord(c->ev_pool[first + 1], c->stream);
}

void enqueue_fused(pimd_ctx *c, int mode, int kind)
{
    FusedArgs a = c->fa;
    a.mode = mode;
    // the step pass uses the matrix-core transforms where available
    const bool mfma = (mode == FUSED_STEP) && c->lay.mfma_grid > 0;
    const int blocks = mfma ? c->lay.mfma_grid : c->lay.fused_grid;
    size_t e = prof_begin(c, kind);
    if (mfma)
        launch_fused_mfma(a, blocks, c->stream);
    else
        launch_fused(a, blocks, c->stream);
    prof_end(c, e);
    e = prof_begin(c, PIMD_KERNEL_FINALIZE);
    launch_finalize(a, blocks, c->stream);
    prof_end(c, e);
}

// One barostat step: pass A (pending closing, estimators, opening O) and
// pass B (kick, A, inverse transform), each with its finalize, then the
// forces in the new box.
void enqueue_step_npt(pimd_ctx *c)
{
    size_t e = prof_begin(c, PIMD_KERNEL_FUSED);
    launch_npt_a(c->na, NPT_STEP, c->stream);
    launch_npt_b(c->na, c->stream);
    prof_end(c, e);
    e = prof_begin(c, PIMD_KERNEL_PAIR);
    launch_pair_npt(c->pa, c->lay.pair_grid, c->stream);
    prof_end(c, e);
}

// The forces of the current positions: the force pass (pair potentials) and,
// for bosons, the trap's and the springs' (rings and exchange links).
void enqueue_forces(pimd_ctx *c)
{
    if (c->lay.pair_grid > 0) {
        size_t e = prof_begin(c, PIMD_KERNEL_PAIR);
        launch_pair(c->pa, c->lay.pair_grid, c->stream);
        prof_end(c, e);
    }
    if (c->p.bosonic) {
        size_t e = prof_begin(c, PIMD_KERNEL_PAIR);
        if (c->lay.trap_grid > 0) launch_boson_trap(c->fa, c->d_f, c->d_fpartials, c->stream);
        launch_boson_springs(c->ba, c->stream);
        prof_end(c, e);
    }
}

void enqueue_step(pimd_ctx *c)
{
    if (c->lay.npt_grid) {
        enqueue_step_npt(c);
        return;
    }
    // fixcom with a force pass: the last step's closing half-kick runs in a
    // pass of its own, so that its centroid momentum is known (and removed at
    // the start of the step pass) before the step's opening half-kick
    if (c->fa.fixcom && c->lay.pair_grid > 0) enqueue_fused(c, FUSED_CLOSE, PIMD_KERNEL_CLOSE);
    enqueue_fused(c, FUSED_STEP, PIMD_KERNEL_FUSED);
    enqueue_forces(c);
}

}  // namespace

extern "C" {

int pimd_workspace_bytes(const pimd_params *p, const double *mass, const pimd_topology *topo,
                         size_t *bytes)
{
    std::string why;
    int rc = validate(p, topo, why);
    if (rc != PIMD_OK) return fail(nullptr, rc, why);
    if (!bytes) return fail(nullptr, PIMD_ERR_ARG, "bytes is NULL");
    if (!mass && is_pair(p->potential) && p->nbr_capacity == 0)
        return fail(nullptr, PIMD_ERR_ARG, "mass is required to size neighbor lists");
    int n_active = 0, n_forced = 0;
    std::vector<int> orig = internal_order(p, topo, &n_active, &n_forced);
    const int cap = is_pair(p->potential) ? neighbor_capacity(p, mass, orig, n_active) : 0;
    *bytes = make_layout(p, n_active, n_forced, cap, excursion_guess(p, mass, orig, n_active)).total;
    return PIMD_OK;
}

int pimd_create(const pimd_params *p, const double *mass, const pimd_topology *topo,
                void *workspace, size_t workspace_bytes, void *stream, pimd_ctx **out)
{
    std::string why;
    int rc = validate(p, topo, why);
    if (rc != PIMD_OK) return fail(nullptr, rc, why);
    if (!out) return fail(nullptr, PIMD_ERR_ARG, "out is NULL");
    if (!mass) return fail(nullptr, PIMD_ERR_ARG, "mass is NULL");
    for (int i = 0; i < p->n_atoms; ++i)
        if (!finite_pos(mass[i])) return fail(nullptr, PIMD_ERR_ARG, "masses must be finite and > 0");
    if (p->bosonic)
        for (int i = 1; i < p->n_atoms; ++i)
            if (mass[i] != mass[0]) return fail(nullptr, PIMD_ERR_ARG, "bosons of one species: all masses equal");

    pimd_ctx *c = new (std::nothrow) pimd_ctx();
    if (!c) return fail(nullptr, PIMD_ERR_OOM, "host allocation failed");
    c->p = *p;
    c->graph_failed = (p->flags & PIMD_FLAG_NO_GRAPHS) != 0;
    int n_active = 0, n_forced = 0;
    c->orig = internal_order(p, topo, &n_active, &n_forced);
    const int N = p->n_atoms, P = p->n_beads;
    const bool pair = is_pair(p->potential);
    const int cap = pair ? neighbor_capacity(p, mass, c->orig, n_active) : 0;
    c->lay = make_layout(p, n_active, n_forced, cap, excursion_guess(p, mass, c->orig, n_active));
    const Layout &L = c->lay;

    auto cleanup = [&](int code, const std::string &msg) {
        if (c->own_ws && c->ws) (void)hipFree(c->ws);
        if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
        delete c;
        return fail(nullptr, code, msg);
    };

    if (workspace) {
        if (workspace_bytes < L.total)
            return cleanup(PIMD_ERR_OOM, "workspace smaller than pimd_workspace_bytes()");
        if (((uintptr_t)workspace & 255) != 0) return cleanup(PIMD_ERR_ARG, "workspace must be 256-byte aligned");
        c->ws = (char *)workspace;
    } else {
        hipError_t e = hipMalloc((void **)&c->ws, L.total);
        if (e != hipSuccess) {
            c->ws = nullptr;
            return cleanup(PIMD_ERR_OOM, std::string("hipMalloc: ") + hipGetErrorString(e));
        }
        c->own_ws = true;
    }
    if (stream) {
        c->stream = (hipStream_t)stream;
    } else {
        hipError_t e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
        if (e != hipSuccess) return cleanup(PIMD_ERR_DEVICE, std::string("hipStreamCreate: ") + hipGetErrorString(e));
        c->own_stream = true;
    }

    char *w = c->ws;
    c->d_x = (double *)(w + L.x);
    c->d_v = (double *)(w + L.v);
    // forces live in d_f for the pair potentials and for the caller's forces
    c->d_f = forces_in_array(p) ? (double *)(w + L.f) : nullptr;
    c->d_stage = (double *)(w + L.stage);
    c->d_cent = (double *)(w + L.cent);
    c->d_cref = (double *)(w + L.cref);
    c->d_M = (double *)(w + L.M);
    c->d_MT = (double *)(w + L.MT);
    c->d_modes = (double *)(w + L.modes);
    c->d_atoms = (double *)(w + L.atoms);
    c->d_mass = (double *)(w + L.mass);
    c->d_orig = (int *)(w + L.orig);
    c->d_bond_j = pair ? (int *)(w + L.bond_j) : nullptr;
    c->d_nbr_count = pair ? (int *)(w + L.nbr_count) : nullptr;
    c->d_nbr = pair ? (int2 *)(w + L.nbr) : nullptr;
    c->d_partials = (double *)(w + L.partials);
    c->d_fpartials = (double *)(w + L.fpartials);
    c->d_ctl = (Ctl *)(w + L.ctl);

    // tables in internal order
    std::vector<double> M = nm_matrix(P), modes = mode_table(p);
    if (p->bosonic) {
        // Cartesian bead velocities: the export's p = m M^T v needs M = 1
        std::fill(M.begin(), M.end(), 0.0);
        for (int k = 0; k < P; ++k) M[(size_t)k * P + k] = 1.0;
    }
    std::vector<double> MT((size_t)P * P);
    for (int k = 0; k < P; ++k)
        for (int j = 0; j < P; ++j) MT[(size_t)j * P + k] = M[(size_t)k * P + j];
    std::vector<double> atoms((size_t)N * 4), m_int(N);
    const double kT = p->kB * p->temp;
    const int32_t *act = (p->potential == PIMD_POT_WATER && topo) ? topo->lj_active : nullptr;
    for (int q = 0; q < N; ++q) {
        const int i = c->orig[q];
        const double m = mass[i];
        m_int[q] = m;
        atoms[(size_t)q * 4 + AT_HALF_M] = 0.5 * m * p->mvv2e;
        atoms[(size_t)q * 4 + AT_INV_M] = 1.0 / (m * p->mvv2e);
        atoms[(size_t)q * 4 + AT_SIGMA] = std::sqrt((double)P * kT / (m * p->mvv2e));
        atoms[(size_t)q * 4 + AT_ACTIVE] = (pair && (!act || act[i])) ? 1.0 : 0.0;
    }
    std::vector<int> bond_j;
    if (pair) {
        std::vector<int> inv(N);
        for (int q = 0; q < N; ++q) inv[c->orig[q]] = q;
        bond_j.assign((size_t)N * kMaxBonds, -1);
        std::vector<int> deg(N, 0);
        // a bond-owned atom (internal index >= n_forced) is flagged in its
        // partner's entry: the partner's lanes write its force
        if (p->potential == PIMD_POT_WATER && topo)
            for (int b = 0; b < topo->n_bonds; ++b) {
                const int i = inv[topo->bonds[2 * b]], j = inv[topo->bonds[2 * b + 1]];
                bond_j[(size_t)i * kMaxBonds + deg[i]++] = j >= L.n_forced ? (j | kBondOwned) : j;
                bond_j[(size_t)j * kMaxBonds + deg[j]++] = i >= L.n_forced ? (i | kBondOwned) : i;
            }
    }
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = hipMemcpy(c->d_M, M.data(), M.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->d_MT, MT.data(), MT.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->d_modes, modes.data(), modes.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->d_atoms, atoms.data(), atoms.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->d_mass, m_int.data(), m_int.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->d_orig, c->orig.data(), c->orig.size() * sizeof(int), hipMemcpyHostToDevice);
    if (e == hipSuccess && pair)
        e = hipMemcpy(c->d_bond_j, bond_j.data(), bond_j.size() * sizeof(int), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(c->d_cref, 0, (size_t)N * 3 * sizeof(double));
    if (e == hipSuccess) e = hipMemset(c->d_cent, 0, (size_t)N * 3 * sizeof(double));
    if (e == hipSuccess && pair) e = hipMemset(c->d_nbr_count, 0, (size_t)N * sizeof(int));
    if (e == hipSuccess) e = hipMemset(c->d_ctl, 0, sizeof(Ctl));
    if (e == hipSuccess && p->bosonic) {
        // no potential: the force array stays zero, one zero energy partial
        e = hipMemset(c->d_f, 0, (size_t)N * 3 * P * sizeof(double));
        if (e == hipSuccess) e = hipMemset(c->d_fpartials, 0, 2 * sizeof(double));
        if (e == hipSuccess) e = hipMemset(w + L.fs, 0, (size_t)N * 3 * P * sizeof(double));
        if (e == hipSuccess) e = hipMemset(w + L.bres, 0, 2 * sizeof(double));
    }
    if (e == hipSuccess && L.ncell)
        e = hipMemset(w + L.cell_scnt, 0, (size_t)L.ncell * sizeof(int));
    if (e != hipSuccess) return cleanup(PIMD_ERR_DEVICE, std::string("table upload: ") + hipGetErrorString(e));

    if (forces_in_array(p) && !c->d_f)
        return cleanup(PIMD_ERR_DEVICE, "internal: no force array for a potential that needs one");
    if (L.n_clusters) set_pair_smem();
    FusedArgs &a = c->fa;
    a.N = N; a.P = P; a.n_active = n_active;
    a.mode = FUSED_STEP;
    a.pair = forces_in_array(p) ? 1 : 0;
    a.lists = pair ? 1 : 0;
    a.nvt = thermostatted(p) ? 1 : 0;
    a.obabo = p->integrator == PIMD_OBABO ? 1 : 0;
    a.fixcom = p->fixcom ? 1 : 0;
    {
        double hsum = 0.0;
        for (int i = 0; i < N; ++i) hsum += atoms[(size_t)i * 4 + AT_HALF_M];
        a.inv_hsum = hsum > 0.0 ? 1.0 / hsum : 0.0;
    }
    a.hdt = 0.5 * p->dt;
    a.omega2 = p->potential == PIMD_POT_HARMONIC ? p->omega * p->omega : 0.0;
    a.skin = p->skin;
    a.rc = p->lj_rc;
    a.kT15N = 1.5 * (double)N * kT;
    a.kT15PN = 1.5 * (double)P * (double)N * kT;
    a.temp_norm = 2.0 / (3.0 * (double)N * (double)P * (double)P * p->kB);
    {
        const double V = p->box[0] * p->box[1] * p->box[2];
        a.inv_3v = (pair && V > 0.0) ? 1.0 / (3.0 * V) : 0.0;
    }
    a.seed = p->seed;
    a.x = c->d_x; a.yt = (double *)(w + L.yt); a.v = c->d_v; a.f = c->d_f; a.vin = c->d_f;
    a.cent = c->d_cent; a.cref = c->d_cref;
    a.M = c->d_M; a.MT = c->d_MT; a.modes = c->d_modes; a.atoms = c->d_atoms; a.orig = c->d_orig;
    a.partials = c->d_partials;
    a.fpartials = c->d_fpartials;
    // the force pass's energy partials; external forces bring one total
    a.n_fpartials = p->potential == PIMD_POT_EXTERNAL ? 1 : L.pair_grid;
    a.boson = p->bosonic ? 1 : 0;
    a.fs = p->bosonic ? (const double *)(w + L.fs) : nullptr;
    a.bres = p->bosonic ? (const double *)(w + L.bres) : nullptr;
    if (p->bosonic) {
        a.n_fpartials = L.pair_grid > 0 ? L.pair_grid : (L.trap_grid > 0 ? L.trap_grid : 1);
        a.inv_3v = 0.0;                 // no pressures for bosons
        BosonArgs &ba = c->ba;
        ba = BosonArgs{};
        ba.x = c->d_x;
        ba.N = N;
        ba.P = P;
        ba.layout = 1;
        const double wn = (double)P * kT / p->hbar;
        ba.ks = 0.5 * mass[0] * p->mvv2e * wn * wn;
        ba.bn = 1.0 / ((double)P * kT);
        for (int d = 0; d < 3; ++d) ba.box[d] = p->box[d] > 0.0 ? p->box[d] : 0.0;
        ba.f = (double *)(w + L.fs);
        ba.prob = nullptr;
        ba.scr = (double *)(w + L.bscr);
        ba.res = (double *)(w + L.bres);
    }
    a.ctl = c->d_ctl;
    a.ncell = L.ncell;
    a.cell_cap = L.cell_cap;
    for (int d = 0; d < 3; ++d) {
        a.nc[d] = L.nc[d];
        a.box[d] = p->box[d];
        a.icw[d] = L.ncell ? (double)L.nc[d] / p->box[d] : 0.0;
    }
    a.cell_ent = L.ncell ? (CellEntry *)(w + L.cell_ent) : nullptr;
    a.cell_scnt = L.ncell ? (int *)(w + L.cell_scnt) : nullptr;
    a.cinfo = L.ncell ? (int4 *)(w + L.cinfo) : nullptr;

    PairArgs &q = c->pa;
    q.N = N; q.P = P; q.n_active = n_active; q.cap = L.cap;
    q.n_forced = L.n_forced;
    q.S = L.pair_S;
    q.paired = pair_lanes_paired(N, P) ? 1 : 0;
    q.n_active_tiles = L.pair_active_tiles;
    for (int d = 0; d < 3; ++d) q.box[d] = p->box[d];
    q.rc2 = p->lj_rc * p->lj_rc;
    q.lj_eps = p->lj_eps;
    q.lj_sig2 = p->lj_sigma * p->lj_sigma;
    {
        const double sr2 = q.lj_sig2 / q.rc2, sr6 = sr2 * sr2 * sr2;
        q.lj_ushift = 4.0 * p->lj_eps * (sr6 * sr6 - sr6);
    }
    q.bond_k = (p->potential == PIMD_POT_WATER) ? p->bond_k : 0.0;
    q.bond_r0 = p->bond_r0;
    q.x = c->d_x; q.f = c->d_f; q.cent = c->d_cent; q.cref = c->d_cref;
    q.nbr_count = c->d_nbr_count; q.nbr = c->d_nbr; q.bond_j = c->d_bond_j;
    q.fpartials = c->d_fpartials;
    q.ctl = c->d_ctl;
    for (int d = 0; d < 3; ++d) q.nc[d] = L.nc[d];
    q.cell_cap = L.cell_cap;
    q.cell_ent = a.cell_ent;
    q.n_clusters = L.n_clusters;
    q.ccap = kClusterMax;
    q.clist = L.n_clusters ? (int4 *)(w + L.clist) : nullptr;
    q.ccount = L.n_clusters ? (int *)(w + L.ccount) : nullptr;
    q.cframe = L.n_clusters ? (int *)(w + L.cframe) : nullptr;
    q.cmode = L.n_clusters ? (int *)(w + L.cmode) : nullptr;
    q.cell_scnt = a.cell_scnt;
    q.cinfo = a.cinfo;

    if (L.npt_grid) {
        for (int d = 0; d < 3; ++d) c->start_box[d] = p->box[d];
        NptArgs &b = c->na;
        b.f = c->fa;
        b.ft = (double *)(w + L.nft);
        b.part = (double *)(w + L.npart);
        b.aniso = p->baro_aniso;
        b.fdiag = p->baro_aniso ? (double *)(w + L.fdiag) : nullptr;
        q.fdiag = p->baro_aniso ? (double *)(w + L.fdiag) : nullptr;
        b.dt = p->dt;
        b.p_ext = p->p_ext;
        const double kT = p->kB * p->temp;
        b.kTP = (double)P * kT;
        b.wmass = 3.0 * (double)P * (double)N * kT * p->tau_p * p->tau_p;
        // v_W's O step: over dt/2 (twice per step) in OBABO, over dt in BAOAB
        const double to = p->integrator == PIMD_OBABO ? 0.5 * p->dt : p->dt;
        b.bc1 = p->ensemble == PIMD_NPT ? std::exp(-to / p->tau) : 1.0;
        b.bc2 = std::sqrt(1.0 - b.bc1 * b.bc1);
        b.bsig = std::sqrt(b.kTP / b.wmass);
    }

    *out = c;
    return PIMD_OK;
}

int pimd_set_state(pimd_ctx *c, const double *x, const double *v, uint64_t step)
{
    if (!c) return fail(nullptr, PIMD_ERR_ARG, "ctx is NULL");
    if (!x || !v) return fail(c, PIMD_ERR_ARG, "x and v must be non-NULL");
    // the noise counter keeps the step in 63 bits (its top bit is the O step)
    if (step >> 63) return fail(c, PIMD_ERR_ARG, "step must be below 2^63");
    const int N = c->p.n_atoms, P = c->p.n_beads;
    const size_t n = (size_t)N * 3 * P;
    for (size_t e = 0; e < n; ++e)
        if (!std::isfinite(x[e]) || !std::isfinite(v[e])) return fail(c, PIMD_ERR_ARG, "non-finite x or v");
    // Positions and Cartesian velocities go through the staging buffer into
    // the device layout; PREP then turns v into v~ = M v in place (each tile
    // is staged in shared memory before it is overwritten).
    launch_ctl_init(c->d_ctl, (unsigned long long)step, c->stream);
    if (c->lay.npt_grid) launch_npt_init(c->d_ctl, c->start_box, c->start_vw, c->stream);
    HIP_TRY(c, hipMemcpyAsync(c->d_stage, x, n * sizeof(double), hipMemcpyHostToDevice, c->stream));
    launch_import(c->d_stage, c->d_x, c->d_orig, N, P, c->stream);
    HIP_TRY(c, hipMemcpyAsync(c->d_stage, v, n * sizeof(double), hipMemcpyHostToDevice, c->stream));
    launch_import(c->d_stage, c->d_v, c->d_orig, N, P, c->stream);
    FusedArgs a = c->fa;
    a.vin = c->d_v;
    a.mode = FUSED_PREP;
    // a barostat's box may differ from params.box (pimd_set_barostat): its
    // first lists come from the all-pairs scan, its cells from later rebuilds
    if (c->lay.npt_grid) a.ncell = 0;
    launch_fused(a, c->lay.fused_grid, c->stream);
    launch_finalize(a, c->lay.fused_grid, c->stream);
    const bool external = c->p.potential == PIMD_POT_EXTERNAL;
    if (c->lay.npt_grid) {
        launch_pair_npt(c->pa, c->lay.pair_grid, c->stream);
        launch_npt_a(c->na, NPT_EST, c->stream);
    } else {
        enqueue_forces(c);
    }
    if (!external && !c->lay.npt_grid) {
        // external forces: the estimators wait for the caller's forces
        a.mode = FUSED_EST;
        launch_fused(a, c->lay.fused_grid, c->stream);
        launch_finalize(a, c->lay.fused_grid, c->stream);
    }
    int rc = launch_error(c, "set_state launch");
    if (rc != PIMD_OK) return rc;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->have_state = true;
    c->forces_current = !external;
    c->synced = true;
    return PIMD_OK;
}

int pimd_step(pimd_ctx *c, int64_t nsteps)
{
    if (!c) return fail(nullptr, PIMD_ERR_ARG, "ctx is NULL");
    if (!c->have_state) return fail(c, PIMD_ERR_STATE, "pimd_step before pimd_set_state");
    if (nsteps < 0) return fail(c, PIMD_ERR_ARG, "nsteps < 0");
    if (nsteps == 0) return PIMD_OK;
    if (c->p.potential == PIMD_POT_EXTERNAL) {
        if (nsteps != 1) return fail(c, PIMD_ERR_ARG, "external forces: one step per call");
        if (!c->forces_current)
            return fail(c, PIMD_ERR_STATE, "external forces: pimd_set_forces for the current positions first");
        enqueue_step(c);
        c->forces_current = false;
        c->synced = false;
        return launch_error(c, "step launch");   // the closing (and fixcom) follow the forces
    }
    int64_t left = nsteps;
    if (left >= kGraphChunk && !c->graph_failed && !c->profiling) {
        if (!c->graph_exec) {
            hipError_t e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                for (int s = 0; s < kGraphChunk; ++s) enqueue_step(c);
                e = hipStreamEndCapture(c->stream, &c->graph);
            }
            if (e == hipSuccess) e = hipGraphInstantiate(&c->graph_exec, c->graph, nullptr, nullptr, 0);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                if (c->graph) (void)hipGraphDestroy(c->graph);
                c->graph = nullptr;
                c->graph_exec = nullptr;
                c->graph_failed = true;
            }
        }
        if (c->graph_exec) {
            while (left >= kGraphChunk) {
                HIP_TRY(c, hipGraphLaunch(c->graph_exec, c->stream));
                left -= kGraphChunk;
            }
        }
    }
    for (; left > 0; --left) enqueue_step(c);
    if (c->lay.npt_grid) {
        size_t e = prof_begin(c, PIMD_KERNEL_CLOSE);
        launch_npt_a(c->na, NPT_CLOSE, c->stream);
        prof_end(c, e);
    } else if (c->lay.pair_grid > 0 || c->p.bosonic) {
        // forces from arrays: the last step's closing kick and its estimators
        enqueue_fused(c, FUSED_CLOSE, PIMD_KERNEL_CLOSE);
    }
    // fixcom: the last step's centroid velocity is removed before the call ends
    if (c->fa.fixcom) launch_apply_ucom(c->fa, c->stream);
    return launch_error(c, "step launch");
}

int pimd_get_launch_info(const pimd_ctx *c, pimd_launch_info *out)
{
    if (!c || !out) return fail(nullptr, PIMD_ERR_ARG, "ctx or out is NULL");
    const Layout &L = c->lay;
    out->transforms = L.mfma_grid > 0 ? 1 : 0;
    out->fused_blocks = L.mfma_grid > 0 ? L.mfma_grid : L.fused_grid;
    out->pair_subgroups = L.pair_grid > 0 ? L.pair_S : 0;
    out->pair_blocks = L.pair_grid;
    out->cells = L.ncell;
    out->cluster_pairs = L.n_clusters > 0 ? 1 : 0;
    out->bead_pairs = (L.pair_grid > 0 && L.n_clusters == 0 && c->pa.paired) ? 1 : 0;
    return PIMD_OK;
}

int pimd_profile_begin(pimd_ctx *c)
{
    if (!c) return fail(nullptr, PIMD_ERR_ARG, "ctx is NULL");
    c->profiling = true;
    c->ev_used.clear();
    return PIMD_OK;
}

int pimd_profile_end(pimd_ctx *c, pimd_profile *out)
{
    if (!c) return fail(nullptr, PIMD_ERR_ARG, "ctx is NULL");
    if (!c->profiling) return fail(c, PIMD_ERR_STATE, "pimd_profile_end without pimd_profile_begin");
    c->profiling = false;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    pimd_profile r;
    for (int q = 0; q < PIMD_NKERNEL; ++q) { r.launches[q] = 0; r.ms[q] = 0.0; }
    for (const auto &u : c->ev_used) {
        float ms = 0.0f;
        HIP_TRY(c, hipEventElapsedTime(&ms, c->ev_pool[u.second], c->ev_pool[u.second + 1]));
        r.launches[u.first] += 1;
        r.ms[u.first] += ms;
    }
    c->ev_used.clear();
    if (out) *out = r;
    return PIMD_OK;
}

int pimd_get_estimators(pimd_ctx *c, pimd_estimators *out)
{
    if (!c) return fail(nullptr, PIMD_ERR_ARG, "ctx is NULL");
    if (!out) return fail(c, PIMD_ERR_ARG, "out is NULL");
    if (!c->have_state) return fail(c, PIMD_ERR_STATE, "no state");
    if (!c->forces_current)
        return fail(c, PIMD_ERR_STATE, "external forces: pimd_set_forces for the current positions first");
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    Ctl h;
    HIP_TRY(c, hipMemcpy(&h, c->d_ctl, sizeof(Ctl), hipMemcpyDeviceToHost));
    out->step = h.est_step;
    for (int q = 0; q < kNumEst; ++q) {
        out->value[q] = h.value[q];
        out->sum[q] = h.sum[q];
        out->sumsq[q] = h.sumsq[q];
    }
    out->count = h.count;
    out->nonfinite = h.nonfinite;
    out->overflow = h.overflow;
    out->n_rebuilds = h.n_rebuilds;
    out->rlist = h.rlist;
    const bool baro = c->lay.npt_grid > 0;
    out->volume = baro ? h.volume : 0.0;
    out->vw = baro ? (c->p.baro_aniso ? (h.vwa[0] + h.vwa[1] + h.vwa[2]) / 3.0 : h.vw) : 0.0;
    for (int d = 0; d < 3; ++d) out->vwa[d] = (baro && c->p.baro_aniso) ? h.vwa[d] : 0.0;
    out->enthalpy = baro ? h.enthalpy : 0.0;
    if (h.nonfinite) return fail(c, PIMD_ERR_NONFINITE, "non-finite position or velocity");
    if (h.overflow) return fail(c, PIMD_ERR_OVERFLOW, "neighbor list capacity exceeded");
    return PIMD_OK;
}

}  // extern "C"

extern "C" {

int pimd_get_barostat(pimd_ctx *c, double *box, double *vw)
{
    if (!c) return fail(nullptr, PIMD_ERR_ARG, "ctx is NULL");
    if (!c->lay.npt_grid) return fail(c, PIMD_ERR_UNSUPPORTED, "no barostat (ensemble is not NPT or NPH)");
    if (!c->have_state) return fail(c, PIMD_ERR_STATE, "no state");
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    Ctl h;
    HIP_TRY(c, hipMemcpy(&h, c->d_ctl, sizeof(Ctl), hipMemcpyDeviceToHost));
    if (box)
        for (int d = 0; d < 3; ++d) box[d] = h.box[d];
    if (vw) {
        if (c->p.baro_aniso)
            for (int d = 0; d < 3; ++d) vw[d] = h.vwa[d];
        else
            *vw = h.vw;
    }
    return PIMD_OK;
}

int pimd_set_barostat(pimd_ctx *c, const double *box, const double *vw)
{
    if (!c) return fail(nullptr, PIMD_ERR_ARG, "ctx is NULL");
    if (!c->lay.npt_grid) return fail(c, PIMD_ERR_UNSUPPORTED, "no barostat (ensemble is not NPT or NPH)");
    const bool an = c->p.baro_aniso != 0;
    bool ok = box != nullptr;
    for (int d = 0; ok && d < 3; ++d) ok = finite_pos(box[d]);
    if (!an) {
        // the isotropic barostat scales all three lengths together: the
        // aspect ratio stays that of params.box
        const double g = ok ? box[0] / c->p.box[0] : 0.0;
        for (int d = 1; ok && d < 3; ++d) ok = std::fabs(box[d] / c->p.box[d] - g) <= 1e-9 * g;
        if (!ok) return fail(c, PIMD_ERR_ARG, "box must hold lengths > 0 in the aspect ratio of params.box");
    } else if (!ok) {
        return fail(c, PIMD_ERR_ARG, "box must hold three lengths > 0");
    }
    const int nv = an ? 3 : 1;
    bool okv = vw != nullptr;
    for (int d = 0; okv && d < nv; ++d) okv = std::isfinite(vw[d]);
    if (!okv) return fail(c, PIMD_ERR_ARG, "vw must be non-NULL and finite");
    for (int d = 0; d < 3; ++d) c->start_box[d] = box[d];
    for (int d = 0; d < 3; ++d) c->start_vw[d] = d < nv ? vw[d] : 0.0;
    return PIMD_OK;
}

int pimd_get_state(pimd_ctx *c, double *x, double *p, uint64_t *step)
{
    if (!c) return fail(nullptr, PIMD_ERR_ARG, "ctx is NULL");
    if (!c->have_state) return fail(c, PIMD_ERR_STATE, "no state");
    if (p && !c->synced)
        return fail(c, PIMD_ERR_STATE, "external forces: momenta need pimd_set_forces for the current positions");
    const int N = c->p.n_atoms, P = c->p.n_beads;
    const size_t n = (size_t)N * 3 * P;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (x) {
        launch_export(c->d_x, c->d_v, c->d_mass, c->d_M, c->d_orig, c->d_stage, nullptr, N, P, c->stream);
        int rc = launch_error(c, "export");
        if (rc != PIMD_OK) return rc;
        HIP_TRY(c, hipMemcpyAsync(x, c->d_stage, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
    }
    if (p) {
        launch_export(c->d_x, c->d_v, c->d_mass, c->d_M, c->d_orig, nullptr, c->d_stage, N, P, c->stream);
        int rc = launch_error(c, "export");
        if (rc != PIMD_OK) return rc;
        HIP_TRY(c, hipMemcpyAsync(p, c->d_stage, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
    }
    if (step) {
        Ctl h;
        HIP_TRY(c, hipMemcpy(&h, c->d_ctl, sizeof(Ctl), hipMemcpyDeviceToHost));
        *step = h.step;
    }
    return PIMD_OK;
}

int pimd_get_positions(pimd_ctx *c, double *x)
{
    if (!c) return fail(nullptr, PIMD_ERR_ARG, "ctx is NULL");
    if (!x) return fail(c, PIMD_ERR_ARG, "x is NULL");
    if (!c->have_state) return fail(c, PIMD_ERR_STATE, "no state");
    launch_export(c->d_x, c->d_v, c->d_mass, c->d_M, c->d_orig, x, nullptr, c->p.n_atoms, c->p.n_beads,
                  c->stream);
    return launch_error(c, "get_positions");
}

int pimd_set_forces(pimd_ctx *c, const double *f, double epot)
{
    if (!c) return fail(nullptr, PIMD_ERR_ARG, "ctx is NULL");
    if (c->p.potential != PIMD_POT_EXTERNAL)
        return fail(c, PIMD_ERR_STATE, "pimd_set_forces needs the external potential");
    if (!c->have_state) return fail(c, PIMD_ERR_STATE, "no state");
    if (!f) return fail(c, PIMD_ERR_ARG, "f is NULL");
    if (!std::isfinite(epot)) return fail(c, PIMD_ERR_ARG, "epot is not finite");
    if (!c->d_f || !c->d_fpartials) return fail(c, PIMD_ERR_STATE, "internal: no force array");
    launch_import(f, c->d_f, c->d_orig, c->p.n_atoms, c->p.n_beads, c->stream);
    launch_store_energy(c->d_fpartials, epot, c->stream);
    // a pending closing kick and the estimators of this state (or, right after
    // set_state, the estimators alone)
    enqueue_fused(c, c->synced ? FUSED_EST : FUSED_CLOSE, PIMD_KERNEL_CLOSE);
    if (c->fa.fixcom) launch_apply_ucom(c->fa, c->stream);
    c->forces_current = true;
    c->synced = true;
    return launch_error(c, "set_forces launch");
}

int pimd_reset_averages(pimd_ctx *c)
{
    if (!c) return fail(nullptr, PIMD_ERR_ARG, "ctx is NULL");
    if (!c->have_state) return fail(c, PIMD_ERR_STATE, "no state");
    launch_ctl_reset_sums(c->d_ctl, c->stream);
    return launch_error(c, "reset_averages");
}

void pimd_destroy(pimd_ctx *c)
{
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    if (c->own_ws && c->ws) (void)hipFree(c->ws);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

const char *pimd_last_error(const pimd_ctx *c)
{
    return c ? c->err.c_str() : g_create_error.c_str();
}

}  // extern "C"

// ===========================================================================
// Batched execution
// ===========================================================================
struct pimd_batch {
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::vector<pimd_ctx *> sys;     // nullptr: removed
    std::vector<char> active;        // has a state
    // device plan
    FusedArgs *d_fa = nullptr;
    PairArgs *d_pa = nullptr;
    int *d_nparts = nullptr;         // [2][n]: step pass, closing pass
    int2 *d_items = nullptr;
    size_t cap_sys = 0, cap_items = 0;
    struct Group {
        int P;        // bead count (MFMA groups) or 0 (vector-ALU group)
        int obabo;    // MFMA groups: the systems' splitting (1: OBABO)
        int off, n;   // items [off, off + n)
    };
    std::vector<Group> step_groups;
    int pair_off = 0, pair_n = 0, pair1_off = 0, pair1_n = 0, close_off = 0, close_n = 0, n_sys_plan = 0;
    int smem_valu = 0;   // dynamic LDS of the batched vector-ALU pass: max over its systems
    bool pair_clusters = false;   // some system's force pass uses cluster lists
    int ncu = 256;
    bool dirty = true;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    bool graph_failed = false;
    std::string err = "no error";
};

namespace {

constexpr int kBatchGraphChunk = 16;

int bfail(pimd_batch *b, int code, const std::string &msg)
{
    if (b) b->err = msg;
    else g_create_error = msg;
    return code;
}

#define BHIP_TRY(b, expr)                                                             \
    do {                                                                              \
        hipError_t e_ = (expr);                                                       \
        if (e_ != hipSuccess)                                                         \
            return bfail((b), PIMD_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

bool valid_sys(const pimd_batch *b, int32_t s)
{
    return b && s >= 0 && (size_t)s < b->sys.size() && b->sys[s] != nullptr;
}

void drop_graph(pimd_batch *b)
{
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->gexec = nullptr;
    b->graph = nullptr;
}

int grow(pimd_batch *b, void **ptr, size_t *cap, size_t need, size_t elem)
{
    if (need <= *cap && *ptr) return PIMD_OK;
    size_t n = std::max<size_t>(need, 2 * *cap);
    if (n == 0) n = 1;
    if (*ptr) (void)hipFree(*ptr);
    *ptr = nullptr;
    BHIP_TRY(b, hipMalloc(ptr, n * elem));
    *cap = n;
    return PIMD_OK;
}

int cu_count()
{
    int dev = 0, ncu = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess) ncu = prop.multiProcessorCount;
    }
    return ncu;
}

// Rebuild the device tables and work lists from the active systems.
int rebuild_plan(pimd_batch *b)
{
    BHIP_TRY(b, hipStreamSynchronize(b->stream));
    drop_graph(b);
    const int n = (int)b->sys.size();
    std::vector<FusedArgs> fa(std::max(n, 1));
    std::vector<PairArgs> pa(std::max(n, 1));
    std::vector<int> nparts(2 * std::max(n, 1), 0);
    std::vector<int2> items;
    b->step_groups.clear();
    b->smem_valu = 0;
    for (int s = 0; s < n; ++s) {
        if (b->sys[s]) {
            fa[s] = b->sys[s]->fa;
            pa[s] = b->sys[s]->pa;
        }
    }
    // MFMA groups by bead count and splitting, then the vector-ALU group
    for (int P : {16, 32, 64})
        for (int ob = 0; ob < 2; ++ob) {
            pimd_batch::Group g{P, ob, (int)items.size(), 0};
            for (int s = 0; s < n; ++s) {
                pimd_ctx *c = b->sys[s];
                if (!c || !b->active[s] || c->p.n_beads != P || c->lay.mfma_grid == 0 ||
                    c->fa.obabo != ob)
                    continue;
                for (int t = 0; t < c->lay.mfma_tiles; ++t) items.push_back(make_int2(s, t));
                nparts[s] = c->lay.mfma_tiles;
            }
            g.n = (int)items.size() - g.off;
            if (g.n) b->step_groups.push_back(g);
        }
    {
        pimd_batch::Group g{0, 0, (int)items.size(), 0};
        for (int s = 0; s < n; ++s) {
            pimd_ctx *c = b->sys[s];
            if (!c || !b->active[s] || c->lay.mfma_grid != 0) continue;
            for (int t = 0; t < c->lay.valu_tiles; ++t) items.push_back(make_int2(s, t));
            nparts[s] = c->lay.valu_tiles;
            b->smem_valu = std::max(b->smem_valu, fused_smem_bytes(c->p.n_beads));
        }
        g.n = (int)items.size() - g.off;
        if (g.n) b->step_groups.push_back(g);
    }
    // force items: the systems whose lanes take bead pairs, then the others
    b->pair_clusters = false;
    for (int pass = 0; pass < 2; ++pass) {
        const int off = (int)items.size();
        for (int s = 0; s < n; ++s) {
            pimd_ctx *c = b->sys[s];
            if (!c || !b->active[s] || !c->fa.pair || (c->pa.paired != 0) != (pass == 0)) continue;
            for (int t = 0; t < c->lay.pair_grid; ++t) items.push_back(make_int2(s, t));
            if (c->lay.n_clusters) b->pair_clusters = true;
        }
        (pass == 0 ? b->pair_off : b->pair1_off) = off;
        (pass == 0 ? b->pair_n : b->pair1_n) = (int)items.size() - off;
    }
    b->close_off = (int)items.size();
    for (int s = 0; s < n; ++s) {
        pimd_ctx *c = b->sys[s];
        if (!c || !b->active[s] || !c->fa.pair) continue;
        for (int t = 0; t < c->lay.valu_tiles; ++t) items.push_back(make_int2(s, t));
        nparts[n + s] = c->lay.valu_tiles;
        b->smem_valu = std::max(b->smem_valu, fused_smem_bytes(c->p.n_beads));
    }
    b->close_n = (int)items.size() - b->close_off;
    b->n_sys_plan = n;
    int rc;
    if (!b->d_fa || fa.size() > b->cap_sys) {
        // the three per-system tables always share one capacity
        const size_t cap = std::max(fa.size(), 2 * b->cap_sys);
        if (b->d_fa) (void)hipFree(b->d_fa);
        if (b->d_pa) (void)hipFree(b->d_pa);
        if (b->d_nparts) (void)hipFree(b->d_nparts);
        b->d_fa = nullptr; b->d_pa = nullptr; b->d_nparts = nullptr; b->cap_sys = 0;
        BHIP_TRY(b, hipMalloc((void **)&b->d_fa, cap * sizeof(FusedArgs)));
        BHIP_TRY(b, hipMalloc((void **)&b->d_pa, cap * sizeof(PairArgs)));
        BHIP_TRY(b, hipMalloc((void **)&b->d_nparts, 2 * cap * sizeof(int)));
        b->cap_sys = cap;
    }
    if ((rc = grow(b, (void **)&b->d_items, &b->cap_items, std::max<size_t>(items.size(), 1), sizeof(int2))) != PIMD_OK)
        return rc;
    BHIP_TRY(b, hipMemcpy(b->d_fa, fa.data(), fa.size() * sizeof(FusedArgs), hipMemcpyHostToDevice));
    BHIP_TRY(b, hipMemcpy(b->d_pa, pa.data(), pa.size() * sizeof(PairArgs), hipMemcpyHostToDevice));
    BHIP_TRY(b, hipMemcpy(b->d_nparts, nparts.data(), nparts.size() * sizeof(int), hipMemcpyHostToDevice));
    if (!items.empty())
        BHIP_TRY(b, hipMemcpy(b->d_items, items.data(), items.size() * sizeof(int2), hipMemcpyHostToDevice));
    set_batch_smem(b->smem_valu);
    set_mfma_batch_smem();
    b->ncu = cu_count();
    b->dirty = false;
    return PIMD_OK;
}

void enqueue_batch_step(pimd_batch *b)
{
    const int ncu = b->ncu;
    for (const auto &g : b->step_groups) {
        if (g.P)
            launch_fused_mfma_batch(g.P, g.obabo != 0, b->d_fa, b->d_items + g.off, g.n, g.n, b->stream);
        else
            launch_fused_batch(b->d_fa, b->d_items + g.off, g.n, FUSED_STEP, b->smem_valu,
                               std::min(g.n, 2 * ncu), b->stream);
    }
    launch_finalize_batch(b->d_fa, b->d_nparts, b->n_sys_plan, FUSED_STEP, b->stream);
    if (b->pair_n)
        launch_pair_batch(b->d_pa, b->d_items + b->pair_off, b->pair_n, std::min(b->pair_n, 8 * ncu),
                          b->pair_clusters, true, b->stream);
    if (b->pair1_n)
        launch_pair_batch(b->d_pa, b->d_items + b->pair1_off, b->pair1_n,
                          std::min(b->pair1_n, 8 * ncu), b->pair_clusters, false, b->stream);
}

}  // namespace

extern "C" {

int pimd_batch_create(void *stream, pimd_batch **out)
{
    if (!out) return bfail(nullptr, PIMD_ERR_ARG, "out is NULL");
    pimd_batch *b = new (std::nothrow) pimd_batch();
    if (!b) return bfail(nullptr, PIMD_ERR_OOM, "host allocation failed");
    if (stream) {
        b->stream = (hipStream_t)stream;
    } else {
        hipError_t e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            delete b;
            return bfail(nullptr, PIMD_ERR_DEVICE, std::string("hipStreamCreate: ") + hipGetErrorString(e));
        }
        b->own_stream = true;
    }
    *out = b;
    return PIMD_OK;
}

int pimd_batch_add(pimd_batch *b, const pimd_params *p, const double *mass, const pimd_topology *topo,
                   int32_t *sys)
{
    if (!b || !sys || !p) return bfail(b, PIMD_ERR_ARG, "NULL argument");
    if (p->potential == PIMD_POT_EXTERNAL)
        return bfail(b, PIMD_ERR_UNSUPPORTED, "external forces are not batched (the caller steps each system)");
    if (p->fixcom) return bfail(b, PIMD_ERR_UNSUPPORTED, "fixcom is not batched");
    if (is_npt(p)) return bfail(b, PIMD_ERR_UNSUPPORTED, "the barostat is not batched");
    if (p->bosonic) return bfail(b, PIMD_ERR_UNSUPPORTED, "bosons are not batched");
    pimd_ctx *c = nullptr;
    int rc = pimd_create(p, mass, topo, nullptr, 0, (void *)b->stream, &c);
    if (rc != PIMD_OK) return bfail(b, rc, pimd_last_error(nullptr));
    int id = -1;
    for (size_t s = 0; s < b->sys.size(); ++s)
        if (!b->sys[s]) { id = (int)s; break; }
    if (id < 0) {
        id = (int)b->sys.size();
        b->sys.push_back(nullptr);
        b->active.push_back(0);
    }
    b->sys[id] = c;
    b->active[id] = 0;
    b->dirty = true;
    *sys = id;
    return PIMD_OK;
}

int pimd_batch_remove(pimd_batch *b, int32_t s)
{
    if (!valid_sys(b, s)) return bfail(b, PIMD_ERR_ARG, "unknown system id");
    BHIP_TRY(b, hipStreamSynchronize(b->stream));
    pimd_destroy(b->sys[s]);
    b->sys[s] = nullptr;
    b->active[s] = 0;
    b->dirty = true;
    return PIMD_OK;
}

int pimd_batch_set_state(pimd_batch *b, int32_t s, const double *x, const double *v, uint64_t step)
{
    if (!valid_sys(b, s)) return bfail(b, PIMD_ERR_ARG, "unknown system id");
    int rc = pimd_set_state(b->sys[s], x, v, step);
    if (rc != PIMD_OK) return bfail(b, rc, b->sys[s]->err);
    if (!b->active[s]) b->dirty = true;
    b->active[s] = 1;
    return PIMD_OK;
}

int pimd_batch_set_budget(pimd_batch *b, int32_t s, int64_t steps)
{
    if (!valid_sys(b, s)) return bfail(b, PIMD_ERR_ARG, "unknown system id");
    if (!b->active[s]) return bfail(b, PIMD_ERR_STATE, "system has no state");
    if (steps < -1) return bfail(b, PIMD_ERR_ARG, "budget must be >= -1");
    launch_ctl_set_budget(b->sys[s]->d_ctl, (long long)steps, b->stream);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return bfail(b, PIMD_ERR_DEVICE, hipGetErrorString(e));
    return PIMD_OK;
}

int pimd_batch_step(pimd_batch *b, int64_t nsteps)
{
    if (!b) return bfail(nullptr, PIMD_ERR_ARG, "batch is NULL");
    if (nsteps < 0) return bfail(b, PIMD_ERR_ARG, "nsteps < 0");
    if (nsteps == 0) return PIMD_OK;
    if (b->dirty) {
        int rc = rebuild_plan(b);
        if (rc != PIMD_OK) return rc;
    }
    if (b->step_groups.empty()) return PIMD_OK;
    int64_t left = nsteps;
    if (left >= kBatchGraphChunk && !b->graph_failed) {
        if (!b->gexec) {
            hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                for (int s = 0; s < kBatchGraphChunk; ++s) enqueue_batch_step(b);
                e = hipStreamEndCapture(b->stream, &b->graph);
            }
            if (e == hipSuccess) e = hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                drop_graph(b);
                b->graph_failed = true;
            }
        }
        if (b->gexec) {
            while (left >= kBatchGraphChunk) {
                BHIP_TRY(b, hipGraphLaunch(b->gexec, b->stream));
                left -= kBatchGraphChunk;
            }
        }
    }
    for (; left > 0; --left) enqueue_batch_step(b);
    if (b->close_n) {
        launch_fused_batch(b->d_fa, b->d_items + b->close_off, b->close_n, FUSED_CLOSE, b->smem_valu,
                           std::min(b->close_n, 2 * b->ncu), b->stream);
        launch_finalize_batch(b->d_fa, b->d_nparts + b->n_sys_plan, b->n_sys_plan, FUSED_CLOSE, b->stream);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return bfail(b, PIMD_ERR_DEVICE, std::string("batch step: ") + hipGetErrorString(e));
    return PIMD_OK;
}

int pimd_batch_get_estimators(pimd_batch *b, int32_t s, pimd_estimators *out)
{
    if (!valid_sys(b, s)) return bfail(b, PIMD_ERR_ARG, "unknown system id");
    int rc = pimd_get_estimators(b->sys[s], out);
    if (rc != PIMD_OK) return bfail(b, rc, b->sys[s]->err);
    return PIMD_OK;
}

int pimd_batch_get_state(pimd_batch *b, int32_t s, double *x, double *p, uint64_t *step)
{
    if (!valid_sys(b, s)) return bfail(b, PIMD_ERR_ARG, "unknown system id");
    int rc = pimd_get_state(b->sys[s], x, p, step);
    if (rc != PIMD_OK) return bfail(b, rc, b->sys[s]->err);
    return PIMD_OK;
}

void pimd_batch_destroy(pimd_batch *b)
{
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    drop_graph(b);
    for (pimd_ctx *c : b->sys) pimd_destroy(c);
    if (b->d_fa) (void)hipFree(b->d_fa);
    if (b->d_pa) (void)hipFree(b->d_pa);
    if (b->d_nparts) (void)hipFree(b->d_nparts);
    if (b->d_items) (void)hipFree(b->d_items);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

const char *pimd_batch_last_error(const pimd_batch *b)
{
    return b ? b->err.c_str() : g_create_error.c_str();
}

}  // extern "C"
