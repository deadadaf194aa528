// Launch-shape table of libpimd.so.  Written by paper_2602_13553_amd/autotune.py
// from kernel timings on the GPU; regenerate with
//   python -m paper_2602_13553_amd.autotune --write
// (the sweep, its workloads and the raw timings are described there).
// Measured on AMD Radeon Graphics (gfx950:sramecc+:xnack-), 2026-12-03, 40 timed steps per point.
#pragma once

namespace pimd {
namespace tuning {

// Smallest N*P from which the matrix-core step pass is faster than the
// vector-ALU one, for P = 16, 32, 64.
constexpr long long kMfmaMinBeadAtoms[3] = {262144LL, 262144LL, 131072LL};

// Force-pass lane sub-groups per atom for P = 8, 16, 32, 64 (rows) and N in
// [2^6, 2^7), [2^7, 2^8), ..., [2^15, 2^16) (columns; clamped at both ends),
// for LJ liquids.  0: the occupancy heuristic decides.
constexpr int kPairSubgroups[4][10] = {
    {16, 16, 16, 16, 16, 8, 4, 4, 2, 1},
    {16, 8, 16, 8, 8, 4, 4, 2, 1, 1},
    {8, 8, 8, 8, 8, 4, 2, 1, 1, 1},
    {4, 4, 4, 4, 4, 2, 1, 1, 1, 1},
};

// The same for the water-shaped potential (O-O LJ plus O-H bonds).
constexpr int kPairSubgroupsWater[4][10] = {
    {16, 16, 16, 16, 16, 16, 16, 8, 4, 2},
    {16, 16, 16, 16, 16, 8, 8, 4, 2, 2},
    {8, 8, 8, 8, 8, 8, 4, 2, 2, 2},
    {4, 4, 4, 4, 4, 4, 2, 2, 2, 1},
};

// Force pass on cluster lists (1) or per-atom lists (0), same rows and
// columns as kPairSubgroups.  The sweep does not time cluster lists (they
// were slower than per-atom lists at every size measured), so they stay off.
constexpr int kClusterPairs[4][10] = {
    {0, 0, 0, 0, 0, 0, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 0, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 0, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 0, 0, 0, 0, 0},
};

}  // namespace tuning
}  // namespace pimd
