// zmc_kernels.hpp -- argument blocks and host-side launchers of the device
// pipeline that runs one level of the tree search over every resident
// integral:
//
//   sample      (cube, trial, chunk) units -> FP64 partial sums S1 = sum f,
//               S2 = sum f^2 over the chunk's points (one kernel per
//               (integrand, D, eval) bucket, persistent over its units)
//   finalize    per cube: I_t = V * S1_t / N, m = mean_t I_t, s = std_t I_t
//   seg_mean / tile_sqdev / seg_thr
//               per integral: thr = mean(s) + sigma_mult * std(s)
//   tile_select per cube: split = s > thr; accepted / selected sums per tile
//   seg_decide  per integral: totals, stop rules, rank base of every tile
//   spawn       2^D children of every split cube, in list order
//   roots       level-0 list of a newly admitted integral
//   level_small finalize .. seg_decide in one launch when every segment of
//               the level is a single tile
#pragma once

#include <hip/hip_runtime.h>

#include "zmc_device.hpp"

namespace zmc {

struct LevelArgs {
    const SlotDesc* slots;
    const Segment* segs;
    int32_t n_segs;
    int32_t fused;           // per-segment steps in the tile kernels' last blocks
    int64_t n_tiles;
    const uint64_t* uid;
    const uint32_t* uid_hi;  // id bits 64..83, or NULL (all zero)
    const double2* partial;
    double* m;
    double* s;
    uint8_t* sel;
    TileRec* tiles;
    SegStats* stats;
    const double2* prev_tot; // per segment: running (M, S2) before this level
    double* tr_S1;           // optional per (cube, trial) sums (trace)
    double* tr_S2;
    uint64_t* next_uid;      // spawn output
    uint32_t* next_uid_hi;   // spawn output: id bits 64..83, or NULL
    double* gthr;            // per-parent thresholds, one per sibling group
    int64_t n_groups;
    int32_t* seg_count;      // per segment: tile blocks done (0 between kernels)
    SegStats* host_stats;    // optional mapped host copy of the decisions
    const int32_t* seg_flags; // per segment: flags the sampling launches raised
};

struct RootArgs {
    const Segment* segs; // segments whose roots are written (cube_base, n_cubes)
    int32_t n_segs;
    int32_t blocks_per_seg;
    uint64_t* uid;
    uint32_t* uid_hi; // written 0 when not NULL
};

// Launchers; each returns the hipError_t of its launch.
// Occupancy variants of every sampling kernel: the minimum waves per SIMD
// the register allocator must allow (1 = no constraint).  More resident waves
// hide more of the Philox latency, until the registers they leave each wave
// make the allocator spill; which variant wins depends on the bucket.
constexpr int kWaveHints[] = {1, 5, 7, 8};
constexpr int kNumWaveHints = 4;
// hint value that selects the sampling kernel that also keeps the sums of
// squares (traced levels); it runs at the compiler's default occupancy
constexpr int kSumsVariant = kNumWaveHints;

// block: threads per sampling block, 64, 128 or 256 (whole waves; results
// do not depend on it: every unit is one wave's work)
hipError_t launch_sample(int integrand, int dim, int eval, int hint, int grid, int block, hipStream_t st,
                         const SampleArgs& a);
const void* sample_kernel_ptr(int integrand, int dim, int eval, int hint);
hipError_t launch_finalize(const LevelArgs& a, hipStream_t st);
// finalize + threshold + selection + decision of a level whose segments are
// all one tile without per-parent thresholds, one block per segment
hipError_t launch_level_small(const LevelArgs& a, hipStream_t st);
hipError_t launch_threshold(const LevelArgs& a, hipStream_t st);
hipError_t launch_group_threshold(const LevelArgs& a, hipStream_t st);
hipError_t launch_select(const LevelArgs& a, hipStream_t st);
// Spawn (a.n_tiles blocks, none when 0) and roots (ra.n_segs segments, none
// when 0) in one launch.
hipError_t launch_next_list(const LevelArgs& a, const RootArgs& ra, hipStream_t st);
hipError_t launch_debug_philox(uint32_t k0, uint32_t k1, const uint32_t* ctr, uint32_t* out, int64_t n,
                               hipStream_t st);
hipError_t launch_debug_points(const SlotDesc* sd, int level, uint64_t uid, int trial, int64_t s0, int64_t n,
                               double* x, hipStream_t st);

// Per-integrand launch tables (one translation unit per integrand).
#define ZMC_DECLARE_SAMPLE(F)                                                                              \
    hipError_t launch_sample_##F(int dim, int eval, int hint, int grid, int block, hipStream_t st,               \
                                 const SampleArgs& a);                                                             \
    const void* sample_kernel_ptr_##F(int dim, int eval, int hint);
ZMC_DECLARE_SAMPLE(0)
ZMC_DECLARE_SAMPLE(1)
ZMC_DECLARE_SAMPLE(2)
ZMC_DECLARE_SAMPLE(3)
ZMC_DECLARE_SAMPLE(4)
ZMC_DECLARE_SAMPLE(5)
ZMC_DECLARE_SAMPLE(6)
ZMC_DECLARE_SAMPLE(7)
#undef ZMC_DECLARE_SAMPLE

} // namespace zmc
