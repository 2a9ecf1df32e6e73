// zmc_device.hpp -- device-side building blocks of the integrator for gfx950:
// the counter-based RNG, the uniform mapping, the sub-domain geometry, the
// integrand registry in FP64 and in cube-relative FP32, and the shared data
// layouts of the level pipeline.
//
// Method: ZMCintegral (arXiv:1902.07916), Sec. 2.1 (stratified sampling and
// heuristic tree search) and Sec. 2.2 (random numbers produced at the time of
// use instead of stored batches).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "zmc.h"

namespace zmc {

constexpr int kMaxDim = ZMC_MAX_DIM;
constexpr int kMaxParams = ZMC_MAX_PARAMS;
constexpr int kTileCubes = 1024;   // cubes per tile of the per-cube kernels
constexpr int kLevelThreads = 256; // threads per block of the per-cube kernels

// ---------------------------------------------------------------------------
// Device-resident tables (structure of arrays where per-cube, small structs
// where per-integral or per-segment).
// ---------------------------------------------------------------------------

// One integral resident on the device (read-only while resident).
struct alignas(16) SlotDesc {
    int32_t integrand, dim, eval, divisions;
    int32_t trials, max_depth, nch, groups; // nch: sample chunks per trial; groups: 4-sample groups per thread per chunk
    int64_t samples, max_cubes;
    double sigma_mult, rtol;
    uint64_t seed;
    int32_t split;  // parts per axis of a split (2 = bisection)
    int32_t kids;   // split^dim children per split
    int32_t scope;  // 0: threshold per level; 1: per parent
    int32_t reserved;
    double lower[kMaxDim];
    double h0[kMaxDim]; // (upper - lower) / d, the root edge lengths
    double params[kMaxParams];
};

// A run of consecutive cubes of the current list that belong to one integral.
struct alignas(16) Segment {
    int32_t slot, level;
    int64_t cube_base, n_cubes;
    int64_t part_base;  // first of its partials, laid out [cube][trial * nch + chunk]
    int64_t tile_base;  // index of its first tile
    int64_t n_tiles;
    int64_t child_base; // where its children start in the next list
    int32_t do_split;   // 1: spawn its selected cubes' children
    int32_t need_thr;   // 1: a threshold is formed at this level
    int64_t group_base; // per-parent thresholds: index of its first sibling group
    int32_t group_size; // per-parent thresholds: cubes per sibling group (0: one threshold)
    int32_t pad;
};

// Sampling work of one (integrand, D, eval) bucket: segment `seg` owns the
// bucket-local units [unit_base, next unit_base).
struct alignas(16) BSeg {
    int64_t unit_base;
    int32_t seg;
    int32_t pad;
};

// Per-tile partial reductions of the per-cube kernels.
struct alignas(16) TileRec {
    double sum_s, sum_sq;
    double s_min, s_max; // extremes of the tile's s (for the scale of the std)
    double accM, accS2, selM, selS2;
    double min_margin;
    int64_t n_sel, sel_prefix;
    int32_t nonfinite, pad;
};

// Population standard deviations are computed with every deviation scaled
// by 2^-e before it is squared and the root scaled by 2^e after, e the
// binary exponent of the largest |deviation| (frexp).  Powers of two scale
// exactly: wherever the unscaled squares neither underflow nor overflow the
// result is the same bit for bit, and deviations below ~1e-154 (the tails of
// a narrow Gaussian) are not lost to underflow.
__device__ __forceinline__ int std_scale_exp(double dmax)
{
    int e = 0;
    if (isfinite(dmax) && dmax > 0.0) (void)frexp(dmax, &e);
    return e;
}

enum Decision : int32_t { kSplit = 0, kDone = 1, kTruncated = 2, kRtolMet = 3 };

// Arguments of one sampling launch (one (integrand, D, eval) bucket).
constexpr int kSampleThreads = 256; // the largest sampling block (launch bound); 64 and 128 are tunable

struct SampleArgs {
    const SlotDesc* slots;
    const Segment* segs;
    const BSeg* bsegs;
    int32_t n_bsegs;
    int32_t pad;
    int64_t unit0;       // first unit of this launch (units are numbered over the level's bucket)
    int64_t total_units; // units of this launch
    const uint64_t* uid;
    const uint32_t* uid_hi; // id bits 64..83 per cube; NULL when every id of the level is below 2^64
    double2* partial;
    int32_t* seg_flags;  // per segment of the level (0 at the level's start):
                         // kRangeLost when an FP32 unit's sum fell below
                         // FP32's normal range
};

// seg_flags / SegStats::range_lost: some sampling unit's FP32 values summed
// to less than (points of the unit) * 2^-126 in magnitude, i.e. they lay
// below FP32's normal range.
constexpr int32_t kRangeLost = 1;

// Per-segment outcome of one level, read back by the host after every level.
struct alignas(16) SegStats {
    double mu, sd, thr, min_margin;
    double s_min, s_max; // extremes of the segment's s
    double accM, accS2, selM, selS2;
    double totM, totS2; // running totals of the integral after this level
    int64_t n_sel;
    int32_t decision, nonfinite;
    int32_t range_lost, pad;
};

// ---------------------------------------------------------------------------
// Cube ids of up to 84 bits: bits 0..63 (lo) and 64..83 (hi).  Bits 64..83
// enter the RNG counter's word 1 above the trial and the level, so every id
// below 2^64 keeps the stream of a 64-bit id.
// ---------------------------------------------------------------------------
constexpr int kIdBits = 84;

__device__ __forceinline__ uint32_t ctr_word1(int trial, int level, uint32_t uid_hi)
{
    return (uint32_t)trial | ((uint32_t)level << 8) | (uid_hi << 12);
}

// Bits 0..63 of (hi:lo) >> k.
__device__ __forceinline__ uint64_t shr_id(uint64_t lo, uint32_t hi, int k)
{
    if (k >= kIdBits) return 0;
    if (k >= 64) return (uint64_t)hi >> (k - 64);
    if (k == 0) return lo;
    return (lo >> k) | ((uint64_t)hi << (64 - k));
}

// (hi:lo) /= k in place for 1 <= k < 2^32, returning the remainder: long
// division over 32-bit limbs with 64-bit intermediates.
__device__ __forceinline__ uint64_t divmod_id(uint64_t& lo, uint32_t& hi, uint64_t k)
{
    uint64_t r = 0;
    const uint64_t t2 = hi;
    const uint64_t q2 = t2 / k;
    r = t2 - q2 * k;
    const uint64_t t1 = (r << 32) | (lo >> 32);
    const uint64_t q1 = t1 / k;
    r = t1 - q1 * k;
    const uint64_t t0 = (r << 32) | (lo & 0xffffffffull);
    const uint64_t q0 = t0 / k;
    r = t0 - q0 * k;
    hi = (uint32_t)q2;
    lo = (q1 << 32) | q0;
    return r;
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64 products
// (constants 0xD2511F53, 0xCD9E8D57), the half-swapping S-box XORed with the
// round key, and the Weyl key schedule (0x9E3779B9, 0xBB67AE85).  On gfx950 a
// round is two v_mad_u64_u32 and two v_bitop3_b32 (three-input XOR, function
// 0x96); the key schedule is wave-uniform and stays on the scalar unit.
// ---------------------------------------------------------------------------
struct U4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ U4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                            uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)c0 * 0xD2511F53u;
        const uint64_t p1 = (uint64_t)c2 * 0xCD9E8D57u;
        const uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, k0);
        const uint32_t n2 = xor3((uint32_t)(p0 >> 32), c3, k1);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return U4{c0, c1, c2, c3};
}

// K Philox4x32-10 blocks whose counters differ only in word 0, computed in
// lockstep round by round: the 2K products of a round are independent, which
// hides the latency of v_mad_u64_u32 even at low occupancy, and the work on
// the shared (wave-uniform) counter words 1-3 in the first rounds is done
// once for all K blocks.  out[4*b + j] is word j of block b.
template <int K>
__device__ __forceinline__ void philox4x32_10_lockstep(const uint32_t (&c0)[K], uint32_t c1, uint32_t c2,
                                                       uint32_t c3, uint32_t k0, uint32_t k1, uint32_t (&out)[4 * K])
{
    uint32_t x0[K], x1[K], x2[K], x3[K];
#pragma unroll
    for (int b = 0; b < K; ++b) {
        x0[b] = c0[b];
        x1[b] = c1;
        x2[b] = c2;
        x3[b] = c3;
    }
#pragma unroll
    for (int r = 0; r < 10; ++r) {
#pragma unroll
        for (int b = 0; b < K; ++b) {
            const uint64_t p0 = (uint64_t)x0[b] * 0xD2511F53u;
            const uint64_t p1 = (uint64_t)x2[b] * 0xCD9E8D57u;
            const uint32_t n0 = xor3((uint32_t)(p1 >> 32), x1[b], k0);
            const uint32_t n2 = xor3((uint32_t)(p0 >> 32), x3[b], k1);
            x1[b] = (uint32_t)p1;
            x3[b] = (uint32_t)p0;
            x0[b] = n0;
            x2[b] = n2;
        }
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
#pragma unroll
    for (int b = 0; b < K; ++b) {
        out[4 * b + 0] = x0[b];
        out[4 * b + 1] = x1[b];
        out[4 * b + 2] = x2[b];
        out[4 * b + 3] = x3[b];
    }
}

// u = (2*(w>>9)+1) * 2^-24, exact in FP64.
__device__ __forceinline__ double uniform_f64(uint32_t w)
{
    return (double)((w >> 8) | 1u) * 0x1p-24;
}

// The same cell as uniform_f64 as a float in [1, 2): 1 + (w>>9) * 2^-23, so
// u = v - (1 - 2^-24).  One v_alignbit_b32 moves the top 23 bits of w under
// the exponent of 1.0f.
__device__ __forceinline__ float unit_interval_f32(uint32_t w)
{
    return __uint_as_float(__builtin_amdgcn_alignbit(0x7Fu, w, 9u));
}

// ---------------------------------------------------------------------------
// Geometry of cube (uid, level): lattice cell K_i on a grid of d*b^level
// cells per axis.  uid = root * (b^D)^level + path, one base-b^D digit per
// split, axis 0 the most significant base-b digit of each; for b = 2 this is
// uid' = (uid << D) | c with bit (D-1-i) of c choosing the upper half of
// axis i.  Edge lengths h = h0 / b^level (exact for b = 2).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double level_parts(int split, int level)
{
    uint64_t p = 1;
    for (int j = 0; j < level; ++j) p *= (uint64_t)split;
    return (double)p;
}

__device__ __forceinline__ void cube_corner(const SlotDesc& sd, int D, int level, uint64_t uid, double* lo,
                                            double* h)
{
    uint64_t K[kMaxDim];
    const uint64_t d = (uint64_t)sd.divisions;
    const uint64_t b = (uint64_t)sd.split;
    const uint64_t kids = (uint64_t)sd.kids;
    uint64_t root;
    if (b == 2) {
        root = (D * level >= 64) ? 0 : (uid >> (uint64_t)(D * level));
    } else {
        root = uid;
        for (int j = 0; j < level; ++j) root /= kids;
    }
    for (int i = D - 1; i >= 0; --i) {
        K[i] = root % d;
        root /= d;
    }
    for (int j = 1; j <= level; ++j) {
        uint64_t c = uid;
        if (b == 2) {
            c = uid >> (uint64_t)(D * (level - j));
            for (int i = 0; i < D; ++i) K[i] = 2u * K[i] + ((c >> (uint64_t)(D - 1 - i)) & 1u);
        } else {
            for (int t = 0; t < level - j; ++t) c /= kids;
            c %= kids;
            uint64_t digits[kMaxDim];
            for (int i = D - 1; i >= 0; --i) {
                digits[i] = c % b;
                c /= b;
            }
            for (int i = 0; i < D; ++i) K[i] = b * K[i] + digits[i];
        }
    }
    const double parts = level_parts(sd.split, level);
    for (int i = 0; i < D; ++i) {
        h[i] = sd.h0[i] / parts;
        lo[i] = fma((double)K[i], h[i], sd.lower[i]);
    }
}

__device__ __forceinline__ double cube_volume(const SlotDesc& sd, int D, int level)
{
    const double parts = level_parts(sd.split, level);
    double v = 1.0;
    for (int i = 0; i < D; ++i) v = v * (sd.h0[i] / parts);
    return v;
}

} // namespace zmc
