// zmc_sample_core.hpp -- the body of the sampling kernel, shared by the
// precompiled integrand registry (zmc_sample.hip) and the run-time compiled
// user integrands (zmc_rtc.cpp): direct Monte Carlo over (cube, trial,
// chunk) units with random numbers produced at the time of use (ZMCintegral,
// Sec. 2.1 and Sec. 2.2).
//
// Work decomposition (gfx950, wave64): every wave takes one (cube, trial,
// chunk) unit at a time, independently of the other waves of its block (no
// LDS, no barrier).  A chunk is 4 * 64 * G points and lane l evaluates the
// 4-point groups g = chunk*G*64 + l + 64*j, j < G.  One group of 4 points uses
// D Philox blocks (4*D words, point q dimension i = word q*D + i), so counter
// word 0 of block k is g*D + k; the other three counter words and the key are
// wave-uniform (SGPRs).  Each lane sums f and f^2 in FP64 and the wave
// reduces with a fixed butterfly, so a unit's partial sums depend only on the
// unit and G.  The grid is persistent: wave w takes a contiguous range of
// units; only the first unit's segment is found by binary search and only
// its position decoded by division, later units follow by increments, and
// a cube's corner and integrand constants are formed once for all of its
// units.
//
// An integrand class I provides P64 / P32 parameter blocks, prep64 / prep32
// (per cube, from the slot descriptor and the cube corner), f64 / f32, the
// FP64 scale P32::scale that multiplies each FP32 unit sum, and kRangeCheck
// (whether its FP32 values can fall below FP32's normal range).
#pragma once

#include "zmc_device.hpp"

namespace zmc {


__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <int D>
__device__ __forceinline__ void corner(const SlotDesc& sd, int level, uint64_t uid, uint32_t uid_hi, double* lo,
                                       double* h)
{
    uint64_t K[D];
    const uint32_t d = (uint32_t)sd.divisions;
    if (sd.split == 2) {
        // uid = root << (D * level) | path, D bits per split
        uint64_t root = shr_id(uid, uid_hi, D * level);
        if (root < (1ull << 32)) {
            uint32_t r32 = (uint32_t)root;
#pragma unroll
            for (int i = D - 1; i >= 0; --i) {
                K[i] = r32 % d;
                r32 /= d;
            }
        } else {
#pragma unroll
            for (int i = D - 1; i >= 0; --i) {
                K[i] = root % d;
                root /= d;
            }
        }
        for (int j = 1; j <= level; ++j) {
            const uint64_t c = shr_id(uid, uid_hi, D * (level - j));
#pragma unroll
            for (int i = 0; i < D; ++i) K[i] = 2u * K[i] + ((c >> (uint64_t)(D - 1 - i)) & 1u);
        }
#pragma unroll
        for (int i = 0; i < D; ++i) {
            h[i] = ldexp(sd.h0[i], -level);
            lo[i] = fma((double)K[i], h[i], sd.lower[i]);
        }
    } else {
        // b-way splits: uid = root * kids^level + path, one base-kids digit
        // per split (kids = b^D <= 2^24).  The digits come off the low end,
        // the last split's first, and each adds its base-b digit for axis i
        // at the place value b^(splits after it): K_i = root_i b^level +
        // sum over splits j of digit_{j,i} b^(level - j).
        const uint64_t b = (uint64_t)sd.split, kids = (uint64_t)sd.kids;
        uint64_t rest = uid;
        uint32_t rest_hi = uid_hi;
        uint64_t mult = 1;
#pragma unroll
        for (int i = 0; i < D; ++i) K[i] = 0;
        for (int j = 0; j < level; ++j) {
            uint64_t c = divmod_id(rest, rest_hi, kids);
#pragma unroll
            for (int i = D - 1; i >= 0; --i) {
                K[i] += (c % b) * mult;
                c /= b;
            }
            mult *= b;
        }
        uint64_t root = rest; // < d^D < 2^64
#pragma unroll
        for (int i = D - 1; i >= 0; --i) {
            K[i] += (root % d) * mult;
            root /= d;
        }
        const uint64_t parts = mult;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            h[i] = sd.h0[i] / (double)parts;
            lo[i] = fma((double)K[i], h[i], sd.lower[i]);
        }
    }
}

// The 4 samples of a thread's group take words s*D + i, s = 0..3, i < D:
// Philox blocks cb .. cb + D - 1 (4 words each).  Blocks are generated in
// lockstep (independent chains for the issue pipeline).  For D >= kHalvesMinD
// they are generated in two halves, the blocks holding samples 0-1 and then
// the rest, and each half's samples are evaluated before the next half is
// generated: the words live at once halve, which leaves registers for more
// waves.  eval(q, w) gets sample q's D words in order.
constexpr int kHalvesMinD = 10;

template <int D, class Eval>
__device__ __forceinline__ void group_samples(uint32_t cb, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                              uint32_t k1, Eval&& eval)
{
    constexpr int HA = D >= kHalvesMinD ? (D + 1) / 2 : D; // blocks of the first half
    constexpr int HB = D - HA;
    uint32_t ca[HA];
    uint32_t wa[4 * HA];
#pragma unroll
    for (int k = 0; k < HA; ++k) ca[k] = cb + (uint32_t)k;
    philox4x32_10_lockstep<HA>(ca, c1, c2, c3, k0, k1, wa);
    constexpr int QA = HB > 0 ? 2 : 4; // samples wholly inside the first half
#pragma unroll
    for (int q = 0; q < QA; ++q) {
        uint32_t ws[D];
#pragma unroll
        for (int i = 0; i < D; ++i) ws[i] = wa[q * D + i];
        eval(q, ws);
    }
    if constexpr (HB > 0) {
        uint32_t cbk[HB];
        uint32_t wb[4 * HB];
#pragma unroll
        for (int k = 0; k < HB; ++k) cbk[k] = cb + (uint32_t)(HA + k);
        philox4x32_10_lockstep<HB>(cbk, c1, c2, c3, k0, k1, wb);
#pragma unroll
        for (int q = 2; q < 4; ++q) {
            uint32_t ws[D];
#pragma unroll
            for (int i = 0; i < D; ++i) {
                const int n = q * D + i; // words 2D .. 4HA - 1 are left from the first half
                ws[i] = n < 4 * HA ? wa[n] : wb[n - 4 * HA];
            }
            eval(q, ws);
        }
    }
}

template <bool B>
struct BoolTag {
    static constexpr bool value = B;
};

// Per-cube state of the sampling loop: FP32 evaluation keeps the integrand's
// cube-relative constants (formed in FP64 from the corner), FP64 evaluation
// the corner and the edge lengths scaled by 2^-24 with the integrand's
// constants.  Computed once per cube, for all of its (trial, chunk) units.
template <class I, int D, bool FP32>
struct CubeState;

template <class I, int D>
struct CubeState<I, D, true> {
    typename I::P32 p;
    __device__ __forceinline__ void set(const SlotDesc& sd, int level, uint64_t uid, uint32_t uid_hi)
    {
        double lo[D], h[D];
        corner<D>(sd, level, uid, uid_hi, lo, h);
        I::prep32(sd, lo, h, p);
    }
};

template <class I, int D>
struct CubeState<I, D, false> {
    typename I::P64 p;
    double lo[D], h24[D];
    __device__ __forceinline__ void set(const SlotDesc& sd, int level, uint64_t uid, uint32_t uid_hi)
    {
        double h[D];
        corner<D>(sd, level, uid, uid_hi, lo, h);
#pragma unroll
        for (int i = 0; i < D; ++i) h24[i] = ldexp(h[i], -24);
        I::prep64(sd, p);
    }
};

// KEEP_S2: also accumulate the sum of squares (only the per-(cube, trial)
// trace reads it; the estimator uses the sums alone).  Without it the
// partial's second member is 0.
// W: the occupancy variant's minimum waves per SIMD (1 = unconstrained); it
// decides whether whole and ragged groups get loops of their own (below).
template <class I, int D, bool FP32, bool KEEP_S2, int W = 1>
__device__ __forceinline__ void sample_units(const SampleArgs& a)
{
    // blocks of 64, 128 or 256 threads (the tile table's block shape)
    const int waves_per_block = (int)(blockDim.x >> 6);
    const int lane = threadIdx.x & 63;
    // the wave index is uniform over the wave: keep it (and all unit
    // bookkeeping derived from it) in scalar registers
    const int64_t wave = (int64_t)blockIdx.x * waves_per_block + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t n_waves = (int64_t)gridDim.x * waves_per_block;
    const int64_t U = a.total_units;
    const int64_t per = (U + n_waves - 1) / n_waves;
    int64_t u = a.unit0 + wave * per;
    const int64_t uend = min(a.unit0 + U, u + per);
    if (u >= uend) return;

    int bs = 0;
    {
        int hi = a.n_bsegs - 1;
        while (bs < hi) {
            const int mid = (bs + hi + 1) >> 1;
            if (a.bsegs[mid].unit_base <= u) bs = mid;
            else hi = mid - 1;
        }
    }

    // The wave's first unit is decoded by division; every later one follows
    // by increments (chunk, then trial, then cube), and a new bucket segment
    // is decoded afresh.  Units are [cube][trial][chunk] within a segment.
    const Segment* sg = nullptr;
    const SlotDesc* sd = nullptr;
    int64_t local = 0, cl = 0;
    int trial = 0, chunk = 0;
    auto decode = [&]() {
        sg = &a.segs[a.bsegs[bs].seg];
        sd = &a.slots[sg->slot];
        local = u - a.bsegs[bs].unit_base;
        const int nch = sd->nch;
        const int64_t upc = (int64_t)sd->trials * nch;
        cl = local / upc;
        const int rem = (int)(local - cl * upc);
        trial = rem / nch;
        chunk = rem - trial * nch;
    };
    decode();
    CubeState<I, D, FP32> cs;
    uint64_t uid = 0;
    uint32_t uid_hi = 0;
    bool fresh = true; // the cube's state is to be (re)computed

    for (; u < uend; ++u) {
        if (bs + 1 < a.n_bsegs && a.bsegs[bs + 1].unit_base <= u) {
            while (bs + 1 < a.n_bsegs && a.bsegs[bs + 1].unit_base <= u) ++bs;
            decode();
            fresh = true;
        }
        const int level = sg->level;
        if (fresh) {
            uid = a.uid[sg->cube_base + cl];
            uid_hi = a.uid_hi ? a.uid_hi[sg->cube_base + cl] : 0u;
            cs.set(*sd, level, uid, uid_hi);
            fresh = false;
        }

        const uint32_t k0 = (uint32_t)sd->seed, k1 = (uint32_t)(sd->seed >> 32);
        const uint32_t c1 = ctr_word1(trial, level, uid_hi);
        const uint32_t c2 = (uint32_t)uid, c3 = (uint32_t)(uid >> 32);
        const int64_t N = sd->samples;
        const int G = sd->groups;
        const int64_t g0 = (int64_t)chunk * G * 64 + lane;

        double S1 = 0.0, S2 = 0.0;
        // Groups of 4 points; with N a multiple of 4 every group a lane
        // reaches is whole, otherwise the group holding point N - 1 is cut
        // short and its points past N count as 0.  Where registers allow,
        // the two cases are separate loops, so that whole groups carry no
        // per-point mask (1-3% faster).  The second loop costs registers: in
        // the 7- and 8-wave variants from D = 7 (8-wave: from D = 5) it made
        // the allocator spill (up to 66% slower), and from D = kHalvesMinD
        // on the mask costs under 1%; those keep the one masked loop.
        // In FP32 evaluation up to D = 3, a chunk holding G * 256 points or
        // more (every lane has G whole groups) also drops the per-lane exit
        // test: a wave-uniform trip count.  From D = 4 on, and in FP64, that
        // loop took more registers than it saved instructions (one wave per
        // SIMD less in several buckets).
        // FP32 evaluation adds a group's 4 values in FP32 and the group's sum
        // in FP64: one conversion and one FP64 add per group instead of per
        // point.  The 4 values are added in point order, except at D = 6 and
        // 7, where (v0 + v1) + (v2 + v3) ran 1-2.4% faster than both the
        // point-order sum and per-value FP64 adds in a same-box A/B (and
        // 0.5-3.7% slower at the other D).
        constexpr bool kWholeLoop = D < kHalvesMinD && (W <= 5 || (W == 7 && D <= 6));
        constexpr bool kUniformLoop = FP32 && D <= 3;
        constexpr bool kPairSum = D == 6 || D == 7;
        auto run = [&](auto masked, auto tested) {
            constexpr bool kMasked = decltype(masked)::value;
            for (int j = 0; j < G; ++j) {
                const int64_t g = g0 + (int64_t)j * 64;
                int nvalid = 4;
                if constexpr (decltype(tested)::value) {
                    const int64_t s0 = 4 * g;
                    if (s0 >= N) break;
                    if constexpr (kMasked) nvalid = (int)min((int64_t)4, N - s0);
                }
                [[maybe_unused]] float gs = 0.0f, gb = 0.0f;
                group_samples<D>((uint32_t)g * (uint32_t)D, c1, c2, c3, k0, k1, [&](int q, const uint32_t* w) {
                    if constexpr (FP32) {
                        float v[D];
#pragma unroll
                        for (int i = 0; i < D; ++i) v[i] = unit_interval_f32(w[i]);
                        float f = I::f32(cs.p, v);
                        if constexpr (kMasked) f = (q < nvalid) ? f : 0.0f;
                        if constexpr (kPairSum) {
                            if (q == 0) gs = f;
                            else if (q == 1) gs = gs + f;
                            else if (q == 2) gb = f;
                            else gb = gb + f;
                        } else {
                            gs = q == 0 ? f : gs + f;
                        }
                        if constexpr (KEEP_S2) {
                            const double fd = (double)f;
                            S2 = fma(fd, fd, S2);
                        }
                    } else {
                        double x[D];
                        // x = fma(h, (2*(w>>9)+1) 2^-24, lo) computed as
                        // fma(h 2^-24, (w>>8)|1, lo): the same exact product
#pragma unroll
                        for (int i = 0; i < D; ++i) x[i] = fma(cs.h24[i], (double)((w[i] >> 8) | 1u), cs.lo[i]);
                        double f = I::f64(cs.p, x);
                        if constexpr (kMasked) f = (q < nvalid) ? f : 0.0;
                        S1 += f;
                        if constexpr (KEEP_S2) S2 = fma(f, f, S2);
                    }
                });
                if constexpr (FP32) S1 += (double)(kPairSum ? gs + gb : gs);
            }
        };
        if constexpr (kWholeLoop && kUniformLoop) {
            const int64_t left = N - (int64_t)chunk * G * 256; // this chunk's points onward (wave-uniform)
            if (left >= (int64_t)G * 256) run(BoolTag<false>{}, BoolTag<false>{});
            else run(BoolTag<true>{}, BoolTag<true>{});
        } else if constexpr (kWholeLoop) {
            if ((N & 3) == 0) run(BoolTag<false>{}, BoolTag<true>{});
            else run(BoolTag<true>{}, BoolTag<true>{});
        } else {
            run(BoolTag<true>{}, BoolTag<true>{});
        }

        S1 = wave_sum(S1);
        if constexpr (KEEP_S2) S2 = wave_sum(S2);
        if constexpr (FP32) {
            if constexpr (I::kRangeCheck) {
                // values below FP32's normal range: report it for the segment
                const int64_t pts = min((int64_t)G * 256, N - (int64_t)chunk * G * 256);
                if (lane == 0 && fabs(S1) < (double)pts * 0x1p-126)
                    atomicOr(a.seg_flags + a.bsegs[bs].seg, kRangeLost);
            }
            S1 *= cs.p.scale;
            if constexpr (KEEP_S2) S2 *= cs.p.scale * cs.p.scale;
        }
        // partial sums in unit order, [cube][trial * nch + chunk]: a wave's
        // consecutive units fill whole cache lines
        if (lane == 0) a.partial[sg->part_base + local] = make_double2(S1, S2);

        // the next unit: chunk, then trial, then cube
        ++local;
        if (++chunk == sd->nch) {
            chunk = 0;
            if (++trial == sd->trials) {
                trial = 0;
                ++cl;
                fresh = true;
            }
        }
    }
}

} // namespace zmc
