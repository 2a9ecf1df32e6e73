// zmc_level.hip -- per-cube and per-integral kernels of one tree level
// (ZMCintegral, Sec. 2.1): trial mean / standard deviation per sub-domain,
// the threshold from the mean and standard deviation of the level's standard
// deviations, selection, acceptance, and the split of the selected cubes.
//
// All of these are HBM-bound and small next to the sampling kernel.  The
// per-cube kernels work on tiles of 1024 consecutive cubes of one segment
// (256 threads, 4 cubes each, strided so that loads coalesce).  The
// per-integral step that follows each of them (the mean of s, the threshold,
// the decision) runs, for small levels, in the same launch: the last tile
// block of a segment to finish, found with a per-segment counter, reduces
// that segment's tile records in tile order, so a level costs three short
// launches after sampling.  Publishing a tile record to the other XCDs takes
// an L2 write-back per block, which outweighs a launch once a level has a few
// hundred tiles; large levels therefore run the per-segment steps as their own
// one-block-per-segment launches.  Every reduction has a fixed shape (thread-serial over its
// elements, then wave64 butterflies, then the 4 waves in order), so results
// are bitwise reproducible and independent of which block finishes last or
// of what else is resident.
#include <float.h>

#include <algorithm>

#include "zmc_kernels.hpp"

namespace zmc {

namespace {

constexpr int kWaves = kLevelThreads / 64;
constexpr int kPerThread = kTileCubes / kLevelThreads;

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ double wave_min(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
    return v;
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

__device__ __forceinline__ int64_t wave_sum_i(int64_t v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Block-wide sum in a fixed order; every thread gets the result.
__device__ double block_sum(double v, double* sh)
{
    v = wave_sum(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = sh[0];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) t += sh[w];
    return t;
}

__device__ double block_min(double v, double* sh)
{
    v = wave_min(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = sh[0];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) t = fmin(t, sh[w]);
    return t;
}

__device__ double block_max(double v, double* sh)
{
    v = wave_max(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = sh[0];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) t = fmax(t, sh[w]);
    return t;
}

__device__ int64_t block_sum_i(int64_t v, int64_t* sh)
{
    v = wave_sum_i(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    int64_t t = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) t += sh[w];
    return t;
}

// The selection totals of a tile or a segment, reduced over the block in one
// exchange: four sums, a minimum and a count, each combined in the same
// fixed order as block_sum / block_min / block_sum_i.
struct SelTotals {
    double accM, accS2, selM, selS2, margin;
    int64_t nsel;
};

__device__ SelTotals block_reduce_sel(SelTotals v)
{
    __shared__ double shd[kWaves][5];
    __shared__ int64_t shn[kWaves];
    v.accM = wave_sum(v.accM);
    v.accS2 = wave_sum(v.accS2);
    v.selM = wave_sum(v.selM);
    v.selS2 = wave_sum(v.selS2);
    v.margin = wave_min(v.margin);
    v.nsel = wave_sum_i(v.nsel);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
        const int w = threadIdx.x >> 6;
        shd[w][0] = v.accM;
        shd[w][1] = v.accS2;
        shd[w][2] = v.selM;
        shd[w][3] = v.selS2;
        shd[w][4] = v.margin;
        shn[w] = v.nsel;
    }
    __syncthreads();
    SelTotals t{shd[0][0], shd[0][1], shd[0][2], shd[0][3], shd[0][4], 0};
    for (int w = 1; w < kWaves; ++w) {
        t.accM += shd[w][0];
        t.accS2 += shd[w][1];
        t.selM += shd[w][2];
        t.selS2 += shd[w][3];
        t.margin = fmin(t.margin, shd[w][4]);
    }
    for (int w = 0; w < kWaves; ++w) t.nsel += shn[w];
    return t;
}

// Exclusive prefix of a 0/1 flag over the block in thread order; *total gets
// the block's count.
__device__ int block_excl_scan_flag(int flag, int* sh, int* total)
{
    const unsigned long long mask = __ballot(flag);
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int in_wave = __popcll(mask & ((1ull << lane) - 1ull));
    __syncthreads();
    if (lane == 0) sh[wv] = __popcll(mask);
    __syncthreads();
    int base = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
        if (w < wv) base += sh[w];
        tot += sh[w];
    }
    *total = tot;
    return base + in_wave;
}

// Segment that owns tile t (segments are in list order, tile_base ascending).
__device__ __forceinline__ int seg_of_tile(const Segment* segs, int n, int64_t t)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (segs[mid].tile_base <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Called by every tile block of segment si once its tile record is written:
// true in the block that completes the segment, which then sees every other
// block's records.  The counter is back at 0 when the launch ends.
__device__ bool last_tile_of_segment(int32_t* count, int si, int64_t n_tiles)
{
    __shared__ int last;
    __syncthreads();
    // a one-tile segment has no other block to wait for: its own record is
    // visible to the block after the barrier, and no device-scope fence (an
    // L2 write-back on this chip) is needed
    if (n_tiles == 1) return true;
    if (threadIdx.x == 0) {
        __threadfence(); // release this block's tile record
        const int old = atomicAdd(&count[si], 1);
        last = (old == (int)n_tiles - 1);
        if (last) atomicExch(&count[si], 0);
    }
    __syncthreads();
    if (last) __threadfence(); // acquire the other blocks' records
    return last != 0;
}

// ---- per-segment steps (one block) ------------------------------------------
__device__ void seg_mean(const LevelArgs& a, int si)
{
    __shared__ double sh[kWaves];
    const Segment& sg = a.segs[si];
    double v = 0.0, lo = DBL_MAX, hi = -DBL_MAX;
    for (int64_t t = threadIdx.x; t < sg.n_tiles; t += kLevelThreads) {
        const TileRec& T = a.tiles[sg.tile_base + t];
        v += T.sum_s;
        lo = fmin(lo, T.s_min);
        hi = fmax(hi, T.s_max);
    }
    const double tot = block_sum(v, sh);
    lo = block_min(lo, sh);
    hi = block_max(hi, sh);
    if (threadIdx.x == 0) {
        a.stats[si].mu = tot / (double)sg.n_cubes;
        a.stats[si].s_min = lo;
        a.stats[si].s_max = hi;
    }
}

// The scale exponent of the threshold's std: the largest |s - mu| is at the
// smallest or the largest s (rounding is monotonic).
__device__ __forceinline__ int thr_scale_exp(double mu, double lo, double hi)
{
    return std_scale_exp(fmax(fabs(hi - mu), fabs(lo - mu)));
}

__device__ void seg_thr(const LevelArgs& a, int si)
{
    __shared__ double sh[kWaves];
    const Segment& sg = a.segs[si];
    double v = 0.0;
    for (int64_t t = threadIdx.x; t < sg.n_tiles; t += kLevelThreads) v += a.tiles[sg.tile_base + t].sum_sq;
    const double tot = block_sum(v, sh);
    if (threadIdx.x == 0) {
        const SegStats& S = a.stats[si];
        const double sd = ldexp(sqrt(tot / (double)sg.n_cubes), thr_scale_exp(S.mu, S.s_min, S.s_max));
        a.stats[si].sd = sd;
        a.stats[si].thr = a.stats[si].mu + a.slots[sg.slot].sigma_mult * sd;
    }
}

__device__ void seg_decide(const LevelArgs& a, int si);
__device__ void decide_write(const LevelArgs& a, int si, double accM, double accS2, double selM, double selS2,
                             double margin, int64_t nsel, int bad);

// ---- finalize: per cube I_t = V * S1_t / N, m = mean I_t, s = std I_t ------
// The partial sums of 256 consecutive cubes are contiguous ([cube][trial *
// nch + chunk]); when they fit kStage pairs, the block first copies them to
// LDS with coalesced loads, and each thread then reads its own cube's row
// there.  Larger rows (many trials or chunks) are read from memory directly.
constexpr int kStage = 2560; // 40 KiB of (S1, S2) pairs

// KEEP: also leave each thread's cubes' m and s in m_r / s_r (pass j at
// index j), for the one-block level path.
// KEEP also returns the tile's sum of s, non-finite flag and extremes of s
// (every thread).
template <bool KEEP = false>
__device__ void finalize_tile(const LevelArgs& a, int64_t tile, int si, double* m_r = nullptr,
                              double* s_r = nullptr, double* tot_s = nullptr, int* any_bad_out = nullptr,
                              double* s_ext = nullptr)
{
    __shared__ double sh[kWaves];
    __shared__ double2 stage[kStage];
    const Segment& sg = a.segs[si];
    const SlotDesc& sd = a.slots[sg.slot];
    const int D = sd.dim, n1 = sd.trials, nch = sd.nch;
    const int per = n1 * nch; // pairs per cube
    const bool staged = per * kLevelThreads <= kStage;
    const double V = cube_volume(sd, D, sg.level);
    const double N = (double)sd.samples;
    const int64_t first = (tile - sg.tile_base) * kTileCubes;
    double sum_s = 0.0, s_lo = DBL_MAX, s_hi = -DBL_MAX;
    int bad = 0;
#pragma unroll
    for (int j = 0; j < kPerThread; ++j) {
        const int64_t c0 = first + (int64_t)j * kLevelThreads; // first cube of this pass
        if (c0 >= sg.n_cubes) break;                            // uniform over the block
        const int cnt = (int)min<int64_t>(kLevelThreads, sg.n_cubes - c0);
        const double2* P;
        if (staged) {
            const double2* src = a.partial + sg.part_base + c0 * per;
            __syncthreads(); // the previous pass is done with the stage
            for (int e = threadIdx.x; e < cnt * per; e += kLevelThreads) stage[e] = src[e];
            __syncthreads();
            P = stage + threadIdx.x * per;
        } else {
            P = a.partial + sg.part_base + (c0 + threadIdx.x) * per;
        }
        if ((int)threadIdx.x >= cnt) continue;
        const int64_t cl = c0 + threadIdx.x;
        const int64_t c = sg.cube_base + cl;
        double sum = 0.0;
        for (int t = 0; t < n1; ++t) {
            double S1 = 0.0, S2 = 0.0;
            for (int ch = 0; ch < nch; ++ch) {
                const double2 v = P[t * nch + ch];
                S1 += v.x;
                S2 += v.y;
            }
            if (a.tr_S1) {
                a.tr_S1[c * n1 + t] = S1;
                a.tr_S2[c * n1 + t] = S2;
            }
            sum += V * (S1 / N);
        }
        const double m = sum / (double)n1;
        double dmax = 0.0;
        for (int t = 0; t < n1; ++t) {
            double S1 = 0.0;
            for (int ch = 0; ch < nch; ++ch) S1 += P[t * nch + ch].x;
            const double d = fabs(V * (S1 / N) - m);
            if (d > dmax) dmax = d;
        }
        const int e = std_scale_exp(dmax);
        double ss = 0.0;
        for (int t = 0; t < n1; ++t) {
            double S1 = 0.0;
            for (int ch = 0; ch < nch; ++ch) S1 += P[t * nch + ch].x;
            const double d = ldexp(V * (S1 / N) - m, -e);
            ss += d * d;
        }
        const double s = ldexp(sqrt(ss / (double)n1), e);
        a.m[c] = m;
        a.s[c] = s;
        if constexpr (KEEP) {
            m_r[j] = m;
            s_r[j] = s;
        }
        sum_s += s;
        s_lo = fmin(s_lo, s);
        s_hi = fmax(s_hi, s);
        bad |= !(isfinite(m) && isfinite(s));
    }
    const double tot = block_sum(sum_s, sh);
    const double lo = block_min(s_lo, sh);
    const double hi = block_max(s_hi, sh);
    const int any_bad = __syncthreads_or(bad);
    if (threadIdx.x == 0) {
        a.tiles[tile].sum_s = tot;
        a.tiles[tile].s_min = lo;
        a.tiles[tile].s_max = hi;
        a.tiles[tile].nonfinite = any_bad;
    }
    if constexpr (KEEP) {
        *tot_s = tot;
        *any_bad_out = any_bad;
        s_ext[0] = lo;
        s_ext[1] = hi;
    }
}

__global__ __launch_bounds__(kLevelThreads) void finalize_kernel(const LevelArgs a)
{
    const int64_t tile = blockIdx.x;
    const int si = seg_of_tile(a.segs, a.n_segs, tile);
    const Segment& sg = a.segs[si];
    finalize_tile(a, tile, si);
    if (a.fused && sg.need_thr && !sg.group_size && last_tile_of_segment(a.seg_count, si, sg.n_tiles))
        seg_mean(a, si);
}

// ---- threshold: std of s around the mean, per segment ----------------------
__device__ void sqdev_tile(const LevelArgs& a, int64_t tile, int si)
{
    __shared__ double sh[kWaves];
    const Segment& sg = a.segs[si];
    const double mu = a.stats[si].mu;
    const int e = thr_scale_exp(mu, a.stats[si].s_min, a.stats[si].s_max);
    const int64_t first = (tile - sg.tile_base) * kTileCubes;
    double acc = 0.0;
    for (int j = 0; j < kPerThread; ++j) {
        const int64_t cl = first + threadIdx.x + (int64_t)j * kLevelThreads;
        if (cl >= sg.n_cubes) break;
        const double d = ldexp(a.s[sg.cube_base + cl] - mu, -e);
        acc += d * d;
    }
    const double tot = block_sum(acc, sh);
    if (threadIdx.x == 0) a.tiles[tile].sum_sq = tot;
}

__global__ __launch_bounds__(kLevelThreads) void tile_sqdev_kernel(const LevelArgs a)
{
    const int64_t tile = blockIdx.x;
    const int si = seg_of_tile(a.segs, a.n_segs, tile);
    const Segment& sg = a.segs[si];
    if (!sg.need_thr || sg.group_size) return;
    sqdev_tile(a, tile, si);
    if (a.fused && last_tile_of_segment(a.seg_count, si, sg.n_tiles)) seg_thr(a, si);
}

// ---- per-segment steps as their own launches (large levels) -----------------
__global__ __launch_bounds__(kLevelThreads) void seg_mean_kernel(const LevelArgs a)
{
    const Segment& sg = a.segs[blockIdx.x];
    if (!sg.need_thr || sg.group_size) return;
    seg_mean(a, blockIdx.x);
}

__global__ __launch_bounds__(kLevelThreads) void seg_thr_kernel(const LevelArgs a)
{
    const Segment& sg = a.segs[blockIdx.x];
    if (!sg.need_thr || sg.group_size) return;
    seg_thr(a, blockIdx.x);
}

// ---- per-parent thresholds: one per group of siblings -----------------------
// One wave per group (groups of the segments with group_size > 0, in list
// order): mean of the group's s, then the population std, in a fixed order.
__device__ __forceinline__ int seg_of_group(const Segment* segs, int n, int64_t g)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (segs[mid].group_base <= g) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(kLevelThreads) void group_thr_kernel(const LevelArgs a)
{
    const int lane = threadIdx.x & 63;
    const int64_t n_waves = (int64_t)gridDim.x * kWaves;
    for (int64_t g = (int64_t)blockIdx.x * kWaves + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
         g < a.n_groups; g += n_waves) {
        const int si = seg_of_group(a.segs, a.n_segs, g);
        const Segment& sg = a.segs[si];
        const int64_t gs = sg.group_size;
        const double* s = a.s + sg.cube_base + (g - sg.group_base) * gs;
        double v = 0.0;
        for (int64_t j = lane; j < gs; j += 64) v += s[j];
        const double mu = wave_sum(v) / (double)gs;
        double dmax = 0.0;
        for (int64_t j = lane; j < gs; j += 64) dmax = fmax(dmax, fabs(s[j] - mu));
        const int e = std_scale_exp(wave_max(dmax));
        double q = 0.0;
        for (int64_t j = lane; j < gs; j += 64) {
            const double d = ldexp(s[j] - mu, -e);
            q += d * d;
        }
        const double sd = ldexp(sqrt(wave_sum(q) / (double)gs), e);
        if (lane == 0) a.gthr[g] = mu + a.slots[sg.slot].sigma_mult * sd;
    }
}

// ---- selection: split = s > thr; accepted and selected sums per tile -------
__device__ void select_tile(const LevelArgs& a, int64_t tile, int si)
{
    const Segment& sg = a.segs[si];
    const bool thr_on = sg.need_thr != 0;
    const double level_thr = (thr_on && !sg.group_size) ? a.stats[si].thr : 0.0;
    const int64_t first = (tile - sg.tile_base) * kTileCubes;
    double accM = 0.0, accS2 = 0.0, selM = 0.0, selS2 = 0.0, margin = DBL_MAX;
    int64_t nsel = 0;
    for (int j = 0; j < kPerThread; ++j) {
        const int64_t cl = first + threadIdx.x + (int64_t)j * kLevelThreads;
        if (cl >= sg.n_cubes) break;
        const int64_t c = sg.cube_base + cl;
        const double m = a.m[c], s = a.s[c];
        const double thr = (thr_on && sg.group_size) ? a.gthr[sg.group_base + cl / sg.group_size] : level_thr;
        const bool sel = thr_on && (s > thr);
        a.sel[c] = sel ? 1 : 0;
        if (sel) {
            selM += m;
            selS2 += s * s;
            ++nsel;
        } else {
            accM += m;
            accS2 += s * s;
        }
        if (thr_on && thr > 0.0) margin = fmin(margin, fabs(s - thr) / thr);
    }
    const SelTotals tot = block_reduce_sel(SelTotals{accM, accS2, selM, selS2, margin, nsel});
    if (threadIdx.x == 0) {
        TileRec& T = a.tiles[tile];
        T.accM = tot.accM;
        T.accS2 = tot.accS2;
        T.selM = tot.selM;
        T.selS2 = tot.selS2;
        T.min_margin = tot.margin;
        T.n_sel = tot.nsel;
    }
}

__global__ __launch_bounds__(kLevelThreads) void tile_select_kernel(const LevelArgs a)
{
    const int64_t tile = blockIdx.x;
    const int si = seg_of_tile(a.segs, a.n_segs, tile);
    const Segment& sg = a.segs[si];
    select_tile(a, tile, si);
    if (a.fused && last_tile_of_segment(a.seg_count, si, sg.n_tiles)) seg_decide(a, si);
}

// ---- per segment: totals, stop rules, rank base of every tile --------------
__device__ void seg_decide(const LevelArgs& a, int si)
{
    __shared__ int64_t shi[kWaves];
    const Segment& sg = a.segs[si];
    const SlotDesc& sd = a.slots[sg.slot];
    double accM = 0.0, accS2 = 0.0, selM = 0.0, selS2 = 0.0, margin = DBL_MAX;
    int64_t nsel = 0;
    int bad = 0;
    for (int64_t t = threadIdx.x; t < sg.n_tiles; t += kLevelThreads) {
        const TileRec& T = a.tiles[sg.tile_base + t];
        accM += T.accM;
        accS2 += T.accS2;
        selM += T.selM;
        selS2 += T.selS2;
        margin = fmin(margin, T.min_margin);
        nsel += T.n_sel;
        bad |= T.nonfinite;
    }
    {
        const SelTotals tot = block_reduce_sel(SelTotals{accM, accS2, selM, selS2, margin, nsel});
        accM = tot.accM;
        accS2 = tot.accS2;
        selM = tot.selM;
        selS2 = tot.selS2;
        margin = tot.margin;
        nsel = tot.nsel;
    }
    bad = __syncthreads_or(bad);

    // exclusive prefix of the tiles' selection counts (rank base for spawn)
    int64_t carry = 0;
    for (int64_t t0 = 0; t0 < sg.n_tiles; t0 += kLevelThreads) {
        const int64_t t = t0 + threadIdx.x;
        const int64_t v = t < sg.n_tiles ? a.tiles[sg.tile_base + t].n_sel : 0;
        // inclusive wave scan
        int64_t x = v;
        const int lane = threadIdx.x & 63;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int64_t y = __shfl_up(x, off, 64);
            if (lane >= off) x += y;
        }
        __syncthreads();
        if (lane == 63) shi[threadIdx.x >> 6] = x;
        __syncthreads();
        int64_t base = carry;
        int64_t chunk = 0;
        for (int w = 0; w < kWaves; ++w) {
            if (w < (threadIdx.x >> 6)) base += shi[w];
            chunk += shi[w];
        }
        if (t < sg.n_tiles) a.tiles[sg.tile_base + t].sel_prefix = base + x - v;
        carry += chunk;
    }

    if (threadIdx.x == 0) decide_write(a, si, accM, accS2, selM, selS2, margin, nsel, bad);
}

// The segment's outcome from its totals (thread 0): stop rules, running
// totals, the record in device memory and in the mapped host buffer.
__device__ void decide_write(const LevelArgs& a, int si, double accM, double accS2, double selM, double selS2,
                             double margin, int64_t nsel, int bad)
{
    const Segment& sg = a.segs[si];
    const SlotDesc& sd = a.slots[sg.slot];
    {
        SegStats& S = a.stats[si];
        const double2 prev = a.prev_tot[si];
        if (!sg.need_thr || sg.group_size) {
            S.mu = S.sd = S.thr = __builtin_nan("");
        }
        S.min_margin = margin;
        S.accM = accM;
        S.accS2 = accS2;
        S.selM = selM;
        S.selS2 = selS2;
        S.n_sel = nsel;
        S.nonfinite = bad;
        S.range_lost = a.seg_flags ? a.seg_flags[si] : 0;
        int32_t dec;
        double totM = prev.x + accM, totS2 = prev.y + accS2;
        if (!sg.need_thr || nsel == 0) {
            dec = kDone;
        } else {
            const double runM = totM + selM, runS2 = totS2 + selS2;
            if (sd.rtol > 0.0 && sqrt(runS2 / (double)(sd.trials - 1)) <= sd.rtol * fabs(runM)) {
                dec = kRtolMet;
            } else if ((uint64_t)nsel * (uint64_t)sd.kids > (uint64_t)sd.max_cubes) {
                dec = kTruncated;
            } else {
                dec = kSplit;
            }
            if (dec != kSplit) {
                totM = runM;
                totS2 = runS2;
            }
        }
        S.decision = dec;
        S.totM = totM;
        S.totS2 = totS2;
        if (a.host_stats) {
            a.host_stats[si] = S;
            __threadfence_system();
        }
    }
}

__global__ __launch_bounds__(kLevelThreads) void seg_decide_kernel(const LevelArgs a) { seg_decide(a, blockIdx.x); }

// ---- a whole small level in one launch ----------------------------------------
// When every segment of the level is one tile (at most 1024 cubes) and no
// segment forms per-parent thresholds, one block per segment runs finalize,
// the mean of s, the threshold, the selection and the decision, with each
// thread's m and s kept in registers between the steps and the reductions in
// LDS.  With one tile per segment each per-segment reduction of the
// multi-launch path reduces a single tile record (the other threads add
// zeros), so this is the same arithmetic in the same order and the results
// are bitwise those of the multi-launch path.
__global__ __launch_bounds__(kLevelThreads) void level_small_kernel(const LevelArgs a)
{
    __shared__ double sh[kWaves];
    const int si = blockIdx.x;
    const Segment& sg = a.segs[si];
    const int64_t tile = sg.tile_base;
    const bool thr_on = sg.need_thr != 0;
    double m_r[kPerThread], s_r[kPerThread];
    double tot_s = 0.0, s_ext[2] = {0.0, 0.0};
    int bad = 0;
    finalize_tile<true>(a, tile, si, m_r, s_r, &tot_s, &bad, s_ext);
    const int64_t n = sg.n_cubes;
    double mu = 0.0, sdv = 0.0, thr = 0.0, tot_sq = 0.0;
    if (thr_on) {
        mu = tot_s / (double)n;
        const int e = thr_scale_exp(mu, s_ext[0], s_ext[1]);
        double acc = 0.0;
#pragma unroll
        for (int j = 0; j < kPerThread; ++j) {
            const int64_t cl = threadIdx.x + (int64_t)j * kLevelThreads;
            if (cl < n) {
                const double d = ldexp(s_r[j] - mu, -e);
                acc += d * d;
            }
        }
        tot_sq = block_sum(acc, sh);
        sdv = ldexp(sqrt(tot_sq / (double)n), e);
        thr = mu + a.slots[sg.slot].sigma_mult * sdv;
    }
    double accM = 0.0, accS2 = 0.0, selM = 0.0, selS2 = 0.0, margin = DBL_MAX;
    int64_t nsel = 0;
#pragma unroll
    for (int j = 0; j < kPerThread; ++j) {
        const int64_t cl = threadIdx.x + (int64_t)j * kLevelThreads;
        if (cl >= n) break;
        const int64_t c = sg.cube_base + cl;
        const double m = m_r[j], s = s_r[j];
        const bool sel = thr_on && (s > thr);
        a.sel[c] = sel ? 1 : 0;
        if (sel) {
            selM += m;
            selS2 += s * s;
            ++nsel;
        } else {
            accM += m;
            accS2 += s * s;
        }
        if (thr_on && thr > 0.0) margin = fmin(margin, fabs(s - thr) / thr);
    }
    const SelTotals tot = block_reduce_sel(SelTotals{accM, accS2, selM, selS2, margin, nsel});
    if (threadIdx.x == 0) {
        TileRec& T = a.tiles[tile];
        T.sum_sq = tot_sq;
        T.accM = tot.accM;
        T.accS2 = tot.accS2;
        T.selM = tot.selM;
        T.selS2 = tot.selS2;
        T.min_margin = tot.margin;
        T.n_sel = tot.nsel;
        T.sel_prefix = 0;
        if (thr_on) {
            a.stats[si].mu = mu;
            a.stats[si].s_min = s_ext[0];
            a.stats[si].s_max = s_ext[1];
            a.stats[si].sd = sdv;
            a.stats[si].thr = thr;
        }
        decide_write(a, si, tot.accM, tot.accS2, tot.selM, tot.selS2, tot.margin, tot.nsel, bad);
    }
}

// ---- spawn: children of the selected cubes, in list order ------------------
// One block per tile of the finished level.
__device__ void spawn_tile(const LevelArgs& a, int64_t tile)
{
    __shared__ uint64_t list[kTileCubes];
    __shared__ uint32_t list_hi[kTileCubes];
    __shared__ int shf[kWaves];
    const int si = seg_of_tile(a.segs, a.n_segs, tile);
    const Segment& sg = a.segs[si];
    if (!sg.do_split) return;
    const SlotDesc& sd = a.slots[sg.slot];
    const int D = sd.dim;
    const int64_t kids = sd.kids;
    const int64_t first = (tile - sg.tile_base) * kTileCubes;
    int base = 0;
    for (int j = 0; j < kPerThread; ++j) {
        const int64_t cl = first + threadIdx.x + (int64_t)j * kLevelThreads;
        const int flag = (cl < sg.n_cubes) ? a.sel[sg.cube_base + cl] : 0;
        int total;
        const int pos = block_excl_scan_flag(flag, shf, &total);
        if (flag) {
            list[base + pos] = a.uid[sg.cube_base + cl];
            list_hi[base + pos] = a.uid_hi ? a.uid_hi[sg.cube_base + cl] : 0u;
        }
        base += total;
    }
    __syncthreads();
    const int64_t n_writes = (int64_t)base * kids;
    const int64_t first_out = sg.child_base + a.tiles[tile].sel_prefix * kids;
    uint64_t* out = a.next_uid + first_out;
    uint32_t* out_hi = a.next_uid_hi ? a.next_uid_hi + first_out : nullptr;
    // child c of (hi:lo) is (hi:lo) * kids + c; with bisection (hi:lo) << D | c
    if (sd.split == 2) {
        const uint64_t mask = (1ull << D) - 1ull;
        for (int64_t w = threadIdx.x; w < n_writes; w += kLevelThreads) {
            const uint64_t parent = list[w >> D];
            out[w] = (parent << D) | ((uint64_t)w & mask);
            if (out_hi) out_hi[w] = (list_hi[w >> D] << D) | (uint32_t)(parent >> (64 - D));
        }
    } else {
        for (int64_t w = threadIdx.x; w < n_writes; w += kLevelThreads) {
            const int64_t i = w / kids;
            const uint64_t plo = list[i] * (uint64_t)kids;
            const uint64_t lo = plo + (uint64_t)(w - i * kids);
            out[w] = lo;
            if (out_hi)
                out_hi[w] = (uint32_t)((uint64_t)list_hi[i] * (uint64_t)kids + __umul64hi(list[i], (uint64_t)kids) +
                                       (lo < plo ? 1u : 0u));
        }
    }
}

// ---- roots: uid = r for the d^D cubes of a newly admitted integral ----------
__device__ void roots_block(const RootArgs& a, int blk)
{
    const int si = blk / a.blocks_per_seg;
    const int part = blk % a.blocks_per_seg;
    const Segment& sg = a.segs[si];
    for (int64_t r = (int64_t)part * kLevelThreads + threadIdx.x; r < sg.n_cubes;
         r += (int64_t)a.blocks_per_seg * kLevelThreads) {
        a.uid[sg.cube_base + r] = (uint64_t)r;
        if (a.uid_hi) a.uid_hi[sg.cube_base + r] = 0u;
    }
}

// The next list in one launch: the first n_spawn blocks spawn children (one
// per tile of the finished level), the rest write roots of new integrals.
__global__ __launch_bounds__(kLevelThreads) void next_list_kernel(const LevelArgs a, const RootArgs ra,
                                                                  int64_t n_spawn)
{
    const int64_t b = blockIdx.x;
    if (b < n_spawn)
        spawn_tile(a, b);
    else
        roots_block(ra, (int)(b - n_spawn));
}

// ---- debug entry points ------------------------------------------------------
__global__ void debug_philox_kernel(uint32_t k0, uint32_t k1, const uint32_t* ctr, uint32_t* out, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const U4 r = philox4x32_10(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3], k0, k1);
    out[4 * i] = r.x;
    out[4 * i + 1] = r.y;
    out[4 * i + 2] = r.z;
    out[4 * i + 3] = r.w;
}

__global__ void debug_points_kernel(const SlotDesc* sdp, int level, uint64_t uid, int trial, int64_t s0, int64_t n,
                                    double* x)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const SlotDesc& sd = *sdp;
    const int D = sd.dim;
    double lo[kMaxDim], h[kMaxDim];
    cube_corner(sd, D, level, uid, lo, h);
    const int64_t s = s0 + k;
    for (int i = 0; i < D; ++i) {
        const uint64_t nw = (uint64_t)s * (uint64_t)D + (uint64_t)i;
        const U4 r = philox4x32_10((uint32_t)(nw >> 2), ctr_word1(trial, level, 0u), (uint32_t)uid,
                                   (uint32_t)(uid >> 32), (uint32_t)sd.seed, (uint32_t)(sd.seed >> 32));
        const uint32_t words[4] = {r.x, r.y, r.z, r.w};
        const uint32_t w = words[nw & 3u];
        x[k * D + i] = fma(ldexp(h[i], -24), (double)((w >> 8) | 1u), lo[i]);
    }
}

} // namespace

hipError_t launch_finalize(const LevelArgs& a, hipStream_t st)
{
    if (a.n_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(finalize_kernel, dim3((unsigned)a.n_tiles), dim3(kLevelThreads), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_level_small(const LevelArgs& a, hipStream_t st)
{
    if (a.n_segs <= 0) return hipSuccess;
    hipLaunchKernelGGL(level_small_kernel, dim3((unsigned)a.n_segs), dim3(kLevelThreads), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_threshold(const LevelArgs& a, hipStream_t st)
{
    if (a.n_tiles <= 0) return hipSuccess;
    if (!a.fused) hipLaunchKernelGGL(seg_mean_kernel, dim3(a.n_segs), dim3(kLevelThreads), 0, st, a);
    hipLaunchKernelGGL(tile_sqdev_kernel, dim3((unsigned)a.n_tiles), dim3(kLevelThreads), 0, st, a);
    if (!a.fused) hipLaunchKernelGGL(seg_thr_kernel, dim3(a.n_segs), dim3(kLevelThreads), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_group_threshold(const LevelArgs& a, hipStream_t st)
{
    if (a.n_groups <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((a.n_groups + kWaves - 1) / kWaves, 65536);
    hipLaunchKernelGGL(group_thr_kernel, dim3((unsigned)blocks), dim3(kLevelThreads), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_select(const LevelArgs& a, hipStream_t st)
{
    if (a.n_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(tile_select_kernel, dim3((unsigned)a.n_tiles), dim3(kLevelThreads), 0, st, a);
    if (!a.fused) hipLaunchKernelGGL(seg_decide_kernel, dim3(a.n_segs), dim3(kLevelThreads), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_next_list(const LevelArgs& a, const RootArgs& ra, hipStream_t st)
{
    const int64_t n_spawn = a.n_tiles > 0 ? a.n_tiles : 0;
    const int64_t n_roots = ra.n_segs > 0 ? (int64_t)ra.n_segs * ra.blocks_per_seg : 0;
    if (n_spawn + n_roots <= 0) return hipSuccess;
    hipLaunchKernelGGL(next_list_kernel, dim3((unsigned)(n_spawn + n_roots)), dim3(kLevelThreads), 0, st, a, ra,
                       n_spawn);
    return hipGetLastError();
}

hipError_t launch_debug_philox(uint32_t k0, uint32_t k1, const uint32_t* ctr, uint32_t* out, int64_t n,
                               hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(debug_philox_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, k0, k1, ctr, out,
                       n);
    return hipGetLastError();
}

hipError_t launch_debug_points(const SlotDesc* sd, int level, uint64_t uid, int trial, int64_t s0, int64_t n,
                               double* x, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(debug_points_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, sd, level, uid,
                       trial, s0, n, x);
    return hipGetLastError();
}

hipError_t launch_sample(int integrand, int dim, int eval, int hint, int grid, int block, hipStream_t st,
                         const SampleArgs& a)
{
    switch (integrand) {
    case 0: return launch_sample_0(dim, eval, hint, grid, block, st, a);
    case 1: return launch_sample_1(dim, eval, hint, grid, block, st, a);
    case 2: return launch_sample_2(dim, eval, hint, grid, block, st, a);
    case 3: return launch_sample_3(dim, eval, hint, grid, block, st, a);
    case 4: return launch_sample_4(dim, eval, hint, grid, block, st, a);
    case 5: return launch_sample_5(dim, eval, hint, grid, block, st, a);
    case 6: return launch_sample_6(dim, eval, hint, grid, block, st, a);
    case 7: return launch_sample_7(dim, eval, hint, grid, block, st, a);
    default: return hipErrorInvalidValue;
    }
}

const void* sample_kernel_ptr(int integrand, int dim, int eval, int hint)
{
    switch (integrand) {
    case 0: return sample_kernel_ptr_0(dim, eval, hint);
    case 1: return sample_kernel_ptr_1(dim, eval, hint);
    case 2: return sample_kernel_ptr_2(dim, eval, hint);
    case 3: return sample_kernel_ptr_3(dim, eval, hint);
    case 4: return sample_kernel_ptr_4(dim, eval, hint);
    case 5: return sample_kernel_ptr_5(dim, eval, hint);
    case 6: return sample_kernel_ptr_6(dim, eval, hint);
    case 7: return sample_kernel_ptr_7(dim, eval, hint);
    default: return nullptr;
    }
}

} // namespace zmc
