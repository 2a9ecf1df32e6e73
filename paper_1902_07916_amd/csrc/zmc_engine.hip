// zmc_engine.hip -- level driver: lays out each level's cube list for all
// resident integrals, launches the level pipeline, reads back one record per
// integral, applies the stop rules of the tree search (ZMCintegral, Sec. 2.1)
// and builds the next level's list.
#include "zmc_engine.hpp"
#include "zmc_rtc.hpp"

#include <float.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <fstream>
#include <sstream>

namespace zmc {

namespace {
thread_local std::string g_err;

double now_ms()
{
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

uint64_t ipow_u64(uint64_t b, int e)
{
    uint64_t r = 1;
    for (int i = 0; i < e; ++i) r *= b;
    return r;
}

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Levels of at most this many tiles run the per-segment steps in the tile
// kernels' last blocks; larger ones launch them separately (each fused block
// pays an L2 write-back to publish its tile record).
constexpr int64_t kFuseMaxTiles = 256;

// Packed per-level tables: segments at 0, running totals, bucket segments,
// per-segment flags (uploaded as zeros), then the segments of the previous
// level's spawn and of the new roots (at most two per slot).
size_t prev_offset(int ns) { return align256((size_t)ns * sizeof(Segment)); }
size_t bseg_offset(int ns) { return prev_offset(ns) + align256((size_t)ns * sizeof(double2)); }
size_t flags_offset(int ns) { return bseg_offset(ns) + align256((size_t)ns * sizeof(BSeg)); }
size_t next_offset(int ns) { return align256(flags_offset(ns) + (size_t)ns * sizeof(int32_t)); }
size_t table_bytes(int max_segs) { return next_offset(max_segs) + 2 * (size_t)max_segs * sizeof(Segment); }

// Built-in occupancy variant per bucket (index into kWaveHints), measured by
// the tuner on gfx950 and embedded at build time; a tuning file overrides it.
#include "zmc_tune_default.inc"

int default_wave_hint(int f, int d, int e)
{
    if (f < 0 || f >= 8 || d < 1 || d > ZMC_MAX_DIM || e < 0 || e > 1) return 0;
    return kDefaultWaveHint[f][d][e] < kNumWaveHints ? kDefaultWaveHint[f][d][e] : 0;
}

int valid_block(int b) { return b == 64 || b == 128 || b == 256; }

int default_block(int f, int d, int e)
{
    if (f < 0 || f >= 8 || d < 1 || d > ZMC_MAX_DIM || e < 0 || e > 1) return kSampleThreads;
    return valid_block(kDefaultBlock[f][d][e]) ? kDefaultBlock[f][d][e] : kSampleThreads;
}

// parts per axis when a cube is split (0 in a request means bisection)
int split_of(const zmc_request& r) { return r.split ? r.split : 2; }

// children of a split cube: split^D
int64_t kids_of(const zmc_request& r) { return (int64_t)ipow_u64((uint64_t)split_of(r), r.dim); }
} // namespace

// Whether a request's cube ids can reach 2^64 (d^D * (split^D)^max_depth >
// 2^64): its levels then carry id bits 64..83 in a second array.
bool wide_ids(const zmc_request& r)
{
    unsigned __int128 top = 1;
    for (int i = 0; i < r.dim; ++i) top *= (unsigned __int128)r.divisions_per_axis;
    const unsigned __int128 lim = (unsigned __int128)1 << 64;
    for (int l = 0; l < r.max_depth && top <= lim; ++l)
        for (int i = 0; i < r.dim && top <= lim; ++i) top *= (unsigned __int128)split_of(r);
    return top > lim;
}

void set_error(const std::string& s) { g_err = s; }
const char* last_error() { return g_err.c_str(); }

#define ZMC_HIP(call)                                                                                      \
    do {                                                                                                   \
        hipError_t e_ = (call);                                                                            \
        if (e_ != hipSuccess) {                                                                            \
            set_error(std::string(#call) + ": " + hipGetErrorString(e_));                                  \
            return ZMC_EDEVICE;                                                                            \
        }                                                                                                  \
    } while (0)

// ---------------------------------------------------------------------------
TileTable::TileTable()
{
    for (int f = 0; f < 8; ++f)
        for (int d = 0; d <= ZMC_MAX_DIM; ++d)
            for (int e = 0; e < 2; ++e) {
                groups[f][d][e] = kDefaultGroups;
                hint[f][d][e] = default_wave_hint(f, d, e);
                threads[f][d][e] = default_block(f, d, e);
            }
}

// Tuning file: a JSON object whose keys "integrand:dim:eval" map to the
// number of 4-point groups per thread per chunk, e.g. {"1:6:1": 8}, whose
// keys "integrand:dim:eval:w" map to the minimum waves per SIMD of the
// occupancy variant (one of kWaveHints), e.g. {"1:6:1:w": 8}, and whose keys
// "integrand:dim:eval:b" map to the threads per sampling block (64, 128 or
// 256), e.g. {"1:6:1:b": 128}.
int TileTable::load(const char* path)
{
    std::ifstream in(path);
    if (!in) return -1;
    std::stringstream ss;
    ss << in.rdbuf();
    const std::string t = ss.str();
    size_t p = 0;
    while ((p = t.find('"', p)) != std::string::npos) {
        const size_t q = t.find('"', p + 1);
        if (q == std::string::npos) break;
        int f, d, e;
        char w = 0;
        const std::string key = t.substr(p + 1, q - p - 1);
        p = q + 1;
        const int nf = sscanf(key.c_str(), "%d:%d:%d:%c", &f, &d, &e, &w);
        if (nf < 3) continue;
        const size_t c = t.find(':', q);
        if (c == std::string::npos) break;
        const int g = atoi(t.c_str() + c + 1);
        if (!(f >= 0 && f < 8 && d >= 1 && d <= ZMC_MAX_DIM && e >= 0 && e < 2)) continue;
        if (nf == 3 && g >= 1 && g <= 64) groups[f][d][e] = g;
        if (nf == 4 && w == 'w')
            for (int h = 0; h < kNumWaveHints; ++h)
                if (kWaveHints[h] == g) hint[f][d][e] = h;
        if (nf == 4 && w == 'b' && valid_block(g)) threads[f][d][e] = g;
    }
    return 0;
}

// ---------------------------------------------------------------------------
int Engine::setup(char* base, size_t bytes, int max_slots, const TileTable* tiles, int device)
{
    region_ = base;
    region_bytes_ = bytes;
    max_slots_ = max_slots;
    tiles_ = tiles;
    device_ = device;
    size_t off = 0;
    auto carve = [&](size_t b) {
        off = (off + 255) & ~(size_t)255;
        char* p = base + off;
        off += b;
        return p;
    };
    d_slots_ = (SlotDesc*)carve(sizeof(SlotDesc) * max_slots);
    // per-level tables (segments, running totals, bucket segments), packed
    // so that one copy uploads them; the offsets depend on the level's size
    tab_bytes_ = table_bytes(max_slots);
    d_tab_ = carve(tab_bytes_);
    d_stats_ = (SegStats*)carve(sizeof(SegStats) * max_slots);
    d_seg_count_ = (int32_t*)carve(sizeof(int32_t) * max_slots);
    off = (off + 255) & ~(size_t)255;
    if (off + (16u << 20) > bytes) {
        set_error("arena too small for the slot tables");
        return ZMC_EINVAL;
    }
    arena_.init(base + off, bytes - off);
    // the tile counters start at 0 and every launch leaves them at 0
    ZMC_HIP(hipMemset(d_seg_count_, 0, sizeof(int32_t) * max_slots));
    ZMC_HIP(hipHostMalloc((void**)&h_slots_, sizeof(SlotDesc) * max_slots, hipHostMallocDefault));
    ZMC_HIP(hipHostMalloc((void**)&h_tab_, tab_bytes_, hipHostMallocDefault));
    ZMC_HIP(hipHostMalloc((void**)&h_nextsegs_, sizeof(Segment) * 2 * max_slots, hipHostMallocDefault));
    // the decision kernel writes each level's per-segment records straight
    // into this mapped host buffer, read after the level's synchronisation
    ZMC_HIP(hipHostMalloc((void**)&h_stats_, sizeof(SegStats) * max_slots, hipHostMallocMapped));
    ZMC_HIP(hipHostGetDevicePointer((void**)&d_hstats_, h_stats_, 0));
    h_segs_ = (Segment*)h_tab_;
    d_segs_ = (Segment*)d_tab_;
    ZMC_HIP(hipDeviceGetAttribute(&n_cu_, hipDeviceAttributeMultiprocessorCount, device));
    ZMC_HIP(hipEventCreate(&ev_sample0_));
    ZMC_HIP(hipEventCreate(&ev_sample1_));
    slots_.assign(max_slots, HostSlot());
    return ZMC_OK;
}

void Engine::teardown()
{
    void* hs[] = {h_slots_, h_tab_, h_nextsegs_, h_stats_};
    for (void* p : hs)
        if (p) (void)hipHostFree(p);
    h_slots_ = nullptr;
    h_tab_ = nullptr;
    h_segs_ = h_nextsegs_ = nullptr;
    h_bsegs_ = nullptr;
    h_stats_ = d_hstats_ = nullptr;
    h_prev_ = nullptr;
    if (ev_sample0_) (void)hipEventDestroy(ev_sample0_);
    if (ev_sample1_) (void)hipEventDestroy(ev_sample1_);
    ev_sample0_ = ev_sample1_ = nullptr;
    slots_.clear();
    cap_cache_.clear();
}

// Chunk of one sampling unit (one wave): 4 * 64 * groups points, with groups
// the smaller of the tile table's cap for the bucket and what N needs, so a
// request's chunking depends only on its own parameters.
int groups_for(const zmc_request& r, const TileTable& t)
{
    const int64_t need = ceil_div(r.samples_per_cube, 4LL * 64);
    return (int)std::max<int64_t>(1, std::min<int64_t>(need, t.get(r.integrand, r.dim, r.eval)));
}

int chunks_for(const zmc_request& r, const TileTable& t)
{
    const int64_t chunk = 4LL * 64 * groups_for(r, t);
    return (int)ceil_div(r.samples_per_cube, chunk);
}

int Engine::groups_of(const zmc_request& r) const { return groups_for(r, *tiles_); }

int Engine::nch_of(const zmc_request& r) const { return chunks_for(r, *tiles_); }

int Engine::capacity(int integrand, int dim, int eval, bool keep_s2, int block)
{
    const int hint = keep_s2 ? kSumsVariant : tiles_->waves(integrand, dim, eval);
    const int key = ((integrand * 1000 + dim * 2 + eval) * (kNumWaveHints + 1) + hint) * 8 + block / 64;
    auto it = cap_cache_.find(key);
    if (it != cap_cache_.end()) return it->second;
    int nb = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, sample_kernel_ptr(integrand, dim, eval, hint),
                                                                block, 0);
    if (e != hipSuccess || nb < 1) nb = 1;
    const int cap = nb * std::max(n_cu_, 1);
    cap_cache_[key] = cap;
    return cap;
}

int Engine::fill_slot_desc(int slot, const zmc_request& r, hipStream_t st)
{
    SlotDesc& d = h_slots_[slot];
    memset(&d, 0, sizeof(d));
    d.integrand = r.integrand;
    d.dim = r.dim;
    d.eval = r.eval;
    d.divisions = r.divisions_per_axis;
    d.trials = r.trials;
    d.max_depth = r.max_depth;
    d.groups = groups_of(r);
    d.nch = nch_of(r);
    d.samples = r.samples_per_cube;
    d.max_cubes = r.max_cubes_per_level > 0 ? r.max_cubes_per_level : ZMC_DEFAULT_MAX_CUBES;
    d.sigma_mult = r.sigma_mult;
    d.rtol = r.rtol;
    d.seed = r.seed;
    d.split = split_of(r);
    d.kids = (int32_t)kids_of(r);
    d.scope = r.threshold_scope;
    for (int i = 0; i < r.dim; ++i) {
        d.lower[i] = r.lower[i];
        d.h0[i] = (r.upper[i] - r.lower[i]) / (double)r.divisions_per_axis;
    }
    for (int j = 0; j < r.n_params && j < ZMC_MAX_PARAMS; ++j) d.params[j] = r.params[j];
    ZMC_HIP(hipMemcpyAsync(d_slots_ + slot, &d, sizeof(SlotDesc), hipMemcpyHostToDevice, st));
    return ZMC_OK;
}

// Bytes one integral can hold at its largest level: current list + work
// arrays + next list, with the next level bounded by Cantelli's inequality
// (at most n / (1 + sigma_mult^2) cubes exceed mean + sigma_mult * std; with
// per-parent thresholds the bound holds in every sibling group, so for the
// level too) and by the per-level cap.  Per cube of a level, step() takes
// its uid, the partial sums, m, s, the selection byte, a share of the tile
// records (96 bytes per 1024 cubes) and, with per-parent thresholds, a share
// of the per-group thresholds (8 bytes per kids cubes); every allocation is
// rounded up to 256 bytes.
size_t Engine::reservation_bytes(const zmc_request& r) const { return request_bytes(r, *tiles_); }

size_t request_bytes(const zmc_request& r, const TileTable& t)
{
    const int64_t cap = r.max_cubes_per_level > 0 ? r.max_cubes_per_level : ZMC_DEFAULT_MAX_CUBES;
    const int64_t k = (int64_t)ipow_u64((uint64_t)r.divisions_per_axis, r.dim);
    int64_t n = k, worst = k, worst_next = 0;
    for (int l = 0; l < r.max_depth; ++l) {
        const double frac = r.sigma_mult > 0 ? 1.0 / (1.0 + r.sigma_mult * r.sigma_mult) : 1.0;
        int64_t nsel = (int64_t)floor((double)n * frac);
        if (r.sigma_mult == 0.0) nsel = n - 1;
        int64_t nn = nsel * kids_of(r);
        if (nn > cap || nn < 0) nn = cap;
        worst_next = std::max(worst_next, nn);
        worst = std::max(worst, nn);
        n = nn;
        if (n == 0) break;
    }
    const int64_t kids = kids_of(r);
    const int64_t per_group_thr = r.threshold_scope == 1 ? (8 + kids - 1) / kids : 0;
    const int64_t per_tile = (int64_t)sizeof(TileRec);
    const int64_t id_bytes = wide_ids(r) ? 8 + 4 : 8; // ids above 2^64 take a second array
    const int64_t per_cube = id_bytes + 16LL * r.trials * chunks_for(r, t) + 8 + 8 + 1 + per_group_thr;
    const int64_t tiles = ceil_div(worst, kTileCubes) + 1;
    return (size_t)(worst * per_cube + tiles * per_tile + worst_next * id_bytes + 10 * 256 + 4 * 4096);
}

void Engine::record_level(HostSlot& hs, const SegStats& S, int64_t n, double ms, float sample_ms, int launches)
{
    zmc_result& R = hs.res;
    const int l = hs.level;
    R.sample_ms_per_level[l] = sample_ms;
    R.sample_launches_per_level[l] = launches;
    R.levels_run = l + 1;
    R.cubes_per_level[l] = (uint64_t)n;
    R.selected_per_level[l] = (uint64_t)S.n_sel;
    R.thr_per_level[l] = S.thr;
    R.min_margin_per_level[l] = (S.min_margin >= DBL_MAX) ? INFINITY : S.min_margin;
    R.ms_per_level[l] = (float)ms;
    R.n_samples += (uint64_t)n * (uint64_t)hs.req.trials * (uint64_t)hs.req.samples_per_cube;
    R.n_cubes += (uint64_t)n;
    hs.totM = S.totM;
    hs.totS2 = S.totS2;
    if (S.decision == kTruncated) R.flags |= ZMC_F_TRUNCATED;
    if (S.decision == kRtolMet) R.flags |= ZMC_F_RTOL_MET;
    if (S.nonfinite) R.status = ZMC_ENONFINITE;
    if (S.range_lost) R.flags |= ZMC_F_FP32_RANGE;
}

void Engine::finish(HostSlot& hs)
{
    zmc_result& R = hs.res;
    if (R.status != ZMC_OK) {
        // a failed or cancelled request has no estimate
        R.integral = R.std = R.stderr_ = NAN;
        return;
    }
    R.integral = hs.totM;
    R.std = sqrt(hs.totS2);
    R.stderr_ = sqrt(hs.totS2 / (double)(hs.req.trials - 1));
}

static void init_result(zmc_result& R)
{
    memset(&R, 0, sizeof(R));
    for (int l = 0; l < ZMC_MAX_LEVELS; ++l) {
        R.thr_per_level[l] = NAN;
        R.min_margin_per_level[l] = NAN;
    }
    R.integral = R.std = R.stderr_ = NAN;
}

// ---------------------------------------------------------------------------
// One level over the whole current list.
int Engine::step(hipStream_t st, const std::vector<LiveSeg>& live, uint64_t* cur_uid, int cur_side,
                 zmc_trace* trace, bool stats_only, bool want_sums)
{
    const int ns = (int)live.size();
    int64_t cube = 0, part = 0, tile = 0, groups = 0;
    bool any_thr = false;
    h_prev_ = (double2*)(h_tab_ + prev_offset(ns));
    h_bsegs_ = (BSeg*)(h_tab_ + bseg_offset(ns));
    d_prev_ = (double2*)(d_tab_ + prev_offset(ns));
    d_bsegs_ = (BSeg*)(d_tab_ + bseg_offset(ns));
    for (int i = 0; i < ns; ++i) {
        HostSlot& hs = slots_[live[i].slot];
        const zmc_request& r = hs.req;
        const int64_t n = live[i].n_cubes;
        if (n < 1) {
            set_error("internal: empty segment in a level list");
            return ZMC_EINVAL;
        }
        Segment& g = h_segs_[i];
        memset(&g, 0, sizeof(g));
        g.slot = live[i].slot;
        g.level = hs.level;
        g.cube_base = cube;
        g.n_cubes = n;
        g.part_base = part;
        g.tile_base = tile;
        g.n_tiles = ceil_div(n, kTileCubes);
        g.need_thr = (!stats_only && hs.level < r.max_depth) ? 1 : 0;
        any_thr |= g.need_thr != 0;
        // per-parent thresholds: below the roots, the list holds whole groups
        // of siblings in spawn order; a single group is the level itself
        const int64_t kids = kids_of(r);
        g.group_base = groups;
        g.group_size = 0;
        if (g.need_thr && r.threshold_scope == 1 && hs.level > 0 && n > kids) {
            g.group_size = (int32_t)kids;
            groups += n / kids;
        }
        h_prev_[i] = make_double2(hs.totM, hs.totS2);
        cube += n;
        part += n * (int64_t)r.trials * nch_of(r);
        tile += g.n_tiles;
    }
    n_list_ = cube;
    n_tiles_ = tile;
    cur_uid_ = cur_uid;
    double2* partial = (double2*)arena_.alloc(cur_side, (size_t)part * sizeof(double2));
    cur_m_ = (double*)arena_.alloc(cur_side, (size_t)cube * sizeof(double));
    cur_s_ = (double*)arena_.alloc(cur_side, (size_t)cube * sizeof(double));
    cur_sel_ = (uint8_t*)arena_.alloc(cur_side, (size_t)cube);
    cur_tiles_ = (TileRec*)arena_.alloc(cur_side, (size_t)tile * sizeof(TileRec));
    double* gthr = groups ? (double*)arena_.alloc(cur_side, (size_t)groups * sizeof(double)) : nullptr;
    cur_S1_ = cur_S2_ = nullptr;
    // per-(cube, trial) sums are only kept for a single integral (trace,
    // cube estimates), where every cube has the same number of trials
    const bool sums = ns == 1 && (want_sums || trace != nullptr);
    int64_t n_trial_entries = 0;
    if (sums) {
        for (int i = 0; i < ns; ++i) n_trial_entries += live[i].n_cubes * slots_[live[i].slot].req.trials;
        cur_S1_ = (double*)arena_.alloc(cur_side, (size_t)n_trial_entries * sizeof(double));
        cur_S2_ = (double*)arena_.alloc(cur_side, (size_t)n_trial_entries * sizeof(double));
    }
    if (!partial || !cur_m_ || !cur_s_ || !cur_sel_ || !cur_tiles_ || (sums && (!cur_S1_ || !cur_S2_)) ||
        (groups && !gthr)) {
        set_error("arena exhausted");
        return ZMC_ENOMEM;
    }


    // sampling: one persistent launch per (integrand, dim, eval) bucket
    std::map<int, std::vector<int>> buckets;
    for (int i = 0; i < ns; ++i) {
        const zmc_request& r = slots_[live[i].slot].req;
        buckets[r.integrand * 1000 + r.dim * 2 + r.eval].push_back(i);
    }
    int nb = 0;
    struct Launch {
        int off, count, integrand, dim, eval;
        int64_t units, unit_samples;
    };
    std::vector<Launch> launches;
    for (auto& kv : buckets) {
        Launch L;
        L.off = nb;
        L.count = (int)kv.second.size();
        const zmc_request& r0 = slots_[live[kv.second[0]].slot].req;
        L.integrand = r0.integrand;
        L.dim = r0.dim;
        L.eval = r0.eval;
        L.unit_samples = 256LL * groups_of(r0);
        int64_t u = 0;
        for (int i : kv.second) {
            const zmc_request& r = slots_[live[i].slot].req;
            h_bsegs_[nb].unit_base = u;
            h_bsegs_[nb].seg = i;
            h_bsegs_[nb].pad = 0;
            ++nb;
            u += live[i].n_cubes * (int64_t)r.trials * nch_of(r);
        }
        L.units = u;
        launches.push_back(L);
    }
    int32_t* h_flags = (int32_t*)(h_tab_ + flags_offset(ns));
    int32_t* d_flags = (int32_t*)(d_tab_ + flags_offset(ns));
    memset(h_flags, 0, (size_t)ns * sizeof(int32_t));
    size_t up = flags_offset(ns) + (size_t)ns * sizeof(int32_t);
    if (pend_next_) {
        const size_t off = next_offset(ns);
        memcpy(h_tab_ + off, h_nextsegs_, (size_t)pend_n_up_ * sizeof(Segment));
        up = off + (size_t)pend_n_up_ * sizeof(Segment);
    }
    ZMC_HIP(hipMemcpyAsync(d_tab_, h_tab_, up, hipMemcpyHostToDevice, st));
    if (pend_next_) {
        // this level's list: children of the last level's selected cubes,
        // then the roots of new integrals
        Segment* d_next = (Segment*)(d_tab_ + next_offset(ns));
        if (pend_la_.n_segs > 0) pend_la_.segs = d_next;
        if (pend_ra_.n_segs > 0) pend_ra_.segs = d_next + pend_n_spawn_segs_;
        pend_next_ = false;
        ZMC_HIP(launch_next_list(pend_la_, pend_ra_, st));
    }
    ZMC_HIP(hipEventRecord(ev_sample0_, st));
    int n_launch = 0;
    for (const Launch& L : launches) {
        if (L.units <= 0) continue;
        SampleArgs a;
        a.slots = d_slots_;
        a.segs = d_segs_;
        a.bsegs = d_bsegs_ + L.off;
        a.n_bsegs = L.count;
        a.uid = cur_uid;
        a.uid_hi = cur_hi_;
        a.partial = partial;
        a.seg_flags = d_flags;
        // one launch, or launches of at most chunk_samples_ samples each
        int64_t chunk = L.units;
        if (chunk_samples_ > 0) chunk = std::max<int64_t>(1, chunk_samples_ / L.unit_samples);
        for (int64_t u0 = 0; u0 < L.units; u0 += chunk) {
            a.unit0 = u0;
            a.total_units = std::min(chunk, L.units - u0);
            if (L.integrand >= kUserBase) {
                const int rc = rtc_launch(L.integrand, L.dim, L.eval, st, a);
                if (rc != ZMC_OK) return rc;
            } else {
                const int block = tiles_->block(L.integrand, L.dim, L.eval);
                const int64_t cap = capacity(L.integrand, L.dim, L.eval, sums, block);
                const int grid = (int)std::min<int64_t>(ceil_div(a.total_units, block / 64), cap);
                const int hint = sums ? kSumsVariant : tiles_->waves(L.integrand, L.dim, L.eval);
                ZMC_HIP(launch_sample(L.integrand, L.dim, L.eval, hint, grid, block, st, a));
            }
            ++n_launch;
        }
    }
    ZMC_HIP(hipEventRecord(ev_sample1_, st));

    LevelArgs la;
    memset(&la, 0, sizeof(la));
    la.slots = d_slots_;
    la.segs = d_segs_;
    la.n_segs = ns;
    la.n_tiles = tile;
    la.uid = cur_uid;
    la.uid_hi = cur_hi_;
    la.partial = partial;
    la.m = cur_m_;
    la.s = cur_s_;
    la.sel = cur_sel_;
    la.tiles = cur_tiles_;
    la.stats = d_stats_;
    la.prev_tot = d_prev_;
    la.tr_S1 = cur_S1_;
    la.tr_S2 = cur_S2_;
    la.gthr = gthr;
    la.n_groups = groups;
    la.seg_count = d_seg_count_;
    la.host_stats = stats_only ? nullptr : d_hstats_;
    la.seg_flags = d_flags;
    // small levels fold the per-segment steps into the tile kernels; a
    // level of one-tile segments without per-parent thresholds runs them all
    // in one launch
    la.fused = tile <= kFuseMaxTiles ? 1 : 0;
    if (!stats_only && tile == ns && groups == 0) {
        ZMC_HIP(launch_level_small(la, st));
    } else {
        ZMC_HIP(launch_finalize(la, st));
        if (!stats_only) {
            if (any_thr) ZMC_HIP(launch_threshold(la, st));
            if (groups) ZMC_HIP(launch_group_threshold(la, st));
            ZMC_HIP(launch_select(la, st));
        }
    }
    if (trace && ns == 1) {
        const HostSlot& hs = slots_[live[0].slot];
        const int l = hs.level;
        if (l < trace->max_levels && l < ZMC_MAX_LEVELS) {
            trace->n[l] = cube;
            const int64_t c = std::min<int64_t>(cube, trace->capacity);
            const int n1 = hs.req.trials;
            if (c > 0) {
                if (trace->uid[l]) ZMC_HIP(hipMemcpyAsync(trace->uid[l], cur_uid, c * 8, hipMemcpyDeviceToHost, st));
                if (trace->uid_hi[l]) {
                    if (cur_hi_)
                        ZMC_HIP(hipMemcpyAsync(trace->uid_hi[l], cur_hi_, c * 4, hipMemcpyDeviceToHost, st));
                    else
                        memset(trace->uid_hi[l], 0, (size_t)c * 4);
                }
                if (trace->m[l]) ZMC_HIP(hipMemcpyAsync(trace->m[l], cur_m_, c * 8, hipMemcpyDeviceToHost, st));
                if (trace->s[l]) ZMC_HIP(hipMemcpyAsync(trace->s[l], cur_s_, c * 8, hipMemcpyDeviceToHost, st));
                if (trace->sel[l]) ZMC_HIP(hipMemcpyAsync(trace->sel[l], cur_sel_, c, hipMemcpyDeviceToHost, st));
                if (trace->S1[l])
                    ZMC_HIP(hipMemcpyAsync(trace->S1[l], cur_S1_, c * n1 * 8, hipMemcpyDeviceToHost, st));
                if (trace->S2[l])
                    ZMC_HIP(hipMemcpyAsync(trace->S2[l], cur_S2_, c * n1 * 8, hipMemcpyDeviceToHost, st));
            }
        }
    }
    ZMC_HIP(hipStreamSynchronize(st));
    ZMC_HIP(hipGetLastError());
    last_sample_launches_ = n_launch;
    last_sample_ms_ = 0.0f;
    ZMC_HIP(hipEventElapsedTime(&last_sample_ms_, ev_sample0_, ev_sample1_));
    return ZMC_OK;
}

// Lay out the next list: children of every continuing segment (in list
// order), then the roots of newly admitted integrals.  Their segments go up
// with the next level's table and one launch writes both (step()).
int Engine::next_list(hipStream_t st, std::vector<LiveSeg>& live, const std::vector<int>& split,
                      const std::vector<LiveSeg>& fresh, uint64_t*& cur_uid, int& cur_side)
{
    std::vector<LiveSeg> nxt;
    int64_t total = 0;
    const int ns = (int)live.size();
    bool any_split = false;
    for (int i = 0; i < ns; ++i) any_split |= split[i] != 0;
    const int n_spawn_segs = any_split ? ns : 0;
    Segment* spawn_segs = h_nextsegs_;
    Segment* root_segs = h_nextsegs_ + n_spawn_segs;
    for (int i = 0; i < n_spawn_segs; ++i) {
        spawn_segs[i] = h_segs_[i];
        spawn_segs[i].do_split = 0;
        spawn_segs[i].child_base = 0;
        if (split[i]) {
            HostSlot& hs = slots_[live[i].slot];
            const int64_t nc = h_stats_[i].n_sel * kids_of(hs.req);
            spawn_segs[i].do_split = 1;
            spawn_segs[i].child_base = total;
            total += nc;
            nxt.push_back({live[i].slot, nc});
        }
    }
    for (size_t j = 0; j < fresh.size(); ++j) {
        Segment& g = root_segs[j];
        memset(&g, 0, sizeof(g));
        g.slot = fresh[j].slot;
        g.cube_base = total;
        g.n_cubes = fresh[j].n_cubes;
        total += fresh[j].n_cubes;
        nxt.push_back(fresh[j]);
    }
    const int other = cur_side ^ 1;
    uint64_t* next_uid = nullptr;
    uint32_t* next_hi = nullptr;
    bool wide = false;
    for (const LiveSeg& g : nxt) wide |= slots_[g.slot].wide;
    if (total > 0) {
        next_uid = (uint64_t*)arena_.alloc(other, (size_t)total * sizeof(uint64_t));
        if (wide) next_hi = (uint32_t*)arena_.alloc(other, (size_t)total * sizeof(uint32_t));
        if (!next_uid || (wide && !next_hi)) {
            set_error("arena exhausted (next level list)");
            return ZMC_ENOMEM;
        }
    }
    // the upload and the launch go with the next level's table (step())
    pend_n_up_ = n_spawn_segs + (int)fresh.size();
    pend_n_spawn_segs_ = n_spawn_segs;
    memset(&pend_la_, 0, sizeof(pend_la_));
    memset(&pend_ra_, 0, sizeof(pend_ra_));
    if (any_split) {
        pend_la_.slots = d_slots_;
        pend_la_.n_segs = ns;
        pend_la_.n_tiles = n_tiles_;
        pend_la_.uid = cur_uid;
        pend_la_.uid_hi = cur_hi_;
        pend_la_.sel = cur_sel_;
        pend_la_.tiles = cur_tiles_;
        pend_la_.next_uid = next_uid;
        pend_la_.next_uid_hi = next_hi;
    }
    if (!fresh.empty()) {
        pend_ra_.n_segs = (int)fresh.size();
        int64_t mx = 1;
        for (auto& f : fresh) mx = std::max(mx, f.n_cubes);
        pend_ra_.blocks_per_seg = (int)std::min<int64_t>(64, ceil_div(mx, 4096));
        pend_ra_.uid = next_uid;
        pend_ra_.uid_hi = next_hi;
    }
    pend_next_ = pend_n_up_ > 0;
    // levels advance for the split segments
    for (int i = 0; i < ns; ++i)
        if (split[i]) slots_[live[i].slot].level += 1;
    for (auto& f : fresh) slots_[f.slot].level = 0;
    arena_.reset(cur_side);
    cur_side = other;
    cur_uid = next_uid;
    cur_hi_ = next_hi;
    live.swap(nxt);
    return ZMC_OK;
}

// ---------------------------------------------------------------------------
// Shared level loop of run() and serving.
int Engine::drive(hipStream_t st, Admission& adm, zmc_trace* trace, const std::atomic<bool>* stop_flag,
                  std::atomic<uint64_t>* levels_stepped)
{
    std::vector<int> free_ids;
    for (int i = max_slots_ - 1; i >= 0; --i) free_ids.push_back(i);
    std::vector<LiveSeg> live;
    uint64_t* cur_uid = nullptr;
    cur_hi_ = nullptr;
    pend_next_ = false;
    int cur_side = 0;
    arena_.reset(0);
    arena_.reset(1);
    size_t reserved = 0;
    bool more = true;
    int rc_all = ZMC_OK;

    while (true) {
        std::vector<int> split(live.size(), 0);
        if (!live.empty()) {
            const double t0 = now_ms();
            int rc = step(st, live, cur_uid, cur_side, trace, false, false);
            const double ms = now_ms() - t0;
            if (levels_stepped) levels_stepped->fetch_add(1, std::memory_order_relaxed);
            for (size_t i = 0; i < live.size(); ++i) {
                HostSlot& hs = slots_[live[i].slot];
                bool done = true;
                if (rc != ZMC_OK) {
                    hs.res.status = rc;
                } else {
                    const SegStats& S = h_stats_[i];
                    record_level(hs, S, live[i].n_cubes, ms, last_sample_ms_, last_sample_launches_);
                    if (hs.res.status == ZMC_OK && S.decision == kSplit) done = false;
                    if (adm.cancelled && adm.cancelled(hs.ticket)) {
                        hs.res.status = ZMC_ECANCELED;
                        done = true;
                    }
                }
                if (done) {
                    finish(hs);
                    adm.retire(hs);
                    reserved -= std::min(reserved, hs.reserve);
                    free_ids.push_back(live[i].slot);
                } else {
                    split[i] = 1;
                }
            }
            if (rc != ZMC_OK) {
                rc_all = rc;
                live.clear();
                split.clear();
                cur_uid = nullptr;
                cur_hi_ = nullptr;
                pend_next_ = false;
                arena_.reset(0);
                arena_.reset(1);
                if (rc == ZMC_EDEVICE) return rc;
            }
        }
        if (stop_flag && stop_flag->load(std::memory_order_acquire)) {
            // retire what is still resident
            for (size_t i = 0; i < live.size(); ++i)
                if (split[i]) {
                    HostSlot& hs = slots_[live[i].slot];
                    hs.res.status = ZMC_ECANCELED;
                    finish(hs);
                    adm.retire(hs);
                }
            return rc_all;
        }
        // admission at the level boundary
        std::vector<HostSlot> incoming;
        bool idle = true;
        double next_samples = 0.0; // samples of the next level before admission
        for (size_t i = 0; i < split.size(); ++i) {
            if (!split[i]) continue;
            idle = false;
            const zmc_request& r = slots_[live[i].slot].req;
            next_samples += (double)h_stats_[i].n_sel * (double)kids_of(r) * (double)r.samples_per_cube * r.trials;
        }
        if (more) {
            const size_t budget = arena_.size() > reserved ? arena_.size() - reserved : 0;
            more = adm.admit(incoming, (int)free_ids.size(), budget, idle, next_samples);
        }
        std::vector<LiveSeg> fresh;
        for (HostSlot& in : incoming) {
            const int id = free_ids.back();
            free_ids.pop_back();
            slots_[id] = in;
            HostSlot& hs = slots_[id];
            hs.wide = wide_ids(hs.req);
            hs.level = 0;
            hs.totM = hs.totS2 = 0.0;
            reserved += hs.reserve;
            int rc = fill_slot_desc(id, hs.req, st);
            if (rc != ZMC_OK) return rc;
            fresh.push_back({id, (int64_t)ipow_u64((uint64_t)hs.req.divisions_per_axis, hs.req.dim)});
        }
        if (idle && fresh.empty()) {
            if (!more) break;
            live.clear();
            continue;
        }
        int rc = next_list(st, live, split, fresh, cur_uid, cur_side);
        if (rc == ZMC_ENOMEM) {
            // the next level does not fit: every affected integral fails
            rc_all = rc;
            for (size_t i = 0; i < live.size(); ++i)
                if (i < split.size() && split[i]) {
                    HostSlot& hs = slots_[live[i].slot];
                    hs.res.status = ZMC_ENOMEM;
                    finish(hs);
                    adm.retire(hs);
                    reserved -= std::min(reserved, hs.reserve);
                    free_ids.push_back(live[i].slot);
                }
            for (auto& f : fresh) {
                HostSlot& hs = slots_[f.slot];
                hs.res.status = ZMC_ENOMEM;
                finish(hs);
                adm.retire(hs);
                reserved -= std::min(reserved, hs.reserve);
                free_ids.push_back(f.slot);
            }
            live.clear();
            cur_uid = nullptr;
            cur_hi_ = nullptr;
            pend_next_ = false;
            arena_.reset(0);
            arena_.reset(1);
            continue;
        }
        if (rc != ZMC_OK) return rc;
    }
    return rc_all;
}

int Engine::run(const zmc_request* reqs, int n, hipStream_t st, zmc_result* outs, zmc_trace* trace)
{
    if (n > max_slots_) {
        set_error("more requests than slots");
        return ZMC_EINVAL;
    }
    std::vector<int> id_of_slot(max_slots_, -1);
    int given = 0;
    Admission adm;
    adm.admit = [&](std::vector<HostSlot>& out, int free_slots, size_t, bool, double) {
        if (given == 0) {
            for (int i = 0; i < n && i < free_slots; ++i) {
                HostSlot hs;
                hs.req = reqs[i];
                init_result(hs.res);
                hs.ticket = (uint64_t)i;
                // in a batch, a request whose worst-case tree cannot fit the
                // arena even alone fails by itself instead of taking the
                // batch's shared levels down
                if (n > 1 && reservation_bytes(reqs[i]) > budget_bytes()) {
                    hs.res.status = ZMC_ENOMEM;
                    outs[i] = hs.res;
                    continue;
                }
                out.push_back(hs);
            }
            given = n;
        }
        return false;
    };
    adm.retire = [&](HostSlot& hs) {
        outs[hs.ticket] = hs.res;
    };
    adm.cancelled = nullptr;
    const double t0 = now_ms();
    int rc = drive(st, adm, n == 1 ? trace : nullptr, nullptr, nullptr);
    const double t1 = now_ms();
    for (int i = 0; i < n; ++i) outs[i].latency_ms = t1 - t0;
    return rc;
}

int Engine::cube_estimates(const zmc_request& req, int level, const uint64_t* uids, int64_t n, double* m,
                           double* s, double* S1, double* S2, hipStream_t st)
{
    if (n <= 0) return ZMC_OK;
    arena_.reset(0);
    arena_.reset(1);
    HostSlot& hs = slots_[0];
    hs = HostSlot();
    hs.req = req;
    init_result(hs.res);
    hs.level = level;
    int rc = fill_slot_desc(0, req, st);
    if (rc != ZMC_OK) return rc;
    uint64_t* d_uid = (uint64_t*)arena_.alloc(1, (size_t)n * 8);
    if (!d_uid) return ZMC_ENOMEM;
    cur_hi_ = nullptr; // ids given here are below 2^64
    pend_next_ = false;
    ZMC_HIP(hipMemcpyAsync(d_uid, uids, (size_t)n * 8, hipMemcpyHostToDevice, st));
    std::vector<LiveSeg> live{{0, n}};
    rc = step(st, live, d_uid, 0, nullptr, true, S1 != nullptr || S2 != nullptr);
    if (rc != ZMC_OK) return rc;
    const int n1 = req.trials;
    if (m) ZMC_HIP(hipMemcpyAsync(m, cur_m_, n * 8, hipMemcpyDeviceToHost, st));
    if (s) ZMC_HIP(hipMemcpyAsync(s, cur_s_, n * 8, hipMemcpyDeviceToHost, st));
    if (S1) ZMC_HIP(hipMemcpyAsync(S1, cur_S1_, n * n1 * 8, hipMemcpyDeviceToHost, st));
    if (S2) ZMC_HIP(hipMemcpyAsync(S2, cur_S2_, n * n1 * 8, hipMemcpyDeviceToHost, st));
    ZMC_HIP(hipStreamSynchronize(st));
    arena_.reset(0);
    arena_.reset(1);
    return ZMC_OK;
}

int Engine::debug_philox(uint32_t k0, uint32_t k1, const uint32_t* ctr, int64_t n, uint32_t* out, hipStream_t st)
{
    arena_.reset(0);
    uint32_t* dc = (uint32_t*)arena_.alloc(0, (size_t)n * 16);
    uint32_t* dout = (uint32_t*)arena_.alloc(0, (size_t)n * 16);
    if (!dc || !dout) return ZMC_ENOMEM;
    ZMC_HIP(hipMemcpyAsync(dc, ctr, (size_t)n * 16, hipMemcpyHostToDevice, st));
    ZMC_HIP(launch_debug_philox(k0, k1, dc, dout, n, st));
    ZMC_HIP(hipMemcpyAsync(out, dout, (size_t)n * 16, hipMemcpyDeviceToHost, st));
    ZMC_HIP(hipStreamSynchronize(st));
    arena_.reset(0);
    return ZMC_OK;
}

int Engine::debug_points(const zmc_request& req, int level, uint64_t uid, int trial, int64_t s0, int64_t n,
                         double* x, hipStream_t st)
{
    arena_.reset(0);
    int rc = fill_slot_desc(0, req, st);
    if (rc != ZMC_OK) return rc;
    double* dx = (double*)arena_.alloc(0, (size_t)n * req.dim * 8);
    if (!dx) return ZMC_ENOMEM;
    ZMC_HIP(launch_debug_points(d_slots_, level, uid, trial, s0, n, dx, st));
    ZMC_HIP(hipMemcpyAsync(x, dx, (size_t)n * req.dim * 8, hipMemcpyDeviceToHost, st));
    ZMC_HIP(hipStreamSynchronize(st));
    arena_.reset(0);
    return ZMC_OK;
}

} // namespace zmc
