// zmc_engine.hpp -- host-side level driver of the tree search.
//
// An Engine owns one region of the caller's device arena.  It keeps every
// resident integral's descriptor in a device slot table and drives the tree
// search level by level for all of them at once: the current list of cubes
// is a sequence of segments (one per integral, each integral's cubes in uid
// order), the level pipeline runs over the whole list, one int per segment
// comes back (the split decision and counts), and the next list is laid out
// from it.  Memory for a level comes from a double-ended stack: the current
// list and its work arrays grow from one end, the next list from the other,
// and the ends swap every level.
#pragma once

#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <atomic>
#include <vector>

#include "zmc.h"
#include "zmc_kernels.hpp"

namespace zmc {

// Double-ended stack allocator over a device region; 256-byte aligned.
class DualStack {
public:
    void init(char* base, size_t bytes)
    {
        base_ = base;
        size_ = bytes;
        lo_ = 0;
        hi_ = bytes;
    }
    void* alloc(int side, size_t bytes)
    {
        bytes = (bytes + 255) & ~(size_t)255;
        if (bytes > hi_ - lo_) return nullptr;
        if (side == 0) {
            void* p = base_ + lo_;
            lo_ += bytes;
            return p;
        }
        hi_ -= bytes;
        return base_ + hi_;
    }
    void reset(int side)
    {
        if (side == 0) lo_ = 0;
        else hi_ = size_;
    }
    size_t free_bytes() const { return hi_ - lo_; }
    size_t size() const { return size_; }

private:
    char* base_ = nullptr;
    size_t size_ = 0, lo_ = 0, hi_ = 0;
};

// Tile shape of the sampling kernel per (integrand, dim, eval): the cap on
// 4-point groups per lane per chunk (default 32; a chunk is one wave's unit),
// the occupancy variant and the block shape (threads per block: 64, 128 or
// 256).  Fixed per build or tuning file, never by the batch composition, so
// a request's result does not depend on its company (the group cap sets how
// a trial's points are split into units; the occupancy variant and the block
// shape change no arithmetic at all).
struct TileTable {
    int groups[8][ZMC_MAX_DIM + 1][2];
    int hint[8][ZMC_MAX_DIM + 1][2];    // index into kWaveHints
    int threads[8][ZMC_MAX_DIM + 1][2]; // threads per sampling block
    TileTable();
    int load(const char* path); // 0 on success
    int get(int integrand, int dim, int eval) const
    {
        // run-time compiled user integrands use the default cap
        return (integrand >= 0 && integrand < 8) ? groups[integrand][dim][eval] : kDefaultGroups;
    }
    int waves(int integrand, int dim, int eval) const
    {
        return (integrand >= 0 && integrand < 8) ? hint[integrand][dim][eval] : 0;
    }
    int block(int integrand, int dim, int eval) const
    {
        return (integrand >= 0 && integrand < 8) ? threads[integrand][dim][eval] : kSampleThreads;
    }
    static constexpr int kDefaultGroups = 32;
};

// Host view of one resident integral.
struct HostSlot {
    zmc_request req;
    zmc_result res;
    int level = 0;
    int64_t n_cubes = 0; // cubes at the current level
    double totM = 0.0, totS2 = 0.0;
    uint64_t ticket = 0;
    size_t reserve = 0;  // serving: worst-case bytes held for it
    bool wide = false;   // its cube ids can reach 2^64 (see wide_ids)
    bool cancel = false;
    std::chrono::steady_clock::time_point t_submit;
};

struct LiveSeg {
    int slot;
    int64_t n_cubes;
};

constexpr int64_t ZMC_DEFAULT_MAX_CUBES = 1LL << 24;

// 4-point groups per lane in one sampling unit, and units (chunks) per
// (cube, trial), of a request under a tile table.
int groups_for(const zmc_request& r, const TileTable& t);
int chunks_for(const zmc_request& r, const TileTable& t);
// Worst-case device bytes of one request's tree (see Engine::reservation_bytes).
size_t request_bytes(const zmc_request& r, const TileTable& t);
bool wide_ids(const zmc_request& r);

class Engine {
public:
    int setup(char* base, size_t bytes, int max_slots, const TileTable* tiles, int device);
    void teardown();

    // Run requests to completion (all admitted at once).  trace: only for
    // n == 1.  Returns ZMC_OK, or the first failure (per-request status in outs).
    int run(const zmc_request* reqs, int n, hipStream_t st, zmc_result* outs, zmc_trace* trace);

    // Sampling + per-cube reduction only, for an explicit cube list.
    int cube_estimates(const zmc_request& req, int level, const uint64_t* uids, int64_t n, double* m, double* s,
                       double* S1, double* S2, hipStream_t st);

    int debug_philox(uint32_t k0, uint32_t k1, const uint32_t* ctr, int64_t n, uint32_t* out, hipStream_t st);
    int debug_points(const zmc_request& req, int level, uint64_t uid, int trial, int64_t s0, int64_t n, double* x,
                     hipStream_t st);

    // Level loop shared by run() and serving: at every level boundary
    // `admit` may hand over new requests (they join with their roots),
    // `retire` receives every finished request, `cancelled` is polled.
    struct Admission {
        // called at each level boundary; next_samples = samples the resident
        // integrals take at the next level (0 when idle)
        std::function<bool(std::vector<HostSlot>& out, int free_slots, size_t free_budget, bool idle,
                           double next_samples)>
            admit;
        std::function<void(HostSlot& done)> retire;
        std::function<bool(uint64_t ticket)> cancelled;
    };
    int drive(hipStream_t st, Admission& adm, zmc_trace* trace, const std::atomic<bool>* stop_flag,
              std::atomic<uint64_t>* levels_stepped);

    size_t reservation_bytes(const zmc_request& r) const;
    size_t budget_bytes() const { return arena_.size(); }
    // 0 (default): one sampling launch per bucket and level; > 0: launches
    // of about this many samples each, so that a long level leaves the
    // device to launches on other streams between them
    void set_chunk_samples(int64_t n) { chunk_samples_ = n; }
    int nch_of(const zmc_request& r) const;
    int groups_of(const zmc_request& r) const;

private:
    int fill_slot_desc(int slot, const zmc_request& r, hipStream_t st);
    int step(hipStream_t st, const std::vector<LiveSeg>& live, uint64_t* cur_uid, int cur_side, zmc_trace* trace,
             bool stats_only, bool want_sums);
    int next_list(hipStream_t st, std::vector<LiveSeg>& live, const std::vector<int>& split,
                  const std::vector<LiveSeg>& fresh, uint64_t*& cur_uid, int& cur_side);
    int capacity(int integrand, int dim, int eval, bool keep_s2, int block);
    void record_level(HostSlot& hs, const SegStats& S, int64_t n, double ms, float sample_ms, int launches);
    void finish(HostSlot& hs);

    char* region_ = nullptr;
    size_t region_bytes_ = 0;
    int max_slots_ = 0;
    int device_ = 0;
    int n_cu_ = 0;
    const TileTable* tiles_ = nullptr;
    // fixed device tables
    SlotDesc* d_slots_ = nullptr;
    char* d_tab_ = nullptr;
    char* h_tab_ = nullptr;
    size_t tab_bytes_ = 0;
    int32_t* d_seg_count_ = nullptr;
    SegStats* d_hstats_ = nullptr;
    Segment* d_segs_ = nullptr;
    BSeg* d_bsegs_ = nullptr;
    SegStats* d_stats_ = nullptr;
    double2* d_prev_ = nullptr;
    // pinned host staging (each buffer is rewritten only after the stream
    // has been synchronised past its previous upload)
    SlotDesc* h_slots_ = nullptr;
    Segment* h_segs_ = nullptr;
    Segment* h_nextsegs_ = nullptr;
    BSeg* h_bsegs_ = nullptr;
    SegStats* h_stats_ = nullptr;
    double2* h_prev_ = nullptr;
    DualStack arena_;
    std::vector<HostSlot> slots_;
    std::map<int, int> cap_cache_;
    int64_t chunk_samples_ = 0;
    // arrays of the level last stepped (valid until its spawn is enqueued)
    uint64_t* cur_uid_ = nullptr;
    uint32_t* cur_hi_ = nullptr; // id bits 64..83 of the current list, or NULL
    double* cur_m_ = nullptr;
    double* cur_s_ = nullptr;
    uint8_t* cur_sel_ = nullptr;
    TileRec* cur_tiles_ = nullptr;
    double* cur_S1_ = nullptr;
    double* cur_S2_ = nullptr;
    int64_t n_list_ = 0;
    int64_t n_tiles_ = 0;
    // the next list's spawn / roots launch, laid out by next_list and issued
    // by the next step() after its table upload, which carries these
    // segments too (one copy per level)
    bool pend_next_ = false;
    LevelArgs pend_la_{};
    RootArgs pend_ra_{};
    int pend_n_up_ = 0;
    int pend_n_spawn_segs_ = 0;
    // GPU time of the last level's sampling launches
    hipEvent_t ev_sample0_ = nullptr, ev_sample1_ = nullptr;
    float last_sample_ms_ = 0.0f;
    int last_sample_launches_ = 0;
};

// Thread-local text of the last error.
void set_error(const std::string& s);
const char* last_error();

} // namespace zmc
