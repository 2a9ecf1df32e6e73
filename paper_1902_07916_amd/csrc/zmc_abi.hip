// zmc_abi.hip -- the extern "C" entry points declared in zmc.h: argument
// checks, the library context (arena split between the synchronous engine
// and the serving engine), and the serving thread (continuous batching at
// tree-level granularity).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <atomic>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "zmc.h"
#include "zmc_engine.hpp"
#include "zmc_rtc.hpp"

using namespace zmc;

namespace {

// One serving lane: an engine (its own slot table and arena share), the
// stream it launches on and the thread that drives it.  Lanes admit from one
// queue at their own level boundaries, so a request that arrives while one
// lane is in a long level starts on another at once; their sampling launches
// use more blocks than fit at a time, so the GPU interleaves the lanes' work.
struct Lane {
    Engine eng;
    hipStream_t st = nullptr;
    bool own_stream = false;
    std::thread th;
    double next_samples = 0.0; // the lane's next level, as of its last boundary (under Server::mu)
};

struct Server {
    std::vector<std::unique_ptr<Lane>> lanes;
    std::mutex mu;
    std::condition_variable cv_q, cv_done;
    std::deque<HostSlot> queue;
    size_t queue_cap = 65536;
    std::unordered_map<uint64_t, zmc_result> done;
    std::unordered_set<uint64_t> pending; // queued or resident
    std::unordered_set<uint64_t> cancelled;
    uint64_t next_ticket = 1;
    std::atomic<bool> stop{false};
    int running = 0;     // lanes whose thread has not returned (under mu)
    bool exited = false; // every lane has returned (under mu)
    uint64_t n_completed = 0;
    std::atomic<uint64_t> n_levels{0};
    int resident = 0;
    int rc = ZMC_OK;
};

// Serving lanes cut a level's sampling into launches of about this many
// samples (about 4 ms of device time for FP32 integrands).  A launch that fills the
// device holds its resources until its last block is dispatched: a kernel on
// another lane whose blocks need more registers or LDS than one retiring
// block frees waits for the whole launch otherwise.
constexpr int64_t kServeChunkSamples = int64_t(1) << 31;
// A busy lane whose next level takes more samples than this leaves newly
// arrived requests to a lighter lane: a request admitted there would wait for
// the whole of each heavy level before its own next level.
constexpr double kLightLevelSamples = 268435456.0; // 2^28

struct Context {
    bool inited = false;
    int device = 0;
    TileTable tiles;
    Engine sync_eng;
    std::mutex sync_mu;
    int default_eval = ZMC_EVAL_FP64; // evaluation mode of zmc_integrate()
    Server* server = nullptr;
    // zmc_integrate_noalloc: a one-integral engine over the device scratch
    Engine static_eng;
    std::mutex static_mu;
};

Context g;
std::mutex g_init_mu;

// Device scratch of zmc_integrate_noalloc, for callers that cannot allocate
// device memory: the arena of a one-integral engine, held by every device
// the library runs on until the process ends.  In host code `scratch` is a
// host-side stand-in for the symbol, not a device address; its address on a
// device comes from hipGetSymbolAddress (once per device, in zmc_init, with
// that device current) and only that address is ever passed on.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
constexpr int kMaxDevices = 64;
void* g_scratch_ptr[kMaxDevices] = {};

uint64_t ipow_sat(uint64_t b, int e, bool* ovf)
{
    uint64_t r = 1;
    *ovf = false;
    for (int i = 0; i < e; ++i) {
        if (b != 0 && r > UINT64_MAX / b) {
            *ovf = true;
            return UINT64_MAX;
        }
        r *= b;
    }
    return r;
}

int n_params_of(int id, int dim)
{
    switch (id) {
    case ZMC_GAUSS: return 2 + dim;
    case ZMC_SIN_SUM: return 0;
    case ZMC_GENZ_OSC: return 1 + dim;
    case ZMC_GENZ_PPEAK: return 2 * dim;
    case ZMC_GENZ_CPEAK: return dim;
    case ZMC_GENZ_GAUSS: return 2 * dim;
    case ZMC_CONST: return 1;
    case ZMC_MONOMIAL: return dim;
    default: return -1;
    }
}

int fail(int code, const char* msg)
{
    set_error(msg);
    return code;
}

// The argument rules of zmc_integrate (see zmc.h).
int validate(const zmc_request& r)
{
    if (r.dim < 1 || r.dim > ZMC_MAX_DIM) return fail(ZMC_EINVAL, "dim must be in 1..16");
    if (r.integrand >= kUserBase) {
        const int np = rtc_n_params(r.integrand);
        if (np < 0) return fail(ZMC_EINVAL, "unknown integrand");
        if (r.n_params != np) return fail(ZMC_EINVAL, "wrong number of params");
    } else {
        if (r.integrand < 0 || r.integrand > ZMC_MONOMIAL) return fail(ZMC_EINVAL, "unknown integrand");
        if (r.n_params != n_params_of(r.integrand, r.dim)) return fail(ZMC_EINVAL, "wrong number of params");
    }
    if (r.integrand == ZMC_MONOMIAL)
        for (int j = 0; j < r.n_params; ++j)
            if (!(r.params[j] >= 0.0 && r.params[j] <= 16.0 && r.params[j] == floor(r.params[j])))
                return fail(ZMC_EINVAL, "monomial exponents must be integers in 0..16");
    if (r.eval != ZMC_EVAL_FP64 && r.eval != ZMC_EVAL_FP32) return fail(ZMC_EINVAL, "unknown eval mode");
    if (r.divisions_per_axis < 1) return fail(ZMC_EINVAL, "divisions_per_axis must be >= 1");
    if (r.split != 0 && (r.split < 2 || r.split > 64)) return fail(ZMC_EINVAL, "split must be 0 (= 2) or in 2..64");
    if (r.threshold_scope != 0 && r.threshold_scope != 1) return fail(ZMC_EINVAL, "threshold_scope must be 0 or 1");
    const uint64_t b = r.split ? (uint64_t)r.split : 2u;
    {
        uint64_t kids = 1;
        for (int i = 0; i < r.dim; ++i) {
            kids *= b;
            if (kids > (1ull << 24)) return fail(ZMC_EINVAL, "split^dim must be <= 2^24");
        }
    }
    if (r.samples_per_cube < 1) return fail(ZMC_EINVAL, "samples_per_cube must be >= 1");
    if ((uint64_t)r.samples_per_cube * (uint64_t)r.dim > (1ull << 34))
        return fail(ZMC_EINVAL, "samples_per_cube * dim must be <= 2^34");
    if (r.trials < 2 || r.trials > 255) return fail(ZMC_EINVAL, "trials must be in 2..255");
    if (r.max_depth < 0 || r.max_depth >= ZMC_MAX_LEVELS) return fail(ZMC_EINVAL, "max_depth must be in 0..15");
    if (!isfinite(r.sigma_mult) || r.sigma_mult < 0.0) return fail(ZMC_EINVAL, "sigma_mult must be finite, >= 0");
    if (!isfinite(r.rtol) || r.rtol < 0.0) return fail(ZMC_EINVAL, "rtol must be finite, >= 0");
    if (r.max_cubes_per_level < 0) return fail(ZMC_EINVAL, "max_cubes_per_level must be >= 0");
    for (int i = 0; i < r.dim; ++i)
        if (!isfinite(r.lower[i]) || !isfinite(r.upper[i]) || !(r.lower[i] < r.upper[i]))
            return fail(ZMC_EINVAL, "bounds must be finite with lower < upper");
    bool ovf = false;
    const uint64_t k = ipow_sat((uint64_t)r.divisions_per_axis, r.dim, &ovf);
    if (ovf) return fail(ZMC_EINVAL, "d^D overflows 64 bits");
    {
        // every cube id is below d^D * (b^D)^max_depth, which must fit the
        // 84 id bits; the lattice cells per axis, d * b^max_depth, 64 bits
        const unsigned __int128 lim = (unsigned __int128)1 << kIdBits;
        unsigned __int128 top = k, cells = (unsigned __int128)r.divisions_per_axis;
        for (int l = 0; l < r.max_depth; ++l) {
            for (int i = 0; i < r.dim; ++i) {
                top *= b;
                if (top > lim) return fail(ZMC_EINVAL, "cube ids would overflow 84 bits");
            }
            cells *= b;
            if (cells > ((unsigned __int128)1 << 64)) return fail(ZMC_EINVAL, "lattice cells per axis overflow 64 bits");
        }
    }
    const int64_t cap = r.max_cubes_per_level > 0 ? r.max_cubes_per_level : ZMC_DEFAULT_MAX_CUBES;
    if (k > (uint64_t)cap) return fail(ZMC_EINVAL, "d^D exceeds max_cubes_per_level");
    return ZMC_OK;
}

zmc_request make_request(int integrand_id, const double* params, int n_params, int dim, const double* lower,
                         const double* upper, int d, int64_t N, int trials, int max_depth, double sigma_mult,
                         uint64_t seed, int eval)
{
    zmc_request r;
    memset(&r, 0, sizeof(r));
    r.integrand = integrand_id;
    r.dim = dim;
    r.divisions_per_axis = d;
    r.trials = trials;
    r.max_depth = max_depth;
    r.eval = eval;
    r.n_params = n_params;
    r.samples_per_cube = N;
    r.sigma_mult = sigma_mult;
    r.seed = seed;
    for (int i = 0; i < dim && i < ZMC_MAX_DIM; ++i) {
        r.lower[i] = lower ? lower[i] : NAN;
        r.upper[i] = upper ? upper[i] : NAN;
    }
    for (int j = 0; j < n_params && j < ZMC_MAX_PARAMS; ++j) r.params[j] = params ? params[j] : NAN;
    if (n_params > ZMC_MAX_PARAMS || n_params < 0) r.n_params = -1;
    return r;
}

void init_result(zmc_result& R)
{
    memset(&R, 0, sizeof(R));
    for (int l = 0; l < ZMC_MAX_LEVELS; ++l) {
        R.thr_per_level[l] = NAN;
        R.min_margin_per_level[l] = NAN;
    }
    R.integral = R.std = R.stderr_ = NAN;
}

double now_ms()
{
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

void server_main(Server* S, Lane* L, int device)
{
    (void)hipSetDevice(device);
    Engine::Admission adm;
    adm.admit = [S, L](std::vector<HostSlot>& out, int free_slots, size_t budget, bool idle,
                       double next_samples) {
        std::unique_lock<std::mutex> lk(S->mu);
        L->next_samples = next_samples;
        if (idle) {
            while (S->queue.empty() && !S->stop) S->cv_q.wait_for(lk, std::chrono::milliseconds(20));
        } else if (next_samples > kLightLevelSamples) {
            for (auto& o : S->lanes)
                if (o.get() != L && o->next_samples < next_samples) return !S->stop;
        }
        while (!S->queue.empty() && free_slots > 0) {
            HostSlot& hs = S->queue.front();
            if (S->cancelled.count(hs.ticket)) {
                zmc_result R;
                init_result(R);
                R.status = ZMC_ECANCELED;
                S->done[hs.ticket] = R;
                S->pending.erase(hs.ticket);
                S->cancelled.erase(hs.ticket);
                S->queue.pop_front();
                S->cv_done.notify_all();
                continue;
            }
            if (hs.reserve > L->eng.budget_bytes()) {
                zmc_result R;
                init_result(R);
                R.status = ZMC_ENOMEM;
                S->done[hs.ticket] = R;
                S->pending.erase(hs.ticket);
                S->queue.pop_front();
                S->cv_done.notify_all();
                continue;
            }
            if (hs.reserve > budget) break; // wait for memory to free up
            budget -= hs.reserve;
            --free_slots;
            out.push_back(hs);
            S->queue.pop_front();
            ++S->resident;
        }
        return !S->stop;
    };
    adm.retire = [S](HostSlot& hs) {
        std::lock_guard<std::mutex> lk(S->mu);
        hs.res.latency_ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - hs.t_submit).count();
        if (S->cancelled.count(hs.ticket)) {
            hs.res.status = ZMC_ECANCELED;
            S->cancelled.erase(hs.ticket);
        }
        S->done[hs.ticket] = hs.res;
        S->pending.erase(hs.ticket);
        ++S->n_completed;
        --S->resident;
        S->cv_done.notify_all();
    };
    adm.cancelled = [S](uint64_t t) {
        std::lock_guard<std::mutex> lk(S->mu);
        return S->cancelled.count(t) > 0;
    };
    int rc = L->eng.drive(L->st, adm, nullptr, &S->stop, &S->n_levels);
    std::lock_guard<std::mutex> lk(S->mu);
    if (rc != ZMC_OK && S->rc == ZMC_OK) S->rc = rc;
    if (rc != ZMC_OK) {
        // a failed lane stops every lane: their requests end below
        S->stop = true;
        S->cv_q.notify_all();
    }
    if (--S->running > 0) return;
    S->exited = true;
    // every ticket not finished ends now: cancelled on shutdown, or with the
    // error that stopped serving (a device error leaves the resident requests
    // of its lane unretired)
    for (uint64_t t : S->pending) {
        zmc_result R;
        init_result(R);
        R.status = S->rc != ZMC_OK ? S->rc : ZMC_ECANCELED;
        S->done[t] = R;
    }
    S->pending.clear();
    S->queue.clear();
    S->cv_done.notify_all();
}

// A stream of a serving lane.  The runtime maps ordinary streams onto a few
// hardware queues and hands a new stream the least used one, which may be
// the queue of another lane: launches on one queue run one after another.
// A stream with a CU mask always gets a hardware queue of its own; the mask
// enables every compute unit.  (Such a stream synchronises with the null
// stream like any stream created without hipStreamNonBlocking.)
hipError_t create_lane_stream(hipStream_t* st)
{
    int n_cu = 0;
    int dev = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n_cu > 0) {
        std::vector<uint32_t> mask((n_cu + 31) / 32, 0xffffffffu);
        if (n_cu % 32) mask.back() = (1u << (n_cu % 32)) - 1u;
        if (hipExtStreamCreateWithCUMask(st, (uint32_t)mask.size(), mask.data()) == hipSuccess) return hipSuccess;
    }
    return hipStreamCreateWithFlags(st, hipStreamNonBlocking);
}

void stop_server()
{
    Server* S = g.server;
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        S->cv_q.notify_all();
    }
    for (auto& L : S->lanes)
        if (L->th.joinable()) L->th.join();
    for (auto& L : S->lanes) {
        L->eng.teardown();
        if (L->own_stream) (void)hipStreamDestroy(L->st);
    }
    delete S;
    g.server = nullptr;
}

} // namespace

extern "C" {

int zmc_init(const zmc_config* cfg)
{
    std::lock_guard<std::mutex> lk(g_init_mu);
    if (!cfg || !cfg->arena) return fail(ZMC_EINVAL, "zmc_init: NULL config or arena");
    if (cfg->arena_bytes < (64ull << 20)) return fail(ZMC_EINVAL, "zmc_init: arena must be >= 64 MiB");
    if (((uintptr_t)cfg->arena & 255) != 0) return fail(ZMC_EINVAL, "zmc_init: arena must be 256-byte aligned");
    if (cfg->serve_lanes < 0 || cfg->serve_lanes > 8) return fail(ZMC_EINVAL, "zmc_init: serve_lanes must be in 0..8");
    if (cfg->serve_chunk_samples < -1) return fail(ZMC_EINVAL, "zmc_init: serve_chunk_samples must be >= -1");
    if (cfg->default_eval != ZMC_EVAL_FP64 && cfg->default_eval != ZMC_EVAL_FP32)
        return fail(ZMC_EINVAL, "zmc_init: default_eval must be a zmc_eval");
    if (g.inited) {
        stop_server();
        g.sync_eng.teardown();
        g.static_eng.teardown();
        g.inited = false;
    }
    if (hipGetDevice(&g.device) != hipSuccess) return fail(ZMC_EDEVICE, "hipGetDevice failed");
    g.tiles = TileTable();
    g.default_eval = cfg->default_eval;
    if (cfg->tune_path && cfg->tune_path[0]) {
        if (g.tiles.load(cfg->tune_path) != 0) return fail(ZMC_EINVAL, "zmc_init: cannot read tune_path");
    }
    const int slots = cfg->max_slots > 0 ? cfg->max_slots : 8192;
    char* base = (char*)cfg->arena;
    size_t bytes = (size_t)cfg->arena_bytes;
    size_t sync_bytes = bytes;
    if (cfg->serve_stream) sync_bytes = (bytes / 4) & ~(size_t)255;
    int rc = g.sync_eng.setup(base, sync_bytes, slots, &g.tiles, g.device);
    if (rc != ZMC_OK) return rc;
    if (g.device < 0 || g.device >= kMaxDevices) {
        g.sync_eng.teardown();
        return fail(ZMC_EDEVICE, "zmc_init: device id out of range");
    }
    if (!g_scratch_ptr[g.device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            g.sync_eng.teardown();
            return fail(ZMC_EDEVICE, (std::string("zmc_init: hipGetSymbolAddress(scratch): ") +
                                      hipGetErrorString(e)).c_str());
        }
        g_scratch_ptr[g.device] = p;
    }
    rc = g.static_eng.setup((char*)g_scratch_ptr[g.device], kStaticScratchBytes, 1, &g.tiles, g.device);
    if (rc != ZMC_OK) {
        g.sync_eng.teardown();
        return rc;
    }
    if (cfg->serve_stream) {
        const int n_lanes = cfg->serve_lanes > 0 ? cfg->serve_lanes : 2;
        Server* S = new Server();
        S->queue_cap = cfg->queue_depth > 0 ? (size_t)cfg->queue_depth : 65536;
        const size_t lane_bytes = ((bytes - sync_bytes) / n_lanes) & ~(size_t)255;
        for (int i = 0; i < n_lanes && rc == ZMC_OK; ++i) {
            S->lanes.emplace_back(new Lane());
            Lane* L = S->lanes.back().get();
            if (i == 0) {
                L->st = (hipStream_t)cfg->serve_stream;
            } else if (create_lane_stream(&L->st) == hipSuccess) {
                L->own_stream = true;
            } else {
                rc = fail(ZMC_EDEVICE, "zmc_init: cannot create a serving stream");
                break;
            }
            rc = L->eng.setup(base + sync_bytes + i * lane_bytes, lane_bytes, slots, &g.tiles, g.device);
            L->eng.set_chunk_samples(cfg->serve_chunk_samples == 0 ? kServeChunkSamples
                                     : cfg->serve_chunk_samples < 0 ? 0
                                                                    : cfg->serve_chunk_samples);
        }
        if (rc != ZMC_OK) {
            for (auto& L : S->lanes) {
                L->eng.teardown();
                if (L->own_stream) (void)hipStreamDestroy(L->st);
            }
            delete S;
            g.sync_eng.teardown();
            g.static_eng.teardown();
            return rc;
        }
        g.server = S;
        S->running = n_lanes;
        for (auto& L : S->lanes) L->th = std::thread(server_main, S, L.get(), g.device);
    }
    g.inited = true;
    return ZMC_OK;
}

int zmc_shutdown(void)
{
    std::lock_guard<std::mutex> lk(g_init_mu);
    if (!g.inited) return ZMC_OK;
    stop_server();
    {
        std::lock_guard<std::mutex> lk2(g.sync_mu);
        g.sync_eng.teardown();
    }
    {
        std::lock_guard<std::mutex> lk3(g.static_mu);
        g.static_eng.teardown();
    }
    g.inited = false;
    return ZMC_OK;
}

int zmc_integrate_request(const zmc_request* req, void* stream, zmc_result* out, zmc_trace* trace)
{
    if (!req || !out) return fail(ZMC_EINVAL, "NULL request or result");
    init_result(*out);
    int rc = validate(*req);
    if (rc != ZMC_OK) {
        out->status = rc;
        return rc;
    }
    if (!g.inited) return fail(ZMC_ENOINIT, "zmc_init has not been called");
    std::lock_guard<std::mutex> lk(g.sync_mu);
    rc = g.sync_eng.run(req, 1, (hipStream_t)stream, out, trace);
    if (rc == ZMC_OK && out->status != ZMC_OK) rc = out->status;
    return rc;
}

int zmc_request_bytes(const zmc_request* req, uint64_t* bytes)
{
    if (!req || !bytes) return fail(ZMC_EINVAL, "NULL request or output");
    const int rc = validate(*req);
    if (rc != ZMC_OK) return rc;
    *bytes = (uint64_t)request_bytes(*req, g.tiles);
    return ZMC_OK;
}

int zmc_integrate_noalloc(const zmc_request* req, void* stream, zmc_result* out)
{
    if (!req || !out) return fail(ZMC_EINVAL, "NULL request or result");
    init_result(*out);
    int rc = validate(*req);
    if (rc != ZMC_OK) {
        out->status = rc;
        return rc;
    }
    if (req->integrand >= kUserBase) {
        out->status = ZMC_EINVAL;
        return fail(ZMC_EINVAL, "zmc_integrate_noalloc: run-time compiled integrands load code objects (an "
                                "allocation); use zmc_integrate_request");
    }
    if (!g.inited) return fail(ZMC_ENOINIT, "zmc_init has not been called");
    std::lock_guard<std::mutex> lk(g.static_mu);
    const size_t need = g.static_eng.reservation_bytes(*req);
    if (need > g.static_eng.budget_bytes()) {
        out->status = ZMC_ENOMEM;
        char msg[192];
        snprintf(msg, sizeof msg,
                 "zmc_integrate_noalloc: the request's worst-case tree needs %zu bytes; the static scratch "
                 "holds %zu",
                 need, g.static_eng.budget_bytes());
        return fail(ZMC_ENOMEM, msg);
    }
    rc = g.static_eng.run(req, 1, (hipStream_t)stream, out, nullptr);
    if (rc == ZMC_OK && out->status != ZMC_OK) rc = out->status;
    return rc;
}

int zmc_integrate(int integrand_id, const double* params, int dim, const double* lower, const double* upper,
                  int divisions_per_axis, int64_t samples_per_cube, int trials, int max_depth, double sigma_mult,
                  uint64_t seed, void* stream, zmc_result* out)
{
    if (out) init_result(*out);
    // the params layout of the registry (or of the registration) for dim
    const int n_params = integrand_id >= kUserBase ? rtc_n_params(integrand_id) : n_params_of(integrand_id, dim);
    if (n_params < 0) {
        if (out) out->status = ZMC_EINVAL;
        return fail(ZMC_EINVAL, "unknown integrand");
    }
    if ((n_params > 0 && !params) || !lower || !upper) return fail(ZMC_EINVAL, "NULL params or bounds");
    const zmc_request r = make_request(integrand_id, params, n_params, dim, lower, upper, divisions_per_axis,
                                       samples_per_cube, trials, max_depth, sigma_mult, seed, g.default_eval);
    return zmc_integrate_request(&r, stream, out, nullptr);
}

int zmc_integrate_batch(const zmc_request* reqs, int n, void* stream, zmc_result* outs)
{
    if (!reqs || !outs || n < 1) return fail(ZMC_EINVAL, "empty batch");
    for (int i = 0; i < n; ++i) {
        init_result(outs[i]);
        const int rc = validate(reqs[i]);
        if (rc != ZMC_OK) {
            outs[i].status = rc;
            return rc;
        }
    }
    if (!g.inited) return fail(ZMC_ENOINIT, "zmc_init has not been called");
    std::lock_guard<std::mutex> lk(g.sync_mu);
    return g.sync_eng.run(reqs, n, (hipStream_t)stream, outs, nullptr);
}

int zmc_submit(const zmc_request* req, uint64_t* ticket)
{
    if (!req || !ticket) return fail(ZMC_EINVAL, "NULL request or ticket");
    const int rc = validate(*req);
    if (rc != ZMC_OK) return rc;
    if (!g.inited || !g.server) return fail(ZMC_ENOINIT, "serving is not configured");
    Server* S = g.server;
    HostSlot hs;
    hs.req = *req;
    init_result(hs.res);
    hs.reserve = S->lanes[0]->eng.reservation_bytes(*req);
    hs.t_submit = std::chrono::steady_clock::now();
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->exited) return fail(S->rc != ZMC_OK ? S->rc : ZMC_ENOINIT, "the serving thread has stopped");
    if (S->queue.size() >= S->queue_cap) return fail(ZMC_EBUSY, "request queue is full");
    hs.ticket = S->next_ticket++;
    S->pending.insert(hs.ticket);
    S->queue.push_back(hs);
    *ticket = hs.ticket;
    S->cv_q.notify_all();
    return ZMC_OK;
}

int zmc_poll(uint64_t ticket, zmc_result* out, int wait)
{
    if (!out) return fail(ZMC_EINVAL, "NULL result");
    if (!g.inited || !g.server) return fail(ZMC_ENOINIT, "serving is not configured");
    Server* S = g.server;
    std::unique_lock<std::mutex> lk(S->mu);
    while (true) {
        auto it = S->done.find(ticket);
        if (it != S->done.end()) {
            *out = it->second;
            S->done.erase(it);
            return ZMC_OK;
        }
        if (!S->pending.count(ticket)) return fail(ZMC_ENOTFOUND, "unknown ticket");
        if (!wait) return ZMC_EAGAIN;
        S->cv_done.wait_for(lk, std::chrono::milliseconds(50));
    }
}

int zmc_cancel(uint64_t ticket)
{
    if (!g.inited || !g.server) return fail(ZMC_ENOINIT, "serving is not configured");
    Server* S = g.server;
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->done.count(ticket)) return ZMC_OK; // finished already: its result stands
    if (!S->pending.count(ticket)) return fail(ZMC_ENOTFOUND, "unknown ticket");
    for (auto it = S->queue.begin(); it != S->queue.end(); ++it) {
        if (it->ticket == ticket) {
            zmc_result R;
            init_result(R);
            R.status = ZMC_ECANCELED;
            S->done[ticket] = R;
            S->pending.erase(ticket);
            S->queue.erase(it);
            S->cv_done.notify_all();
            return ZMC_OK;
        }
    }
    S->cancelled.insert(ticket);
    return ZMC_OK;
}

int zmc_serve_stats(uint64_t out4[4])
{
    if (!out4) return fail(ZMC_EINVAL, "NULL output");
    if (!g.inited || !g.server) return fail(ZMC_ENOINIT, "serving is not configured");
    Server* S = g.server;
    std::lock_guard<std::mutex> lk(S->mu);
    out4[0] = S->queue.size();
    out4[1] = (uint64_t)S->resident;
    out4[2] = S->n_completed;
    out4[3] = S->n_levels.load(std::memory_order_relaxed);
    return ZMC_OK;
}

int zmc_debug_philox(uint32_t key_lo, uint32_t key_hi, const uint32_t* ctr, int64_t n, uint32_t* out, void* stream)
{
    if (!ctr || !out || n < 0) return fail(ZMC_EINVAL, "bad debug_philox arguments");
    if (!g.inited) return fail(ZMC_ENOINIT, "zmc_init has not been called");
    if (n == 0) return ZMC_OK;
    std::lock_guard<std::mutex> lk(g.sync_mu);
    return g.sync_eng.debug_philox(key_lo, key_hi, ctr, n, out, (hipStream_t)stream);
}

int zmc_debug_points(const zmc_request* req, int level, uint64_t uid, int trial, int64_t s0, int64_t n, double* x,
                     void* stream)
{
    if (!req || !x || n < 0 || s0 < 0 || level < 0 || level >= ZMC_MAX_LEVELS || trial < 0)
        return fail(ZMC_EINVAL, "bad debug_points arguments");
    int rc = validate(*req);
    if (rc != ZMC_OK) return rc;
    if (trial >= req->trials || s0 + n > req->samples_per_cube) return fail(ZMC_EINVAL, "sample out of range");
    if (!g.inited) return fail(ZMC_ENOINIT, "zmc_init has not been called");
    if (n == 0) return ZMC_OK;
    std::lock_guard<std::mutex> lk(g.sync_mu);
    return g.sync_eng.debug_points(*req, level, uid, trial, s0, n, x, (hipStream_t)stream);
}

int zmc_cube_estimates(const zmc_request* req, int level, const uint64_t* uids, int64_t n, double* m, double* s,
                       double* S1, double* S2, void* stream)
{
    if (!req || (n > 0 && !uids) || n < 0 || level < 0 || level >= ZMC_MAX_LEVELS)
        return fail(ZMC_EINVAL, "bad cube_estimates arguments");
    int rc = validate(*req);
    if (rc != ZMC_OK) return rc;
    if (!g.inited) return fail(ZMC_ENOINIT, "zmc_init has not been called");
    if (n == 0) return ZMC_OK;
    std::lock_guard<std::mutex> lk(g.sync_mu);
    return g.sync_eng.cube_estimates(*req, level, uids, n, m, s, S1, S2, (hipStream_t)stream);
}

const char* zmc_strerror(int status)
{
    switch (status) {
    case ZMC_OK: return "ok";
    case ZMC_EINVAL: return last_error()[0] ? last_error() : "invalid argument";
    case ZMC_ENOMEM: return last_error()[0] ? last_error() : "arena exhausted";
    case ZMC_ENONFINITE: return "integrand produced a non-finite value";
    case ZMC_EDEVICE: return last_error()[0] ? last_error() : "HIP error";
    case ZMC_EAGAIN: return "not finished";
    case ZMC_EBUSY: return "queue full";
    case ZMC_ENOINIT: return "not initialised";
    case ZMC_ECANCELED: return "cancelled";
    case ZMC_ENOTFOUND: return "unknown ticket";
    default: return "unknown status";
    }
}

const char* zmc_version(void) { return "zmc-mi355x 0.1 (gfx950)"; }

int zmc_register_integrand(const char* body, int n_params, int* integrand_id)
{
    return rtc_register(body, n_params, integrand_id);
}

int zmc_struct_size(int which)
{
    switch (which) {
    case 0: return (int)sizeof(zmc_result);
    case 1: return (int)sizeof(zmc_request);
    case 2: return (int)sizeof(zmc_config);
    case 3: return (int)sizeof(zmc_trace);
    default: return -1;
    }
}

} // extern "C"
