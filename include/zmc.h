/*
 * zmc.h -- C ABI of the MI355X (gfx950) stratified-sampling + heuristic
 * tree-search Monte Carlo integrator.
 *
 * Method: "ZMCintegral: a Package for Multi-Dimensional Monte Carlo
 * Integration on Multi-GPUs" (Wu, Zhang, Pang, Wang; arXiv:1902.07916),
 * Sec. 2.1 (stratified sampling and heuristic tree search), Sec. 2.2
 * (random numbers produced at the time of use), Sec. 2.3 (user parameters).
 *
 *  1. The domain [lower, upper] is divided into k = d^D equal hypercubes
 *     (root cubes, level 0), numbered in row-major order, axis 0 most
 *     significant.
 *  2. In every cube, `trials` (the paper's n1) independent direct Monte Carlo
 *     estimates I_t = V * mean_s f(x_s) are formed, each from
 *     `samples_per_cube` points.  Point s, dimension i of trial t in the cube
 *     (uid, level) uses word n = s*D + i of the Philox4x32-10 stream with key
 *     = seed and counter (n >> 2, t | level << 8 | uid_hi << 12, lo32(uid),
 *     hi32(uid)), lane n & 3, where a cube id has up to 84 bits, uid holding
 *     bits 0..63 and uid_hi bits 64..83; the word w maps to
 *     u = (2*(w >> 9) + 1) * 2^-24 and x_i = fma(h_i, u, lo_i).
 *  3. Per cube: m = mean of the I_t, s = population std of the I_t.  Every
 *     population std scales the deviations by 2^-e before squaring and the
 *     root by 2^e after (e the binary exponent of the largest deviation):
 *     the same number where the plain squares neither underflow nor
 *     overflow, and no deviation lost where they would.
 *  4. Per level and per integral: thr = mean(s) + sigma_mult * std(s)
 *     (population std); a cube with s > thr is split (unless the level is
 *     max_depth), all other cubes are accepted with their m.  With
 *     threshold_scope = 1, below the roots each split parent's children get
 *     their own threshold from their own s.
 *  5. A split cube is replaced by its 2^D children (every axis bisected);
 *     child c of uid has uid' = (uid << D) | c, bit (D-1-i) of c choosing the
 *     upper half of axis i.  With split = b every axis is cut into b parts:
 *     uid' = uid * b^D + c, digit (D-1-i) of c in base b giving axis i.  The
 *     same estimate is run on the new list.
 *  6. Result: integral = sum of accepted m; std = sqrt(sum of accepted s^2);
 *     stderr = sqrt(sum s^2 / (n1 - 1)).
 *
 * Conventions for every function:
 *  - return value: ZMC_OK (0) or a negative zmc_status; no exception or
 *    signal crosses the ABI; zmc_strerror() describes the last error of the
 *    calling thread;
 *  - host pointers are read (and copied where kept) during the call; the
 *    caller keeps ownership of everything it passes in;
 *  - device memory is used only from the arena handed to zmc_init(); the
 *    library never allocates or frees device memory itself (it allocates
 *    pinned host staging buffers);
 *  - `stream` is a hipStream_t owned by the caller (NULL = the default
 *    stream); the library enqueues on it and, for synchronous calls,
 *    synchronises it before returning.
 */
#ifndef ZMC_H
#define ZMC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ZMC_MAX_DIM 16
#define ZMC_MAX_LEVELS 16
#define ZMC_MAX_PARAMS (2 * ZMC_MAX_DIM + 2)

typedef enum {
    ZMC_OK = 0,
    ZMC_EINVAL = -1,      /* an argument is out of range (list below)          */
    ZMC_ENOMEM = -2,      /* the arena cannot hold a level of the tree         */
    ZMC_ENONFINITE = -3,  /* the integrand produced a NaN or an infinity       */
    ZMC_EDEVICE = -4,     /* a HIP call failed; zmc_strerror() has its text    */
    ZMC_EAGAIN = -5,      /* zmc_poll: the request is not finished yet         */
    ZMC_EBUSY = -6,       /* zmc_submit: the request queue is full             */
    ZMC_ENOINIT = -7,     /* zmc_init() has not been called                    */
    ZMC_ECANCELED = -8,   /* the request was cancelled                         */
    ZMC_ENOTFOUND = -9    /* unknown ticket                                    */
} zmc_status;

/* Integrand registry.  params layout (FP64; length n_params must match):
 *  ZMC_GAUSS       [sigma, A, mu_1..mu_D]  A exp(-sum (x_i-mu_i)^2 / (2 sigma^2))
 *                  (the paper's f2, Sec. 3, is sigma = 0.01,
 *                   A = (sqrt(2 pi) sigma)^-9, mu = 0)
 *  ZMC_SIN_SUM     []                      sin(sum x_i)   (the paper's f1, Sec. 3)
 *  ZMC_GENZ_OSC    [u, c_1..c_D]           cos(2 pi u + sum c_i x_i)
 *  ZMC_GENZ_PPEAK  [c_1..c_D, w_1..w_D]    prod 1 / (c_i^-2 + (x_i - w_i)^2)
 *  ZMC_GENZ_CPEAK  [c_1..c_D]              (1 + sum c_i x_i)^-(D+1)
 *  ZMC_GENZ_GAUSS  [c_1..c_D, w_1..w_D]    exp(-sum c_i^2 (x_i - w_i)^2)
 *  ZMC_CONST       [A]                     A
 *  ZMC_MONOMIAL    [p_1..p_D]              prod x_i^p_i, integers 0 <= p_i <= 16 */
typedef enum {
    ZMC_GAUSS = 0,
    ZMC_SIN_SUM = 1,
    ZMC_GENZ_OSC = 2,
    ZMC_GENZ_PPEAK = 3,
    ZMC_GENZ_CPEAK = 4,
    ZMC_GENZ_GAUSS = 5,
    ZMC_CONST = 6,
    ZMC_MONOMIAL = 7
} zmc_integrand;

/* Arithmetic of the integrand evaluation.  Sums over samples, the per-cube
 * mean/std, the threshold and every total are FP64 in both modes.
 *  ZMC_EVAL_FP64: x and f in FP64; x is bitwise the value of step 2 above.
 *  ZMC_EVAL_FP32: x and f in FP32 using cube-relative coordinates (offsets
 *                 and phases formed in FP64 per cube) and the hardware
 *                 transcendental units; the FP32 value is f divided by a
 *                 per-cube FP64 scale (the amplitude and, for the Gaussian
 *                 families, the value at the cube's point nearest the peak;
 *                 the product of c_i^2 for the product peak; the value at the
 *                 lower corner for the corner peak; the largest |x_i|^p_i for
 *                 the monomial), applied to each FP64 sum. */
typedef enum { ZMC_EVAL_FP64 = 0, ZMC_EVAL_FP32 = 1 } zmc_eval;

/* result.flags */
#define ZMC_F_TRUNCATED 1 /* a level would have exceeded max_cubes_per_level:
                             the cubes selected there were accepted instead */
#define ZMC_F_RTOL_MET 2  /* the search stopped because stderr <= rtol*|I|  */
#define ZMC_F_FP32_RANGE 4 /* ZMC_EVAL_FP32: in some cube the FP32 values lay
                              below FP32's normal range (a sampling unit's
                              values summed to less than its points times
                              2^-126 in magnitude, after the per-cube scaling
                              described at zmc_eval), so the tree and the
                              result may differ from FP64 evaluation beyond
                              rounding: evaluate this integrand in FP64 */

/* Result of one integration.  integral, std and stderr_ are NaN unless
 * status is ZMC_OK; the per-level fields cover the levels that ran. */
typedef struct {
    double integral;   /* sum of accepted per-cube means                     */
    double std;        /* sqrt(sum of accepted s^2)                          */
    double stderr_;    /* sqrt(sum of accepted s^2 / (trials - 1))           */
    uint64_t n_samples;/* every evaluated point: sum_levels cubes*trials*N   */
    uint64_t n_cubes;  /* cubes evaluated over all levels                    */
    int32_t levels_run;
    int32_t flags;     /* ZMC_F_*                                            */
    int32_t status;    /* ZMC_OK or the request's zmc_status                 */
    int32_t reserved;
    uint64_t cubes_per_level[ZMC_MAX_LEVELS];
    uint64_t selected_per_level[ZMC_MAX_LEVELS];
    double thr_per_level[ZMC_MAX_LEVELS];        /* NaN where none was formed  */
    double min_margin_per_level[ZMC_MAX_LEVELS]; /* min |s - thr| / thr        */
    float ms_per_level[ZMC_MAX_LEVELS];          /* wall time of each level    */
    float sample_ms_per_level[ZMC_MAX_LEVELS];   /* GPU time of the level's
                                                    sampling launches (HIP
                                                    events on the stream)      */
    int32_t sample_launches_per_level[ZMC_MAX_LEVELS];
    double latency_ms; /* serving: submit -> completion; otherwise call time */
} zmc_result;

/* One integration request: the arguments of zmc_integrate() as a struct, for
 * zmc_integrate_batch() and zmc_submit(). */
typedef struct {
    int32_t integrand;           /* zmc_integrand                                */
    int32_t dim;                 /* D, 1..16                                     */
    int32_t divisions_per_axis;  /* d >= 1: k = d^D root cubes                   */
    int32_t trials;              /* n1, 2..255                                   */
    int32_t max_depth;           /* refinement rounds after level 0, 0..15       */
    int32_t eval;                /* zmc_eval                                     */
    int32_t n_params;
    int32_t split;               /* 0 or 2: a split bisects every axis (2^D
                                    children); b in 3..64: b parts per axis (b^D
                                    children, at most 2^24; b = d is the paper's
                                    split into k equal parts, Sec. 2.1)         */
    int32_t threshold_scope;     /* 0: one threshold per level over all its cubes;
                                    1: one per parent, over its children (the
                                    roots share one)                             */
    int32_t reserved;
    int64_t samples_per_cube;    /* N >= 1 points per trial, N * D <= 2^34       */
    int64_t max_cubes_per_level; /* 0 = default (2^24)                           */
    double sigma_mult;           /* >= 0                                         */
    double rtol;                 /* 0 = off; else stop once stderr <= rtol*|I|   */
    uint64_t seed;               /* Philox key                                   */
    double lower[ZMC_MAX_DIM];
    double upper[ZMC_MAX_DIM];
    double params[ZMC_MAX_PARAMS];
} zmc_request;

/* Library configuration. */
typedef struct {
    void* arena;            /* device memory, >= 64 MiB, 256-byte aligned;
                               owned by the caller and never freed here       */
    uint64_t arena_bytes;
    int32_t max_slots;      /* integrals resident at once (batch / serving);
                               0 = default 8192                               */
    int32_t queue_depth;    /* zmc_submit queue capacity; 0 = default 65536   */
    void* serve_stream;     /* hipStream_t of the first serving lane; NULL =
                               serving disabled.  With serving, 1/4 of the
                               arena serves the synchronous calls and 3/4 is
                               split evenly among the lanes                  */
    const char* tune_path;  /* JSON tile table written by the autotuner; NULL
                               or "" = built-in defaults                      */
    int32_t serve_lanes;    /* serving lanes (engine + thread + stream each;
                               lane 0 uses serve_stream, the others streams
                               the library creates, each on a hardware queue
                               of its own); 0 = default 2, max 8              */
    int32_t default_eval;   /* zmc_eval of zmc_integrate() (the requests of
                               the other entry points carry their own);
                               0 = ZMC_EVAL_FP64                              */
    int64_t serve_chunk_samples; /* serving splits a level's sampling into
                               launches of about this many samples, so that
                               lanes share the device between launches;
                               0 = default 2^31, -1 = one launch per level    */
} zmc_config;

/* Per-level trace of a synchronous integration (test and debugging hook).
 * For every level l < max_levels the library copies up to `capacity`
 * entries, in list order, into the caller's host buffers (any may be NULL):
 * uid[l][c] (cube id bits 0..63), m[l][c], s[l][c], sel[l][c] (1 = split)
 * and, per trial, S1[l][c*trials + t] = sum f and S2[l][c*trials + t] =
 * sum f^2; uid_hi[l][c] receives id bits 64..83 (0 below 2^64).
 * n[l] receives the number of cubes at level l (even if > capacity). */
typedef struct {
    int32_t max_levels;
    int32_t reserved;
    int64_t capacity;
    int64_t n[ZMC_MAX_LEVELS];
    uint64_t* uid[ZMC_MAX_LEVELS];
    double* m[ZMC_MAX_LEVELS];
    double* s[ZMC_MAX_LEVELS];
    uint8_t* sel[ZMC_MAX_LEVELS];
    double* S1[ZMC_MAX_LEVELS];
    double* S2[ZMC_MAX_LEVELS];
    uint32_t* uid_hi[ZMC_MAX_LEVELS];
} zmc_trace;

/* Initialise the library on the current HIP device with the caller's arena.
 * EINVAL: NULL cfg/arena, arena_bytes < 64 MiB, misaligned arena,
 * serve_lanes outside 0..8, serve_chunk_samples < -1, default_eval not a
 * zmc_eval.
 * Calling it again after zmc_shutdown() is allowed. */
int zmc_init(const zmc_config* cfg);

/* Stop the serving thread (pending tickets end with ZMC_ECANCELED), release
 * host staging memory.  The arena is not touched. */
int zmc_shutdown(void);

/* Integrate one function (Sec. 2.1 steps 1-6 above), synchronously, with
 * the user parameters of Sec. 2.3: the k = d^D root sub-domains
 * (divisions_per_axis), the points per trial (samples_per_cube), the trials,
 * the maximal partition depth (max_depth refinements after the roots) and the
 * threshold multiplier (sigma_mult).
 * params: FP64 values, as many as the integrand's layout above takes for dim
 * (a run-time compiled integrand: the n_params it was registered with);
 * lower/upper: dim FP64 values each; the evaluation mode is the
 * configuration's default_eval; splits bisect every axis, one threshold per
 * level, level cap 2^24 cubes (zmc_integrate_request() sets all of these).
 * out: caller memory, valid when ZMC_OK is returned (and filled with status
 * on ZMC_ENONFINITE / ZMC_ENOMEM).
 * EINVAL when: params NULL where the layout takes values, lower/upper NULL;
 * dim not in 1..16; lower_i >= upper_i or not finite; d < 1;
 * N < 1 or N*D > 2^34; trials not in 2..255; max_depth not in 0..15;
 * sigma_mult < 0 or not finite; unknown integrand; a MONOMIAL exponent
 * outside 0..16 or not an integer; d^D * (b^D)^max_depth > 2^84 (cube ids
 * hold 84 bits; b = 2 unless the request sets split) or d * b^max_depth >
 * 2^64 (lattice cells per axis); d^D > max_cubes_per_level; split or
 * threshold_scope out of range.
 * ENOMEM when a level does not fit the arena. */
int zmc_integrate(int integrand_id, const double* params, int dim, const double* lower, const double* upper,
                  int divisions_per_axis, int64_t samples_per_cube, int trials, int max_depth, double sigma_mult,
                  uint64_t seed, void* stream, zmc_result* out);

/* zmc_integrate() with every field of zmc_request (rtol, level cap) and an
 * optional trace (NULL = none). */
int zmc_integrate_request(const zmc_request* req, void* stream, zmc_result* out, zmc_trace* trace);

/* zmc_integrate_request() without a trace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation): the call allocates nothing.  Its level arrays live
 * in a static device array of the library (64 MiB per device, held from the
 * first zmc_init() on that device until the process ends) instead of the
 * arena; its pinned staging was allocated by zmc_init().  Results are bitwise
 * those of zmc_integrate_request() (the same kernels).  Calls share that one
 * array and keep no state in it between calls (the level counters it holds
 * are left at zero by every launch); the library serialises them, and each
 * call synchronises its stream before returning, so calls do not overlap on
 * the device: a caller that replays such a call asynchronously (e.g. from a
 * captured graph) must not let two of them run at once.
 * ENOMEM (before any device work, with the sizes in zmc_strerror) when the
 * request's worst-case tree (zmc_request_bytes) exceeds the static array;
 * EINVAL for a run-time compiled integrand (loading its code allocates) and
 * as for zmc_integrate_request(); ENOINIT before zmc_init(). */
int zmc_integrate_noalloc(const zmc_request* req, void* stream, zmc_result* out);

/* Integrate n independent requests together (each with its own threshold per
 * level): all their cubes are evaluated by the same launches, level by level.
 * outs[i] receives request i's result; each result is bitwise the one
 * zmc_integrate_request() returns for that request alone.  Returns ZMC_OK if
 * the batch ran (per-request failures are in outs[i].status), EINVAL if n <
 * 1, n > max_slots or any request is invalid, ENOMEM if the arena cannot
 * hold the batch's first level.  A request whose worst-case tree (the level
 * bound the serving admission uses) exceeds the whole arena is not run and
 * gets status ENOMEM on its own; if the requests that do run exhaust the
 * arena together, those still resident at that level get ENOMEM. */
int zmc_integrate_batch(const zmc_request* reqs, int n, void* stream, zmc_result* outs);

/* Worst-case device bytes of req's tree: the largest level's list, work
 * arrays and next list, with every level's selections bounded by Cantelli's
 * inequality (at most n / (1 + sigma_mult^2) of n cubes exceed mean +
 * sigma_mult * std; n - 1 when sigma_mult = 0) and by max_cubes_per_level.
 * It is the reservation serving admission makes and the size a batch member
 * may not exceed alone.  Needs no zmc_init() (uses the built-in tile table
 * before it).  EINVAL as for zmc_integrate_request(). */
int zmc_request_bytes(const zmc_request* req, uint64_t* bytes);

/* Serving (continuous batching at level granularity): enqueue a copy of req
 * and return a ticket.  Each serving lane admits queued requests at its level
 * boundaries whenever its slots and arena share allow (a busy lane whose next
 * level is large leaves new requests to a lighter lane), runs every resident
 * request's current level in shared launches, and retires finished requests.
 * A request whose worst-case tree exceeds one lane's arena share ends with
 * status ENOMEM.  Lanes run concurrently; calls may come from any thread.
 * EINVAL: invalid request; EBUSY: queue full; ENOINIT: no serve_stream was
 * configured. */
int zmc_submit(const zmc_request* req, uint64_t* ticket);

/* Result of a ticket.  wait = 0: returns EAGAIN while it runs; wait != 0:
 * blocks until done.  On completion the result (with its own status) is
 * copied to out, the ticket is released and ZMC_OK is returned; ENOTFOUND
 * for an unknown or already-collected ticket. */
int zmc_poll(uint64_t ticket, zmc_result* out, int wait);

/* Cancel a queued or running request; its poll then returns a result with
 * status ECANCELED.  A request that has already finished keeps its result
 * (ZMC_OK, no effect).  ENOTFOUND for unknown or already-collected tickets. */
int zmc_cancel(uint64_t ticket);

/* Serving counters: queued, resident, completed, levels stepped. */
int zmc_serve_stats(uint64_t out4[4]);

/* Evaluate Philox4x32-10 on the device for n counters (key = (key_lo,
 * key_hi) for all): ctr is n*4 u32 (host), out n*4 u32 (host).  The same
 * device function the sampling kernels use. */
int zmc_debug_philox(uint32_t key_lo, uint32_t key_hi, const uint32_t* ctr, int64_t n, uint32_t* out,
                     void* stream);

/* Device sample points: for cube (uid, level) of req, trial t, samples
 * s0 .. s0+n-1, write x (n*D FP64, host) exactly as the FP64 path forms them. */
int zmc_debug_points(const zmc_request* req, int level, uint64_t uid, int trial, int64_t s0, int64_t n,
                     double* x, void* stream);

/* Per-cube estimates for an explicit list of cubes (all at `level`) of one
 * request: the sampling and per-cube reduction kernels of zmc_integrate run
 * on uids[0..n) (host array) and write m[n], s[n] and, if non-NULL,
 * S1[n*trials], S2[n*trials] (host arrays). */
int zmc_cube_estimates(const zmc_request* req, int level, const uint64_t* uids, int64_t n, double* m,
                       double* s, double* S1, double* S2, void* stream);

/* User-defined integrand (the paper's package integrates general user
 * functions, abstract and Sec. 3.3): `body` is the body of
 *     template <typename real> real f(const real* x, const double* p)
 * in C++ device syntax, where x[0..D-1] is the point (`real` is double in
 * ZMC_EVAL_FP64 and float in ZMC_EVAL_FP32, with absolute coordinates), p
 * holds the request's n_params params and `D` is a compile-time constant,
 * e.g. "real t = 0; for (int i = 0; i < D; ++i) t += x[i]; return sin(t);".
 * The body is compiled with hipRTC for gfx950 now (to report errors) and once
 * per (D, eval) on first use; the returned id (>= 100) is then used as
 * integrand_id / zmc_request.integrand with n_params params.  Does not need
 * zmc_init().  EINVAL: NULL arguments, n_params outside 0..34, a body that
 * does not compile (zmc_strerror(ZMC_EINVAL) holds the compiler log), or more
 * than 64 registrations. */
int zmc_register_integrand(const char* body, int n_params, int* integrand_id);

/* Text for a status code, or the last HIP error text for ZMC_EDEVICE. */
const char* zmc_strerror(int status);

/* Version string of the library build. */
const char* zmc_version(void);

/* sizeof of the ABI structs, for bindings that mirror them: which = 0
 * zmc_result, 1 zmc_request, 2 zmc_config, 3 zmc_trace; -1 otherwise. */
int zmc_struct_size(int which);

#ifdef __cplusplus
}
#endif

#endif /* ZMC_H */
