// zmc_rtc.hip -- user-defined integrands compiled at run time with hipRTC.
//
// The paper's package integrates general user-defined functions written in
// Python/Numba (abstract, Sec. 3.3).  Here the user supplies the body of a
// device function in C++ syntax,
//
//     template <typename real> real f(const real* x, const double* p)
//     { constexpr int D = <dim>;  <body> }
//
// using x[0..D-1] (the point, `real` is double or float), p[0..n_params-1]
// (the request's params) and D.  The body is compiled once per (D, eval) on
// first use, around the same sampling body as the precompiled registry
// (zmc_sample_core.hpp); the device headers are embedded in the library at
// build time, so nothing is read from disk at run time.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "zmc_engine.hpp"
#include "zmc_rtc.hpp"
#include "zmc_rtc_embed.inc" // kRtcHeaderNames / kRtcHeaderSources / kRtcHeaderCount

namespace zmc {

namespace {

struct UserDef {
    std::string body;
    int n_params;
};

struct Compiled {
    hipModule_t module = nullptr;
    hipFunction_t fn = nullptr;
    int capacity = 0;
};

std::mutex g_mu;
std::vector<UserDef> g_defs;
std::map<std::tuple<int, int, int>, Compiled> g_cache;

const char* kPrelude = R"ZMCRTC(
typedef __hip_internal::uint64_t uint64_t;
typedef __hip_internal::int64_t int64_t;
typedef __hip_internal::uint32_t uint32_t;
typedef __hip_internal::int32_t int32_t;
typedef __hip_internal::uint8_t uint8_t;
)ZMCRTC";

std::string program_source(const std::string& body, int dim, bool fp32)
{
    std::string s = kPrelude;
    s += "#define ZMC_D " + std::to_string(dim) + "\n";
    s += "#define ZMC_FP32 " + std::string(fp32 ? "true" : "false") + "\n";
    s += R"ZMCRTC(
#include "zmc_sample_core.hpp"
namespace zmc_user {
template <typename real>
__device__ __forceinline__ real f(const real* x, const double* p)
{
    constexpr int D = ZMC_D;
    (void)D;
    (void)p;
#line 1 "user integrand"
)ZMCRTC";
    s += body;
    s += R"ZMCRTC(
}
} // namespace zmc_user
namespace zmc {
// Adapter to the sampling body: FP64 from the absolute point; FP32 from the
// cell values v in [1, 2), x_i = (lo_i - h_i (1 - 2^-24)) + h_i v_i.
template <int D>
struct UserIntegrand {
    static constexpr bool kRangeCheck = true;
    struct P64 {
        const double* prm;
    };
    struct P32 {
        float b[D], m[D];
        const double* prm;
        double scale;
    };
    __device__ static void prep64(const SlotDesc& sd, P64& p) { p.prm = sd.params; }
    __device__ static double f64(const P64& p, const double* x) { return zmc_user::f<double>(x, p.prm); }
    __device__ static void prep32(const SlotDesc& sd, const double* lo, const double* h, P32& p)
    {
        for (int i = 0; i < D; ++i) {
            p.b[i] = (float)(lo[i] - h[i] * (1.0 - 0x1p-24));
            p.m[i] = (float)h[i];
        }
        p.prm = sd.params;
        p.scale = 1.0;
    }
    __device__ static float f32(const P32& p, const float* v)
    {
        float x[D];
#pragma unroll
        for (int i = 0; i < D; ++i) x[i] = __builtin_fmaf(p.m[i], v[i], p.b[i]);
        return zmc_user::f<float>(x, p.prm);
    }
};
} // namespace zmc
extern "C" __global__ __launch_bounds__(256) void zmc_user_kernel(const zmc::SampleArgs a)
{
    zmc::sample_units<zmc::UserIntegrand<ZMC_D>, ZMC_D, ZMC_FP32, true>(a);
}
)ZMCRTC";
    return s;
}

// Compile one variant to a code object; returns 0 and fills `code`, or -1
// with the compiler log in `log`.
int compile(const std::string& body, int dim, bool fp32, std::vector<char>& code, std::string& log)
{
    const std::string src = program_source(body, dim, fp32);
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, src.c_str(), "zmc_user.hip", kRtcHeaderCount, kRtcHeaderSources,
                            kRtcHeaderNames) != HIPRTC_SUCCESS) {
        log = "hiprtcCreateProgram failed";
        return -1;
    }
    // no packed FP32 instructions (v_pk_*_f32), as in the precompiled kernels
    const char* opts[] = {"--gpu-architecture=gfx950", "-O3", "-std=c++17",
                          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
    const hiprtcResult rc = hiprtcCompileProgram(prog, 7, opts);
    size_t ls = 0;
    hiprtcGetProgramLogSize(prog, &ls);
    if (ls > 1) {
        std::vector<char> b(ls + 1, 0);
        hiprtcGetProgramLog(prog, b.data());
        log = b.data();
    }
    if (rc != HIPRTC_SUCCESS) {
        hiprtcDestroyProgram(&prog);
        if (log.empty()) log = hiprtcGetErrorString(rc);
        return -1;
    }
    size_t cs = 0;
    hiprtcGetCodeSize(prog, &cs);
    code.resize(cs);
    hiprtcGetCode(prog, code.data());
    hiprtcDestroyProgram(&prog);
    return 0;
}

} // namespace

int rtc_register(const char* body, int n_params, int* id)
{
    if (!body || !id || n_params < 0 || n_params > ZMC_MAX_PARAMS) {
        set_error("register_integrand: bad arguments");
        return ZMC_EINVAL;
    }
    // compile once (D = 4, FP64) so that syntax errors surface now
    std::vector<char> code;
    std::string log;
    if (compile(body, 4, false, code, log) != 0) {
        set_error("user integrand does not compile:\n" + log);
        return ZMC_EINVAL;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    if ((int)g_defs.size() >= kMaxUserIntegrands) {
        set_error("too many user integrands");
        return ZMC_EINVAL;
    }
    g_defs.push_back(UserDef{body, n_params});
    *id = kUserBase + (int)g_defs.size() - 1;
    return ZMC_OK;
}

int rtc_n_params(int id)
{
    std::lock_guard<std::mutex> lk(g_mu);
    const int k = id - kUserBase;
    if (k < 0 || k >= (int)g_defs.size()) return -1;
    return g_defs[k].n_params;
}

// The kernel for (id, D, eval) on the current device, compiled on first use.
// The compiler runs outside the lock, so launches of kernels already built
// never wait behind a compilation.
static int rtc_get(int id, int dim, int eval, Compiled& out)
{
    const auto key = std::make_tuple(id, dim, eval);
    std::string body;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_cache.find(key);
        if (it != g_cache.end()) {
            out = it->second;
            return ZMC_OK;
        }
        const int k = id - kUserBase;
        if (k < 0 || k >= (int)g_defs.size()) {
            set_error("unknown user integrand");
            return ZMC_EINVAL;
        }
        body = g_defs[k].body;
    }
    std::vector<char> code;
    std::string log;
    if (compile(body, dim, eval == ZMC_EVAL_FP32, code, log) != 0) {
        set_error("user integrand does not compile:\n" + log);
        return ZMC_EINVAL;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_cache.find(key);
    if (it != g_cache.end()) { // built meanwhile by another thread
        out = it->second;
        return ZMC_OK;
    }
    Compiled c;
    hipError_t e = hipModuleLoadData(&c.module, code.data());
    if (e == hipSuccess) e = hipModuleGetFunction(&c.fn, c.module, "zmc_user_kernel");
    if (e != hipSuccess) {
        set_error(std::string("loading the user kernel: ") + hipGetErrorString(e));
        return ZMC_EDEVICE;
    }
    int nb = 0, dev = 0, ncu = 0;
    if (hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&nb, c.fn, kSampleThreads, 0) != hipSuccess || nb < 1)
        nb = 1;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    c.capacity = nb * (ncu > 0 ? ncu : 1);
    g_cache[key] = c;
    out = c;
    return ZMC_OK;
}

int rtc_launch(int id, int dim, int eval, hipStream_t st, const SampleArgs& a)
{
    Compiled c;
    const int rc = rtc_get(id, dim, eval, c);
    if (rc != ZMC_OK) return rc;
    const unsigned grid = (unsigned)std::min<int64_t>(a.total_units, c.capacity);
    SampleArgs arg = a;
    void* params[] = {&arg};
    const hipError_t e = hipModuleLaunchKernel(c.fn, grid, 1, 1, kSampleThreads, 1, 1, 0, st, params, nullptr);
    if (e != hipSuccess) {
        set_error(std::string("launching the user kernel: ") + hipGetErrorString(e));
        return ZMC_EDEVICE;
    }
    return ZMC_OK;
}

} // namespace zmc
