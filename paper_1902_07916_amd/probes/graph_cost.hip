// graph_cost.hip -- what a captured HIP graph per tree level would cost.
// One "level" here has the shape of a small level of the integrator: one
// 4 KiB host-to-device copy from pinned memory and six short kernels on one
// stream, then a synchronisation.  Timed per level (host wall clock, mean of
// 2000 levels after 200 warm-up levels):
//   eager        the seven operations launched directly;
//   capture      captured, instantiated, launched and destroyed every level
//                (a level's topology and addresses change from level to level);
//   update       captured every level and applied to one executable graph with
//                hipGraphExecUpdate instead of a new instantiation;
//   replay       one graph captured once and replayed (a fixed topology: the
//                lower bound, not available to the integrator).
// Build:
//   hipcc -O2 --offload-arch=gfx950 -Xclang -target-feature -Xclang -packed-fp32-ops \
//         paper_1902_07916_amd/probes/graph_cost.hip -o graph_cost
#include <hip/hip_runtime.h>
#include <chrono>
#include <cstdio>

__global__ void tiny(int* p, int v)
{
    p[blockIdx.x * blockDim.x + threadIdx.x] = v;
}

#define CK(x)                                                                                                   \
    do {                                                                                                        \
        hipError_t e_ = (x);                                                                                    \
        if (e_ != hipSuccess) {                                                                                 \
            printf("%s: %s\n", #x, hipGetErrorString(e_));                                                      \
            return 1;                                                                                           \
        }                                                                                                       \
    } while (0)

constexpr int kBlocks = 4, kThreads = 256, kKernels = 6, kCopy = 4096;

static int enqueue(hipStream_t st, int* d, const void* h, void* dtab, int it)
{
    CK(hipMemcpyAsync(dtab, h, kCopy, hipMemcpyHostToDevice, st));
    for (int k = 0; k < kKernels; ++k) tiny<<<kBlocks, kThreads, 0, st>>>(d + k * kBlocks * kThreads, it + k);
    return 0;
}

static double now_us()
{
    return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

int main()
{
    hipStream_t st;
    CK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    int* d;
    void* dtab;
    void* h;
    CK(hipMalloc(&d, sizeof(int) * kKernels * kBlocks * kThreads));
    CK(hipMalloc(&dtab, kCopy));
    CK(hipHostMalloc(&h, kCopy, hipHostMallocDefault));
    const int warm = 200, n = 2000;
    double t0;

    for (int it = 0; it < warm + n; ++it) {
        if (it == warm) t0 = now_us();
        if (enqueue(st, d, h, dtab, it)) return 1;
        CK(hipStreamSynchronize(st));
    }
    printf("eager   : %7.2f us per level\n", (now_us() - t0) / n);

    for (int it = 0; it < warm + n; ++it) {
        if (it == warm) t0 = now_us();
        hipGraph_t g;
        hipGraphExec_t ge;
        CK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        if (enqueue(st, d, h, dtab, it)) return 1;
        CK(hipStreamEndCapture(st, &g));
        CK(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
        CK(hipGraphLaunch(ge, st));
        CK(hipStreamSynchronize(st));
        CK(hipGraphExecDestroy(ge));
        CK(hipGraphDestroy(g));
    }
    printf("capture : %7.2f us per level\n", (now_us() - t0) / n);

    {
        hipGraph_t g0;
        hipGraphExec_t ge;
        CK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        if (enqueue(st, d, h, dtab, 0)) return 1;
        CK(hipStreamEndCapture(st, &g0));
        CK(hipGraphInstantiate(&ge, g0, nullptr, nullptr, 0));
        int failed = 0;
        for (int it = 0; it < warm + n; ++it) {
            if (it == warm) t0 = now_us();
            hipGraph_t g;
            CK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
            if (enqueue(st, d, h, dtab, it)) return 1;
            CK(hipStreamEndCapture(st, &g));
            hipGraphNode_t bad = nullptr;
            hipGraphExecUpdateResult res;
            if (hipGraphExecUpdate(ge, g, &bad, &res) != hipSuccess) ++failed;
            CK(hipGraphLaunch(ge, st));
            CK(hipStreamSynchronize(st));
            CK(hipGraphDestroy(g));
        }
        printf("update  : %7.2f us per level (%d updates refused)\n", (now_us() - t0) / n, failed);
        hipGraphExec_t ge0;
        CK(hipGraphInstantiate(&ge0, g0, nullptr, nullptr, 0));
        for (int it = 0; it < warm + n; ++it) {
            if (it == warm) t0 = now_us();
            CK(hipGraphLaunch(ge0, st));
            CK(hipStreamSynchronize(st));
        }
        printf("replay  : %7.2f us per level\n", (now_us() - t0) / n);
        CK(hipGraphExecDestroy(ge0));
        CK(hipGraphExecDestroy(ge));
        CK(hipGraphDestroy(g0));
    }
    // the last value each kernel wrote must be what the last replay wrote
    int last[kKernels];
    for (int k = 0; k < kKernels; ++k)
        CK(hipMemcpy(&last[k], d + k * kBlocks * kThreads, sizeof(int), hipMemcpyDeviceToHost));
    int ok = 1;
    for (int k = 0; k < kKernels; ++k) ok &= last[k] == k;
    printf("replayed values %s\n", ok ? "ok" : "WRONG");
    CK(hipHostFree(h));
    CK(hipFree(dtab));
    CK(hipFree(d));
    return ok ? 0 : 1;
}
