// queue_share.hip -- how long a one-block kernel on a second stream waits
// while another stream keeps the device full, for three shapes of the
// long work: (0) one non-persistent grid of 2048 * 1000 short blocks,
// (1) a chain of 1000 launches of 2048 blocks, (2) one persistent grid of
// 2048 blocks that each loop 1000 times longer.  All loops are bounded.
// Build:
//   hipcc -O2 --offload-arch=gfx950 -Xclang -target-feature -Xclang -packed-fp32-ops \
//         paper_1902_07916_amd/probes/queue_share.hip -o queue_share
#include <hip/hip_runtime.h>
#include <chrono>
#include <cstdio>
#include <thread>

__global__ void spin(int iters, float* out)
{
    float a = threadIdx.x * 1e-3f;
    for (int i = 0; i < iters; ++i) a = a * 0.999f + 1e-4f;
    if (a == 1234.5f) out[0] = a; // never true; keeps the loop
}

#define CK(x)                                                                                                   \
    do {                                                                                                        \
        hipError_t e_ = (x);                                                                                    \
        if (e_ != hipSuccess) {                                                                                 \
            printf("%s: %s\n", #x, hipGetErrorString(e_));                                                      \
            return 1;                                                                                           \
        }                                                                                                       \
    } while (0)

static double now_ms()
{
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

int main()
{
    float* out;
    CK(hipMalloc(&out, 4));
    hipStream_t busy, probe;
    CK(hipStreamCreateWithFlags(&busy, hipStreamNonBlocking));
    CK(hipStreamCreateWithFlags(&probe, hipStreamNonBlocking));
    hipEvent_t e0, e1;
    CK(hipEventCreate(&e0));
    CK(hipEventCreate(&e1));
    float ms;
    CK(hipEventRecord(e0, busy));
    spin<<<2048, 256, 0, busy>>>(20000, out);
    CK(hipEventRecord(e1, busy));
    CK(hipEventSynchronize(e1));
    CK(hipEventElapsedTime(&ms, e0, e1));
    printf("2048 blocks x 20000 iterations: %.3f ms\n", ms);
    double t = now_ms();
    spin<<<1, 64, 0, probe>>>(100, out);
    CK(hipStreamSynchronize(probe));
    printf("one-block kernel alone: %.3f ms\n", now_ms() - t);
    const char* names[3] = {"one grid of short blocks", "chain of launches", "persistent grid"};
    for (int mode = 0; mode < 3; ++mode) {
        CK(hipEventRecord(e0, busy));
        if (mode == 0) {
            spin<<<2048 * 1000, 256, 0, busy>>>(20000, out);
        } else if (mode == 1) {
            for (int k = 0; k < 1000; ++k) spin<<<2048, 256, 0, busy>>>(20000, out);
        } else {
            spin<<<2048, 256, 0, busy>>>(20000 * 1000, out);
        }
        CK(hipEventRecord(e1, busy));
        std::this_thread::sleep_for(std::chrono::milliseconds(20));
        double worst = 0, sum = 0;
        for (int r = 0; r < 5; ++r) {
            t = now_ms();
            spin<<<1, 64, 0, probe>>>(100, out);
            CK(hipStreamSynchronize(probe));
            const double d = now_ms() - t;
            sum += d;
            worst = d > worst ? d : worst;
        }
        CK(hipEventSynchronize(e1));
        CK(hipEventElapsedTime(&ms, e0, e1));
        printf("%-26s: long work %.1f ms; one-block kernel mean %.3f worst %.3f ms\n", names[mode], ms, sum / 5,
               worst);
    }
    return 0;
}
