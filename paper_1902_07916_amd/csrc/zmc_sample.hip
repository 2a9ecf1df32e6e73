// zmc_sample.hip -- the precompiled sampling kernels: one translation unit
// per registry integrand (-DZMC_F=<id>), each instantiating D = 1..16 in FP64
// and FP32 evaluation, in every occupancy variant and in the variant that
// keeps sums of squares, around the shared body in zmc_sample_core.hpp.
#include "zmc_integrands.hpp"
#include "zmc_kernels.hpp"
#include "zmc_sample_core.hpp"

#ifndef ZMC_F
#error "compile with -DZMC_F=<integrand id>"
#endif

namespace zmc {

namespace {

template <int F, int D, bool FP32, int W>
__global__ __launch_bounds__(kSampleThreads) __attribute__((amdgpu_waves_per_eu(W))) void sample_kernel(
    const SampleArgs a)
{
    sample_units<Integrand<F, D>, D, FP32, false, W>(a);
}

// the variant that also keeps the sums of squares, for traced levels
template <int F, int D, bool FP32>
__global__ __launch_bounds__(kSampleThreads) void sample_sums_kernel(const SampleArgs a)
{
    sample_units<Integrand<F, D>, D, FP32, true>(a);
}

template <int F, int D, bool FP32>
const void* ptr_dew(int hint)
{
    static_assert(kNumWaveHints == 4, "one case per occupancy variant");
    switch (hint) {
    case 1: return (const void*)&sample_kernel<F, D, FP32, kWaveHints[1]>;
    case 2: return (const void*)&sample_kernel<F, D, FP32, kWaveHints[2]>;
    case 3: return (const void*)&sample_kernel<F, D, FP32, kWaveHints[3]>;
    case kSumsVariant: return (const void*)&sample_sums_kernel<F, D, FP32>;
    default: return (const void*)&sample_kernel<F, D, FP32, kWaveHints[0]>;
    }
}

template <int F, int D>
const void* ptr_d(int eval, int hint)
{
    return eval == ZMC_EVAL_FP32 ? ptr_dew<F, D, true>(hint) : ptr_dew<F, D, false>(hint);
}

template <int F, int D>
hipError_t launch_d(int eval, int hint, int grid, int block, hipStream_t st, const SampleArgs& a)
{
    SampleArgs arg = a;
    void* args[] = {&arg};
    return hipLaunchKernel(ptr_d<F, D>(eval, hint), dim3(grid), dim3(block), args, 0, st);
}

} // namespace

#define ZMC_CAT2(a, b) a##b
#define ZMC_CAT(a, b) ZMC_CAT2(a, b)

#define ZMC_DIM_CASES(X)                                                                                   \
    X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)

hipError_t ZMC_CAT(launch_sample_, ZMC_F)(int dim, int eval, int hint, int grid, int block, hipStream_t st,
                                          const SampleArgs& a)
{
    switch (dim) {
#define X(d)                                                                                               \
    case d: return launch_d<ZMC_F, d>(eval, hint, grid, block, st, a);
        ZMC_DIM_CASES(X)
#undef X
    default: return hipErrorInvalidValue;
    }
}

const void* ZMC_CAT(sample_kernel_ptr_, ZMC_F)(int dim, int eval, int hint)
{
    switch (dim) {
#define X(d)                                                                                               \
    case d: return ptr_d<ZMC_F, d>(eval, hint);
        ZMC_DIM_CASES(X)
#undef X
    default: return nullptr;
    }
}

} // namespace zmc
