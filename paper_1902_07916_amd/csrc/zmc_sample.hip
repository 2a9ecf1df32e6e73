// zmc_sample.hip -- the precompiled sampling kernels: one translation unit
// per registry integrand (-DZMC_F=<id>), each instantiating D = 1..16 in FP64
// and FP32 evaluation around the shared body in zmc_sample_core.hpp.
#include "zmc_integrands.hpp"
#include "zmc_kernels.hpp"
#include "zmc_sample_core.hpp"

#ifndef ZMC_F
#error "compile with -DZMC_F=<integrand id>"
#endif

namespace zmc {

namespace {

template <int F, int D, bool FP32>
__global__ __launch_bounds__(kSampleThreads) void sample_kernel(const SampleArgs a)
{
    sample_units<Integrand<F, D>, D, FP32>(a);
}

template <int F, int D>
hipError_t launch_d(int eval, int grid, hipStream_t st, const SampleArgs& a)
{
    if (eval == ZMC_EVAL_FP32)
        hipLaunchKernelGGL((sample_kernel<F, D, true>), dim3(grid), dim3(kSampleThreads), 0, st, a);
    else
        hipLaunchKernelGGL((sample_kernel<F, D, false>), dim3(grid), dim3(kSampleThreads), 0, st, a);
    return hipGetLastError();
}

template <int F, int D>
const void* ptr_d(int eval)
{
    return eval == ZMC_EVAL_FP32 ? (const void*)&sample_kernel<F, D, true> : (const void*)&sample_kernel<F, D, false>;
}

} // namespace

#define ZMC_CAT2(a, b) a##b
#define ZMC_CAT(a, b) ZMC_CAT2(a, b)

#define ZMC_DIM_CASES(X)                                                                                   \
    X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)

hipError_t ZMC_CAT(launch_sample_, ZMC_F)(int dim, int eval, int grid, hipStream_t st, const SampleArgs& a)
{
    switch (dim) {
#define X(d)                                                                                               \
    case d: return launch_d<ZMC_F, d>(eval, grid, st, a);
        ZMC_DIM_CASES(X)
#undef X
    default: return hipErrorInvalidValue;
    }
}

const void* ZMC_CAT(sample_kernel_ptr_, ZMC_F)(int dim, int eval)
{
    switch (dim) {
#define X(d)                                                                                               \
    case d: return ptr_d<ZMC_F, d>(eval);
        ZMC_DIM_CASES(X)
#undef X
    default: return nullptr;
    }
}

} // namespace zmc
