// zmc_sample.hip -- the hot kernel: direct Monte Carlo over (cube, trial,
// chunk) units with random numbers produced at the time of use (ZMCintegral,
// Sec. 2.1 and Sec. 2.2).  Compiled once per integrand (-DZMC_F=<id>); every
// translation unit instantiates D = 1..16 in FP64 and FP32 evaluation.
//
// Work decomposition (gfx950, wave64): a block of 256 threads takes one
// (cube, trial, chunk) unit at a time; a chunk is 4 * 256 * G points and
// thread t evaluates the 4-point groups g = chunk*G*256 + t + 256*j, j < G.
// One group of 4 points uses D Philox blocks (4*D words, point q dimension i
// = word q*D + i), so the counter word 0 of block k is g*D + k and the other
// three counter words and the key are wave-uniform (SGPRs).  Each thread sums
// f and f^2 in FP64; the block reduces with wave64 butterflies and LDS in a
// fixed order, so a unit's partial sums depend only on the unit and G.
// The grid is persistent: block b takes a contiguous range of units, and
// only the first unit's segment is found by binary search.
#include "zmc_integrands.hpp"
#include "zmc_kernels.hpp"

#ifndef ZMC_F
#error "compile with -DZMC_F=<integrand id>"
#endif

namespace zmc {

namespace {

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <int D>
__device__ __forceinline__ void corner(const SlotDesc& sd, int level, uint64_t uid, double* lo, double* h)
{
    uint64_t K[D];
    uint64_t root = (D * level >= 64) ? 0 : (uid >> (uint64_t)(D * level));
    const uint32_t d = (uint32_t)sd.divisions;
    if (root < (1ull << 32)) {
        uint32_t r32 = (uint32_t)root;
#pragma unroll
        for (int i = D - 1; i >= 0; --i) {
            K[i] = r32 % d;
            r32 /= d;
        }
    } else {
#pragma unroll
        for (int i = D - 1; i >= 0; --i) {
            K[i] = root % d;
            root /= d;
        }
    }
    for (int j = 1; j <= level; ++j) {
        const uint64_t c = uid >> (uint64_t)(D * (level - j));
#pragma unroll
        for (int i = 0; i < D; ++i) K[i] = 2u * K[i] + ((c >> (uint64_t)(D - 1 - i)) & 1u);
    }
#pragma unroll
    for (int i = 0; i < D; ++i) {
        h[i] = ldexp(sd.h0[i], -level);
        lo[i] = fma((double)K[i], h[i], sd.lower[i]);
    }
}

template <int F, int D, bool FP32>
__global__ __launch_bounds__(kSampleThreads) void sample_kernel(const SampleArgs a)
{
    using I = Integrand<F, D>;
    __shared__ double red[2][kSampleThreads / 64];
    const int tid = threadIdx.x;
    const int64_t U = a.total_units;
    const int64_t per = (U + gridDim.x - 1) / gridDim.x;
    int64_t u = (int64_t)blockIdx.x * per;
    const int64_t uend = min(U, u + per);
    if (u >= uend) return;

    int bs = 0;
    {
        int hi = a.n_bsegs - 1;
        while (bs < hi) {
            const int mid = (bs + hi + 1) >> 1;
            if (a.bsegs[mid].unit_base <= u) bs = mid;
            else hi = mid - 1;
        }
    }

    for (; u < uend; ++u) {
        while (bs + 1 < a.n_bsegs && a.bsegs[bs + 1].unit_base <= u) ++bs;
        const Segment& sg = a.segs[a.bsegs[bs].seg];
        const SlotDesc& sd = a.slots[sg.slot];
        const int64_t local = u - a.bsegs[bs].unit_base;
        const int nch = sd.nch;
        const int64_t upc = (int64_t)sd.trials * nch;
        const int64_t cl = local / upc;
        const int rem = (int)(local - cl * upc);
        const int trial = rem / nch;
        const int chunk = rem - trial * nch;
        const uint64_t uid = a.uid[sg.cube_base + cl];
        const int level = sg.level;

        double lo[D], h[D];
        corner<D>(sd, level, uid, lo, h);

        const uint32_t k0 = (uint32_t)sd.seed, k1 = (uint32_t)(sd.seed >> 32);
        const uint32_t c1 = (uint32_t)trial | ((uint32_t)level << 8);
        const uint32_t c2 = (uint32_t)uid, c3 = (uint32_t)(uid >> 32);
        const int64_t N = sd.samples;
        const int G = sd.groups;
        const int64_t g0 = (int64_t)chunk * G * kSampleThreads + tid;

        double S1 = 0.0, S2 = 0.0;
        if constexpr (FP32) {
            typename I::P32 p;
            I::prep32(sd, lo, h, p);
            for (int j = 0; j < G; ++j) {
                const int64_t g = g0 + (int64_t)j * kSampleThreads;
                const int64_t s0 = 4 * g;
                if (s0 >= N) break;
                const int nvalid = (int)min((int64_t)4, N - s0); // < 4 only in a ragged last group
                uint32_t w[4 * D];
                uint32_t ctr[D];
                const uint32_t cb = (uint32_t)g * (uint32_t)D;
#pragma unroll
                for (int k = 0; k < D; ++k) ctr[k] = cb + (uint32_t)k;
                philox4x32_10_lockstep<D>(ctr, c1, c2, c3, k0, k1, w);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    float v[D];
#pragma unroll
                    for (int i = 0; i < D; ++i) v[i] = unit_interval_f32(w[q * D + i]);
                    float f = I::f32(p, v);
                    f = (q < nvalid) ? f : 0.0f;
                    const double fd = (double)f;
                    S1 += fd;
                    S2 = fma(fd, fd, S2);
                }
            }
        } else {
            typename I::P64 p;
            I::prep64(sd, p);
            double h24[D];
#pragma unroll
            for (int i = 0; i < D; ++i) h24[i] = ldexp(h[i], -24);
            for (int j = 0; j < G; ++j) {
                const int64_t g = g0 + (int64_t)j * kSampleThreads;
                const int64_t s0 = 4 * g;
                if (s0 >= N) break;
                const int nvalid = (int)min((int64_t)4, N - s0);
                uint32_t w[4 * D];
                uint32_t ctr[D];
                const uint32_t cb = (uint32_t)g * (uint32_t)D;
#pragma unroll
                for (int k = 0; k < D; ++k) ctr[k] = cb + (uint32_t)k;
                philox4x32_10_lockstep<D>(ctr, c1, c2, c3, k0, k1, w);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    double x[D];
                    // x = fma(h, (2*(w>>9)+1) 2^-24, lo) computed as
                    // fma(h 2^-24, (w>>8)|1, lo): the same exact product
#pragma unroll
                    for (int i = 0; i < D; ++i) x[i] = fma(h24[i], (double)((w[q * D + i] >> 8) | 1u), lo[i]);
                    double f = I::f64(p, x);
                    f = (q < nvalid) ? f : 0.0;
                    S1 += f;
                    S2 = fma(f, f, S2);
                }
            }
        }

        S1 = wave_sum(S1);
        S2 = wave_sum(S2);
        if ((tid & 63) == 0) {
            red[0][tid >> 6] = S1;
            red[1][tid >> 6] = S2;
        }
        __syncthreads();
        if (tid == 0) {
            double t1 = red[0][0], t2 = red[1][0];
#pragma unroll
            for (int wv = 1; wv < kSampleThreads / 64; ++wv) {
                t1 += red[0][wv];
                t2 += red[1][wv];
            }
            a.partial[sg.part_base + local] = make_double2(t1, t2);
        }
        __syncthreads();
    }
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
