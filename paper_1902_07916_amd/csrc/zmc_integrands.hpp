// zmc_integrands.hpp -- the integrand registry on the device, in two forms:
//
//  * FP64: f(x) from the absolute point x, the plain definition;
//  * FP32: f from the per-dimension cell values v_i in [1, 2) (see
//    unit_interval_f32) and per-cube constants formed once in FP64, so that
//    every FP32 quantity is cube-relative (an offset from the cube corner, a
//    phase reduced modulo one revolution).  Absolute coordinates such as
//    x ~ 10 never enter FP32 arithmetic.
//
// With u = v - (1 - 2^-24) and x_i = lo_i + h_i u_i, every coordinate is
// x_i = b_i + h_i v_i with b_i = lo_i - h_i (1 - 2^-24).
//
// FP32 range: an FP32 form evaluates f / scale, where scale (P32::scale,
// FP64, per cube) carries the integrand's amplitude and, where the family
// allows, its size at the cube's nearest point (e.g. the Gaussian's value
// there); the sampling body multiplies each unit's FP64 sum by it.  The FP32
// values are then of order one near the cube's largest values instead of
// underflowing with the amplitude.  Families whose FP32 values can still
// fall below the normal range (kRangeCheck) have every unit's sum checked.
//
// The paper's test functions are f1 = sin(sum x_i) and the 9-D Gaussian f2
// (Sec. 3); the Genz families are the batched/serving workloads' integrands.
#pragma once

#include "zmc_device.hpp"

namespace zmc {

constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr double kInvTwoPi = 0.15915494309189533576888376337251;
constexpr double kLog2e = 1.4426950408889634073599246810019;
constexpr double kOneMinus = 1.0 - 0x1p-24;

// sin(2 pi r): r is reduced by the exact steps t = r - rint(r) and
// a = min(|t|, 1/2 - |t|) in [0, 1/4], which keep the result odd-symmetric
// (so its error has no mean over a period); the Taylor series of
// sin(2 pi a) through a^13 (truncation < 7e-10) is summed by Horner in a^2
// and takes the sign of t.  Coefficients: (-1)^k (2 pi)^(2k+1) / (2k+1)!.
__device__ __forceinline__ float sin_rev(float r)
{
    const float t = r - __builtin_rintf(r);
    // fold |t| in [0, 1/2] to a in [0, 1/4] with sin(2 pi |t|) = sin(2 pi a):
    // 1/2 - |t| is exact for |t| >= 1/4, and min() is a floating-point
    // instruction, so the fold needs no integer select
    const float at = __builtin_fabsf(t);
    const float a = __builtin_fminf(at, 0.5f - at);
    const float t2 = a * a;
    float p = 3.8199524879455566f;
    p = __builtin_fmaf(p, t2, -15.094642639160156f);
    p = __builtin_fmaf(p, t2, 42.058692932128906f);
    p = __builtin_fmaf(p, t2, -76.70585632324219f);
    p = __builtin_fmaf(p, t2, 81.6052474975586f);
    p = __builtin_fmaf(p, t2, -41.34170150756836f);
    p = __builtin_fmaf(p, t2, 6.2831854820251465f);
    return __builtin_copysignf(p * a, t); // the polynomial is odd: sin(2 pi t) = sign(t) sin(2 pi a)
}

// 2^y in FP64 for |y| up to the exponent range, from the FP32 exp2 of the
// fractional part (relative error about 1e-7, the size of FP32 rounding) and
// an exact ldexp: a per-cube scale without an FP64 exp, whose temporaries
// would raise the sampling kernel's register count.
__device__ __forceinline__ double exp2_scale(double y)
{
    const double fl = floor(y);
    return ldexp((double)__builtin_amdgcn_exp2f((float)(y - fl)), (int)fmax(fmin(fl, 2000.0), -2000.0));
}

// frac(x) in FP64 for the per-cube phase offsets.
__device__ __forceinline__ double frac64(double x) { return x - floor(x); }

// A per-cube phase offset (revolutions) as a float pair hi + lo.
__device__ __forceinline__ void split_phase(double r0, float& hi, float& lo)
{
    hi = (float)r0;
    lo = (float)(r0 - (double)hi);
}

// Phase of a point in revolutions: r0 + sum m_i v_i in FP32.  The cube
// offsets r0 form a lattice, so rounding r0 itself to FP32 would give errors
// that correlate with the phases and do not average out over the domain (for
// sin(sum x) over [0,10]^6, whose integral is 1.3e4 times smaller than that of
// |f|, it biases the result by ~1e-4).  The low part therefore enters first,
// where the rounding varies from point to point: fma(m_0, v_0, lo), then + hi.
template <int D>
__device__ __forceinline__ float phase_sum(const float* m, const float* v, float hi, float lo)
{
    float r = __builtin_fmaf(m[0], v[0], lo) + hi;
#pragma unroll
    for (int i = 1; i < D; ++i) r = __builtin_fmaf(m[i], v[i], r);
    return r;
}

// Integer power by squaring (exponent known per launch, small).
template <typename T>
__device__ __forceinline__ T ipow(T x, int n)
{
    T r = (T)1;
    while (n > 0) {
        if (n & 1) r *= x;
        x *= x;
        n >>= 1;
    }
    return r;
}

template <int F, int D>
struct Integrand;

// ---- ZMC_GAUSS: A exp(-sum (x_i - mu_i)^2 / (2 sigma^2)) -------------------
// FP32: exp2(k2 (q - q0)) with q = sum (x_i - mu_i)^2, k2 = -log2(e) / (2
// sigma^2) and q0 the FP32 value of q's minimum over the cube; scale =
// A 2^(k2 q0) in FP64, so the product is A exp2(k2 q) with the amplitude and
// the cube's distance from the peak outside FP32.
template <int D>
struct Integrand<ZMC_GAUSS, D> {
    static constexpr bool kRangeCheck = true;
    struct P64 {
        double mu[D], k, A;
    };
    struct P32 {
        float a[D], m[D], k2, q0;
        double scale;
    };
    __device__ static void prep64(const SlotDesc& sd, P64& p)
    {
        const double s = sd.params[0];
        p.A = sd.params[1];
        p.k = -1.0 / (2.0 * s * s);
        for (int i = 0; i < D; ++i) p.mu[i] = sd.params[2 + i];
    }
    __device__ static double f64(const P64& p, const double* x)
    {
        double q = 0.0;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const double d = x[i] - p.mu[i];
            q = fma(d, d, q);
        }
        return p.A * exp(q * p.k);
    }
    __device__ static void prep32(const SlotDesc& sd, const double* lo, const double* h, P32& p)
    {
        const double s = sd.params[0];
        const double k2 = -kLog2e / (2.0 * s * s);
        double qmin = 0.0;
        for (int i = 0; i < D; ++i) {
            const double mu = sd.params[2 + i];
            p.a[i] = (float)(lo[i] - h[i] * kOneMinus - mu);
            p.m[i] = (float)h[i];
            const double d = fmax(0.0, fmax(lo[i] - mu, mu - (lo[i] + h[i])));
            qmin = fma(d, d, qmin);
        }
        p.k2 = (float)k2;
        p.q0 = (float)qmin;
        p.scale = sd.params[1] * exp2_scale(k2 * (double)p.q0);
    }
    __device__ static float f32(const P32& p, const float* v)
    {
        float q = -p.q0;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const float t = __builtin_fmaf(p.m[i], v[i], p.a[i]);
            q = __builtin_fmaf(t, t, q);
        }
        return __builtin_amdgcn_exp2f(q * p.k2);
    }
};

// ---- ZMC_SIN_SUM: sin(sum x_i) ---------------------------------------------
template <int D>
struct Integrand<ZMC_SIN_SUM, D> {
    struct P64 {
        int dummy;
    };
    static constexpr bool kRangeCheck = false; // |f| is not small over a cube: a sum near 0 is cancellation
    struct P32 {
        float m[D], r0_hi, r0_lo;
        double scale;
    };
    __device__ static void prep64(const SlotDesc&, P64&) {}
    __device__ static double f64(const P64&, const double* x)
    {
        double t = 0.0;
#pragma unroll
        for (int i = 0; i < D; ++i) t += x[i];
        return sin(t);
    }
    __device__ static void prep32(const SlotDesc&, const double* lo, const double* h, P32& p)
    {
        double b = 0.0;
        for (int i = 0; i < D; ++i) {
            b += lo[i] - h[i] * kOneMinus;
            p.m[i] = (float)(h[i] * kInvTwoPi);
        }
        split_phase(frac64(b * kInvTwoPi), p.r0_hi, p.r0_lo);
        p.scale = 1.0;
    }
    __device__ static float f32(const P32& p, const float* v) { return sin_rev(phase_sum<D>(p.m, v, p.r0_hi, p.r0_lo)); }
};

// ---- ZMC_GENZ_OSC: cos(2 pi u + sum c_i x_i) = sin(2 pi (u + 1/4 + sum c_i x_i / 2pi))
template <int D>
struct Integrand<ZMC_GENZ_OSC, D> {
    static constexpr bool kRangeCheck = false; // as for the sine
    struct P64 {
        double c[D], ph;
    };
    struct P32 {
        float m[D], r0_hi, r0_lo;
        double scale;
    };
    __device__ static void prep64(const SlotDesc& sd, P64& p)
    {
        p.ph = kTwoPi * sd.params[0];
        for (int i = 0; i < D; ++i) p.c[i] = sd.params[1 + i];
    }
    __device__ static double f64(const P64& p, const double* x)
    {
        double t = p.ph;
#pragma unroll
        for (int i = 0; i < D; ++i) t = fma(p.c[i], x[i], t);
        return cos(t);
    }
    __device__ static void prep32(const SlotDesc& sd, const double* lo, const double* h, P32& p)
    {
        double b = sd.params[0] + 0.25; // revolutions
        for (int i = 0; i < D; ++i) {
            const double c = sd.params[1 + i];
            b += c * (lo[i] - h[i] * kOneMinus) * kInvTwoPi;
            p.m[i] = (float)(c * h[i] * kInvTwoPi);
        }
        split_phase(frac64(b), p.r0_hi, p.r0_lo);
        p.scale = 1.0;
    }
    __device__ static float f32(const P32& p, const float* v) { return sin_rev(phase_sum<D>(p.m, v, p.r0_hi, p.r0_lo)); }
};

// ---- ZMC_GENZ_PPEAK: prod 1 / (c_i^-2 + (x_i - w_i)^2) ----------------------
// FP32: prod 1 / (1 + u_i^2) with u_i = c_i (x_i - w_i); scale = prod c_i^2.
template <int D>
struct Integrand<ZMC_GENZ_PPEAK, D> {
    static constexpr bool kRangeCheck = true;
    struct P64 {
        double e[D], w[D];
    };
    struct P32 {
        float a[D], m[D];
        double scale;
    };
    __device__ static void prep64(const SlotDesc& sd, P64& p)
    {
        for (int i = 0; i < D; ++i) {
            const double c = sd.params[i];
            p.e[i] = 1.0 / (c * c);
            p.w[i] = sd.params[D + i];
        }
    }
    __device__ static double f64(const P64& p, const double* x)
    {
        double den = 1.0;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const double d = x[i] - p.w[i];
            den *= fma(d, d, p.e[i]);
        }
        return 1.0 / den;
    }
    __device__ static void prep32(const SlotDesc& sd, const double* lo, const double* h, P32& p)
    {
        double scale = 1.0;
        for (int i = 0; i < D; ++i) {
            const double c = sd.params[i];
            p.a[i] = (float)(c * (lo[i] - h[i] * kOneMinus - sd.params[D + i]));
            p.m[i] = (float)(c * h[i]);
            scale *= c * c;
        }
        p.scale = scale;
    }
    __device__ static float f32(const P32& p, const float* v)
    {
        float den = 1.0f;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const float u = __builtin_fmaf(p.m[i], v[i], p.a[i]);
            den *= __builtin_fmaf(u, u, 1.0f);
        }
        return __builtin_amdgcn_rcpf(den);
    }
};

// ---- ZMC_GENZ_CPEAK: (1 + sum c_i x_i)^-(D+1) -------------------------------
// FP32: tau^-(D+1) with tau = t / t0, t = 1 + sum c_i x_i and t0 its value at
// the cube's lower corner (when positive); scale = t0^-(D+1).
template <int D>
struct Integrand<ZMC_GENZ_CPEAK, D> {
    static constexpr bool kRangeCheck = true;
    struct P64 {
        double c[D];
    };
    struct P32 {
        float m[D], b0;
        double scale;
    };
    __device__ static void prep64(const SlotDesc& sd, P64& p)
    {
        for (int i = 0; i < D; ++i) p.c[i] = sd.params[i];
    }
    __device__ static double f64(const P64& p, const double* x)
    {
        double t = 1.0;
#pragma unroll
        for (int i = 0; i < D; ++i) t = fma(p.c[i], x[i], t);
        return 1.0 / ipow(t, D + 1);
    }
    __device__ static void prep32(const SlotDesc& sd, const double* lo, const double* h, P32& p)
    {
        double b = 1.0, t0 = 1.0;
        for (int i = 0; i < D; ++i) {
            const double c = sd.params[i];
            b += c * (lo[i] - h[i] * kOneMinus);
            t0 += c * lo[i];
        }
        const double r = t0 > 0.0 ? 1.0 / t0 : 1.0;
        for (int i = 0; i < D; ++i) p.m[i] = (float)(sd.params[i] * h[i] * r);
        p.b0 = (float)(b * r);
        p.scale = t0 > 0.0 ? 1.0 / ipow(t0, D + 1) : 1.0;
    }
    __device__ static float f32(const P32& p, const float* v)
    {
        float t = p.b0;
#pragma unroll
        for (int i = 0; i < D; ++i) t = __builtin_fmaf(p.m[i], v[i], t);
        return __builtin_amdgcn_rcpf(ipow(t, D + 1));
    }
};

// ---- ZMC_GENZ_GAUSS: exp(-sum c_i^2 (x_i - w_i)^2) --------------------------
// FP32: exp2(-(q - q0)) with q = log2(e) sum c_i^2 (x_i - w_i)^2 and q0 the
// FP32 value of q's minimum over the cube; scale = 2^-q0.
template <int D>
struct Integrand<ZMC_GENZ_GAUSS, D> {
    static constexpr bool kRangeCheck = true;
    struct P64 {
        double c[D], w[D];
    };
    struct P32 {
        float a[D], m[D], q0;
        double scale;
    };
    __device__ static void prep64(const SlotDesc& sd, P64& p)
    {
        for (int i = 0; i < D; ++i) {
            p.c[i] = sd.params[i];
            p.w[i] = sd.params[D + i];
        }
    }
    __device__ static double f64(const P64& p, const double* x)
    {
        double q = 0.0;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const double t = p.c[i] * (x[i] - p.w[i]);
            q = fma(t, t, q);
        }
        return exp(-q);
    }
    __device__ static void prep32(const SlotDesc& sd, const double* lo, const double* h, P32& p)
    {
        // exp(-q) = exp2(-q log2 e): fold sqrt(log2 e) into the offsets
        const double s = sqrt(kLog2e);
        double qmin = 0.0;
        for (int i = 0; i < D; ++i) {
            const double c = sd.params[i] * s, w = sd.params[D + i];
            p.a[i] = (float)(c * (lo[i] - h[i] * kOneMinus - w));
            p.m[i] = (float)(c * h[i]);
            const double d = c * fmax(0.0, fmax(lo[i] - w, w - (lo[i] + h[i])));
            qmin = fma(d, d, qmin);
        }
        p.q0 = (float)qmin;
        p.scale = exp2_scale(-(double)p.q0);
    }
    __device__ static float f32(const P32& p, const float* v)
    {
        float q = -p.q0;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const float t = __builtin_fmaf(p.m[i], v[i], p.a[i]);
            q = __builtin_fmaf(t, t, q);
        }
        return __builtin_amdgcn_exp2f(-q);
    }
};

// ---- ZMC_CONST: A -------------------------------------------------------------
// FP32: 1, scale = A (every unit's sum is then exact).
template <int D>
struct Integrand<ZMC_CONST, D> {
    static constexpr bool kRangeCheck = false;
    struct P64 {
        double A;
    };
    struct P32 {
        double scale;
    };
    __device__ static void prep64(const SlotDesc& sd, P64& p) { p.A = sd.params[0]; }
    __device__ static double f64(const P64& p, const double*) { return p.A; }
    __device__ static void prep32(const SlotDesc& sd, const double*, const double*, P32& p)
    {
        p.scale = sd.params[0];
    }
    __device__ static float f32(const P32&, const float*) { return 1.0f; }
};

// ---- ZMC_MONOMIAL: prod x_i^p_i -----------------------------------------------
// FP32: prod (x_i / r_i)^p_i with r_i = max |x_i| over the cube; scale =
// prod r_i^p_i.
template <int D>
struct Integrand<ZMC_MONOMIAL, D> {
    static constexpr bool kRangeCheck = true;
    struct P64 {
        int e[D];
    };
    struct P32 {
        float b[D], m[D];
        int e[D];
        double scale;
    };
    __device__ static void prep64(const SlotDesc& sd, P64& p)
    {
        for (int i = 0; i < D; ++i) p.e[i] = (int)sd.params[i];
    }
    __device__ static double f64(const P64& p, const double* x)
    {
        double f = 1.0;
#pragma unroll
        for (int i = 0; i < D; ++i) f *= ipow(x[i], p.e[i]);
        return f;
    }
    __device__ static void prep32(const SlotDesc& sd, const double* lo, const double* h, P32& p)
    {
        double scale = 1.0;
        for (int i = 0; i < D; ++i) {
            const double r = fmax(fabs(lo[i]), fabs(lo[i] + h[i]));
            p.e[i] = (int)sd.params[i];
            p.b[i] = (float)((lo[i] - h[i] * kOneMinus) / r);
            p.m[i] = (float)(h[i] / r);
            scale *= ipow(r, p.e[i]);
        }
        p.scale = scale;
    }
    __device__ static float f32(const P32& p, const float* v)
    {
        float f = 1.0f;
#pragma unroll
        for (int i = 0; i < D; ++i) f *= ipow(__builtin_fmaf(p.m[i], v[i], p.b[i]), p.e[i]);
        return f;
    }
};

} // namespace zmc
