// Device-side arithmetic of the renewal tau-leap step for gfx950:
// compensated (float-float) logarithm, the four hazards, and the
// Philox4x32-10 draw.  FP32 only; no double precision on the device.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fs_internal.hpp"

extern "C" __device__ float __ocml_erfcx_f32(float);

namespace fsd {

using fsi::HazardDev;

// ---------------------------------------------------------------------------
// Float-float helpers (Dekker / Knuth error-free transformations).
// ---------------------------------------------------------------------------
struct ff {
    float hi, lo;
};

__device__ __forceinline__ ff two_sum(float a, float b)
{
    float s = a + b;
    float bb = s - a;
    float e = (a - (s - bb)) + (b - bb);
    return {s, e};
}

__device__ __forceinline__ ff quick_two_sum(float a, float b) // requires |a| >= |b|
{
    float s = a + b;
    return {s, b - (s - a)};
}

__device__ __forceinline__ ff two_prod(float a, float b)
{
    float p = a * b;
    return {p, __builtin_fmaf(a, b, -p)};
}

// 1/x by the hardware reciprocal (v_rcp_f32, within 1 ulp): a quarter of the
// instructions of a correctly rounded division, used where an ulp of the
// quotient is far inside the result's error budget.
__device__ __forceinline__ float rcp(float x)
{
    return __builtin_amdgcn_rcpf(x);
}

__device__ __forceinline__ ff ff_add(ff a, ff b)
{
    ff s = two_sum(a.hi, b.hi);
    float lo = s.lo + (a.lo + b.lo);
    return quick_two_sum(s.hi, lo);
}

__device__ __forceinline__ ff ff_mul(ff a, ff b)
{
    ff p = two_prod(a.hi, b.hi);
    float lo = p.lo + (a.hi * b.lo + a.lo * b.hi);
    return quick_two_sum(p.hi, lo);
}

// ---------------------------------------------------------------------------
// ln(x) for finite x > 0 as a float-float pair, accurate to about 2^-44
// relative.  x = m 2^e with m in [sqrt(1/2), sqrt(2)); ln m = 2 atanh(s),
// s = (m - 1)/(m + 1), |s| <= 0.1716, summed as 2s + 2s^3 P(s^2) with the
// atanh Taylor series truncated after the s^17 term (remainder < 2^-40).
// ---------------------------------------------------------------------------
__device__ __forceinline__ ff log_ff(float x)
{
    int e;
    float m = __builtin_frexpf(x, &e); // m in [0.5, 1)
    if (m < 0.70710678118654752f) {
        m = m * 2.0f;
        e -= 1;
    }
    float f = m - 1.0f; // exact (Sterbenz)
    ff d = two_sum(m, 1.0f);
    // s = f / d: an approximate quotient, its exact remainder (one fma), and
    // the remainder's quotient as the low part; s_hi need not be correctly
    // rounded for the remainder to be exact
    const float rd = rcp(d.hi);
    float s_hi = f * rd;
    float r = __builtin_fmaf(-s_hi, d.hi, f) - s_hi * d.lo;
    float s_lo = r * rd;
    float s2 = s_hi * s_hi;
    float p = 1.0f / 17.0f;
    p = __builtin_fmaf(p, s2, 1.0f / 15.0f);
    p = __builtin_fmaf(p, s2, 1.0f / 13.0f);
    p = __builtin_fmaf(p, s2, 1.0f / 11.0f);
    p = __builtin_fmaf(p, s2, 1.0f / 9.0f);
    p = __builtin_fmaf(p, s2, 1.0f / 7.0f);
    p = __builtin_fmaf(p, s2, 1.0f / 5.0f);
    p = __builtin_fmaf(p, s2, 1.0f / 3.0f);
    float tail = 2.0f * s_hi * s2 * p;
    // ln 2 split so that e * LN2_HI is exact for |e| < 2^8
    const float LN2_HI = 0.693145751953125f;
    const float LN2_LO = 1.428606820309417232e-06f;
    float fe = (float)e;
    ff a = two_sum(fe * LN2_HI, 2.0f * s_hi);
    float lo = a.lo + (fe * LN2_LO + (2.0f * s_lo + tail));
    return quick_two_sum(a.hi, lo);
}

// ---------------------------------------------------------------------------
// Hazards.  x is the age in the unit the parameters were prepared for
// (days, or an integer step count held exactly in a float).
// ---------------------------------------------------------------------------

// Proposition 1 (stable log-normal hazard): h = sqrt(2/pi)/(tau sigma erfcx(z)).
// z is formed in float-float (its condition number in ln tau reaches ~13 at
// small ages).  For z < 0 the reflection erfcx(z) = 2 exp(z^2) - erfcx(-z)
// is used with z^2 split exactly (hi + lo) so exp(z^2) = exp(hi)(1 + lo);
// exp(z^2) overflowing means h is below the FP32 range and returns 0.
// erfcx is evaluated once, at |z|, so a wavefront holding ages on both sides
// of the median pays for one evaluation.
__device__ __forceinline__ float hazard_lognormal(const HazardDev& h, float x)
{
    if (!(x > 0.0f)) return 0.0f;
    ff L = log_ff(x);
    ff t = ff_add(L, ff{h.c_hi, h.c_lo});
    ff z = ff_mul(t, ff{h.g_hi, h.g_lo});
    float ex = __ocml_erfcx_f32(__builtin_fabsf(z.hi));
    if (z.hi < 0.0f) {
        ff sq = two_prod(z.hi, z.hi);
        float lo = __builtin_fmaf(2.0f * z.hi, z.lo, sq.lo);
        float E = expf(sq.hi);
        // (an overflowed E stays infinite: inf * lo + inf would be NaN for lo < 0)
        E = __builtin_isinf(E) ? E : __builtin_fmaf(E, lo, E);
        ex = 2.0f * E - ex;
    }
    // (x ex = inf gives 0, the underflowed hazard)
    return h.K * rcp(x * ex);
}

// Weibull: h = (k/lambda) (tau/lambda)^(k-1), as K exp((k-1) ln(tau/lambda)).
__device__ __forceinline__ float hazard_weibull(const HazardDev& h, float x)
{
    if (h.g_hi == 0.0f) return h.K; // shape 1: exponential
    if (!(x > 0.0f)) return 0.0f;
    ff L = log_ff(x);
    ff u = ff_add(L, ff{h.c_hi, h.c_lo});
    ff t = ff_mul(u, ff{h.g_hi, h.g_lo});
    float E = expf(t.hi);
    return h.K * (__builtin_isinf(E) ? E : __builtin_fmaf(E, t.lo, E));
}

// Erlang(k, rate): the exponentials of f and S cancel,
//   h = rate / sum_{j<k} (k-1)!/j! y^(k-1-j),   y = 1/(rate tau),
// evaluated by Horner from the innermost term (all terms positive).
__device__ __forceinline__ float hazard_erlang(const HazardDev& h, float x)
{
    if (h.k <= 1) return h.K;
    ff xr = two_prod(h.x_hi, x);
    float xx = xr.hi + __builtin_fmaf(h.x_lo, x, xr.lo);
    if (!(xx > 0.0f)) return 0.0f;
    float y = rcp(xx);
    float R = 1.0f;
    for (int m = 1; m <= h.k - 1; ++m) R = __builtin_fmaf((float)m * y, R, 1.0f);
    return h.K * rcp(R);
}

__device__ __forceinline__ float hazard(const HazardDev& h, float x)
{
    switch (h.kind) {
    case fsi::K_LN: return hazard_lognormal(h, x);
    case fsi::K_WB: return hazard_weibull(h, x);
    case fsi::K_ERL: return hazard_erlang(h, x);
    default: return h.K;
    }
}

// ---------------------------------------------------------------------------
// Shedding profiles s(x) (Eq. (infectivity)); parameters as in ShedDev.
// Exponents are formed in float-float and exp(e_hi + e_lo) is taken as
// exp(e_hi) (1 + e_lo).
// ---------------------------------------------------------------------------
using fsi::ShedDev;

__device__ __forceinline__ float exp_ff(ff e)
{
    const float E = expf(e.hi);
    return __builtin_isinf(E) ? E : __builtin_fmaf(E, e.lo, E);
}

__device__ __forceinline__ float shed_density(const ShedDev& s, float x)
{
    if (!(x > 0.0f)) return s.s0;
    const HazardDev& h = s.hz;
    switch (h.kind) {
    case fsi::K_LN: {
        const ff t = ff_add(log_ff(x), ff{h.c_hi, h.c_lo});
        const ff z = ff_mul(t, ff{h.g_hi, h.g_lo});
        const ff sq = two_prod(z.hi, z.hi);
        const float lo = __builtin_fmaf(2.0f * z.hi, z.lo, sq.lo);
        return h.K * exp_ff(ff{-sq.hi, -lo}) / x;
    }
    case fsi::K_WB: {
        const ff t = ff_add(log_ff(x), ff{h.c_hi, h.c_lo});
        const ff a = ff_mul(t, ff{h.g_hi, h.g_lo});
        const float w = exp_ff(ff_mul(t, ff{s.m_hi, s.m_lo})); // (tau / scale)^shape
        return h.K * exp_ff(ff_add(a, ff{-w, 0.0f}));
    }
    case fsi::K_ERL: {
        const ff p = two_prod(h.x_hi, x);
        const ff y = quick_two_sum(p.hi, __builtin_fmaf(h.x_lo, x, p.lo));
        const ff L = ff_add(log_ff(y.hi), ff{y.lo / y.hi, 0.0f});
        ff e = ff_mul(L, ff{(float)(h.k - 1), 0.0f});
        e = ff_add(e, ff{-y.hi, -y.lo});
        e = ff_add(e, ff{-s.lf_hi, -s.lf_lo});
        return h.K * exp_ff(e);
    }
    default: {
        const ff p = two_prod(h.x_hi, x);
        return h.K * exp_ff(ff{-p.hi, -__builtin_fmaf(h.x_lo, x, p.lo)});
    }
    }
}

__device__ __forceinline__ float shed(const ShedDev& s, float x)
{
    return s.density ? shed_density(s, x) : hazard(s.hz, x);
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds of
//   (c0,c1,c2,c3) <- (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0))
// with the key advanced by the Weyl increments between rounds.
// ---------------------------------------------------------------------------
constexpr uint32_t PH_M0 = 0xD2511F53u;
constexpr uint32_t PH_M1 = 0xCD9E8D57u;
constexpr uint32_t PH_W0 = 0x9E3779B9u;
constexpr uint32_t PH_W1 = 0xBB67AE85u;

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        // one 32x32 -> 64-bit product per multiplier (a single v_mad_u64_u32)
        const unsigned long long p0 = (unsigned long long)PH_M0 * c.x;
        const unsigned long long p1 = (unsigned long long)PH_M1 * c.z;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
        k0 += PH_W0;
        k1 += PH_W1;
    }
    return c;
}

// The step's uniform: word 0 at counter (node, step, replica, 0), top 24 bits.
__device__ __forceinline__ float step_uniform(uint32_t node, uint32_t step, uint32_t replica,
                                              uint32_t k0, uint32_t k1)
{
    uint4 w = philox4x32_10(make_uint4(node, step, replica, 0u), k0, k1);
    return (float)(w.x >> 8) * 0x1p-24f;
}

} // namespace fsd
