// Device arithmetic of the sum-product check rule, shared by every kernel so
// that all decoding paths round identically.
//
// Check rule (arxiv 1812.06545, Section I: belief propagation / sum-product;
// Algorithm 1, Loop 2): r_mn = 2 atanh(prod_{n' != n} tanh(q_mn'/2)).
// It is evaluated in the equivalent "phi" form: with
//     phi(x) = -ln tanh(x/2) = ln((1 + e^-x) / (1 - e^-x))   (x >= 0),
// prod tanh(|q|/2) = exp(-sum phi(|q|)) and 2 atanh(exp(-S)) = phi(S), so
//     |r_mn| = phi( sum_{n' != n} phi(|q_mn'|) ),  sign = prod_{n' != n} sign(q_mn').
// The exclusive sum is prefix + suffix (never total minus self, which cancels
// catastrophically when one term dominates).
//
// FP32 runs in base-2 LLR units (every LLR multiplied by log2(e) on entry and
// by ln 2 on exit), where phi becomes phi2(x) = log2((1 + 2^-x) / (1 - 2^-x))
// and maps straight onto the hardware exp2 / log2 / reciprocal.  phi2 is
// written as log2(1 + z), z = 2e / (1 - e), e = 2^-x, with the rounding error
// of w = fl(1 + z) added back (c = (1 - w) + z is exact), which keeps the
// result accurate to a few ulp when z is small (x large); for small x the
// denominator 1 - e comes from a short series instead of the subtraction.  FP64 uses the
// natural-log form with libm-quality exp / expm1 / log1p.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ldpc {

struct ArithF32 {
    using T = float;
    static constexpr float kIn = 1.44269504088896341f;   // natural LLR -> internal (log2 e)
    static constexpr float kOut = 0.693147180559945309f; // internal -> natural LLR (ln 2)
    static constexpr float kRmax = 28.8539008177792681f; // R_MAX = 20 in internal units

    __device__ static __forceinline__ float phi(float x)
    {
        const float e = __builtin_amdgcn_exp2f(-x);
        // d = 1 - 2^-x.  For small x the subtraction loses relative accuracy,
        // and phi(S) for a small exclusive sum S is a large, confident message
        // that needs it; there d comes from the Taylor series of
        // -expm1(-x ln 2) (5 terms: truncation below 1e-8 relative for x < 1/8).
        float p = __builtin_fmaf(-x, 1.33335581e-3f, 9.61812911e-3f);   // ln2^5/120, ln2^4/24
        p = __builtin_fmaf(-x, p, 5.55041087e-2f);                       // ln2^3/6
        p = __builtin_fmaf(-x, p, 2.40226507e-1f);                       // ln2^2/2
        p = __builtin_fmaf(-x, p, 6.93147181e-1f);                       // ln2
        const float d = (x < 0.125f) ? x * p : 1.0f - e;
        float z = (e + e) * __builtin_amdgcn_rcpf(d);
        z = __builtin_fminf(z, 0x1p100f);  // x -> 0: keeps the result finite (about 100)
        const float w = 1.0f + z;
        float c = (1.0f - w) + z;
        c = (z < 1.0f) ? c : 0.0f;
        return __builtin_fmaf(c, 1.44269504088896341f, __builtin_amdgcn_logf(w));
    }
    __device__ static __forceinline__ uint32_t sign_bit(float v) { return __float_as_uint(v) >> 31; }
    __device__ static __forceinline__ float with_sign(float mag, uint32_t neg)
    {
        return __uint_as_float(__float_as_uint(mag) | (neg << 31));
    }
    __device__ static __forceinline__ float mag_with_sign_of(float mag, float src)
    {
        return __uint_as_float(__float_as_uint(mag) | (__float_as_uint(src) & 0x80000000u));
    }
};

struct ArithF64 {
    using T = double;
    static constexpr double kIn = 1.0;
    static constexpr double kOut = 1.0;
    static constexpr double kRmax = 20.0;

    __device__ static __forceinline__ double phi(double x)
    {
        const double e = exp(-x);
        const double d = -expm1(-x);
        return log1p((e + e) / d);
    }
    __device__ static __forceinline__ uint32_t sign_bit(double v)
    {
        return static_cast<uint32_t>(static_cast<uint64_t>(__double_as_longlong(v)) >> 63);
    }
    __device__ static __forceinline__ double with_sign(double mag, uint32_t neg)
    {
        return __longlong_as_double(static_cast<long long>(static_cast<uint64_t>(__double_as_longlong(mag)) |
                                                           (static_cast<uint64_t>(neg) << 63)));
    }
    __device__ static __forceinline__ double mag_with_sign_of(double mag, double src)
    {
        const uint64_t s = static_cast<uint64_t>(__double_as_longlong(src)) & 0x8000000000000000ull;
        return __longlong_as_double(static_cast<long long>(static_cast<uint64_t>(__double_as_longlong(mag)) | s));
    }
};

// Exclusive sums of one check row.  The row's d edges are split at
// h = ceil(d/2) into halves H0 = [0, h) and H1 = [h, d); for edge k in half
// H, with p_k the sum of the earlier edges of H (left to right), s_k the sum
// of the later edges of H (right to left) and S_other the total of the other
// half (left to right),
//     excl_k = (p_k + s_k) + S_other.
// Every term is non-negative, so the order costs no accuracy; fixing it lets
// the fused kernel spread a row over two lanes (one half each, exchanging
// S and the sign) while the streaming kernel evaluates the same expression in
// one lane, bit for bit.

// Forward step for an edge with incoming message q: a_k = sign(q) phi(|q|)
// (sign in the sign bit), p_k = the half's running sum, which then grows.
template <class A>
__device__ __forceinline__ void check_forward(typename A::T q, typename A::T &a_k, typename A::T &p_k,
                                              typename A::T &acc, uint32_t &sign)
{
    const typename A::T mag = A::phi(fabs(q));
    a_k = A::mag_with_sign_of(mag, q);
    p_k = acc;
    acc += mag;
    sign ^= A::sign_bit(q);
}

// Backward step: outgoing message of an edge from its a_k, p_k, the half's
// running suffix s (which then grows), the other half's total and the row's
// total sign.
template <class A>
__device__ __forceinline__ typename A::T check_backward(typename A::T a_k, typename A::T p_k, typename A::T &s,
                                                        typename A::T s_other, uint32_t sign_total)
{
    using T = typename A::T;
    const T ex = (p_k + s) + s_other;
    s += fabs(a_k);
    T mag = A::phi(ex);
    mag = mag < A::kRmax ? mag : A::kRmax;
    return A::with_sign(mag, sign_total ^ A::sign_bit(a_k));
}

}  // namespace ldpc
