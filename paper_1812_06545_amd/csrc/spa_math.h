// Device arithmetic of the sum-product check rule, shared by every kernel so
// that all decoding paths round identically.
//
// Check rule (arxiv 1812.06545, Section I: belief propagation / sum-product;
// Algorithm 1, Loop 2): r_mn = 2 atanh(prod_{n' != n} tanh(q_mn'/2)).
// Signs and magnitudes separate: sign = prod sign(q_mn'), and the magnitude
// follows from the |q|.  Each kernel evaluates a row as two halves with
// prefix and suffix combinations (never "total minus self" or a division,
// which cancel or fail when one term dominates or is zero), through an
// arithmetic type A that supplies:
//     Term  term(q)        per-edge quantity, q's sign in its sign bit;
//     Acc   identity()     the empty combination;
//     Acc   add(Acc, Term) combination grown by one edge;
//     Acc   merge(Acc, Acc) combination of two disjoint edge sets;
//     Acc   seed(Acc)      a combination in the form message() takes it
//                          (FP32: its product doubled), applied once per
//                          half row to the other half's combination;
//     T     message(Acc)   |r| from the seeded combination of the other
//                          edges, clamped to R_MAX.
//
// FP32 (base-2 LLR units: every LLR is multiplied by log2(e) on entry and by
// ln 2 on exit) uses the product form directly.  An edge carries
//     t = tanh(|q| ln2 / 2) = (1 - e) / (1 + e)   and   u = 1 - t = 2e / (1 + e),
// with e = 2^-|q|, both to relative accuracy (1 - e for small |q| comes from a
// short series instead of the subtraction).  A combination carries the
// product P = prod t and its complement Q = 1 - P, the latter grown by
// a (+) b = a + b - ab = 1 - (1 - a)(1 - b), so that Q stays accurate when P is
// close to 1 (confident rows) just as P does when it is small.  The message
// is 2 atanh(P) = log2((1 + P) / Q) = log2(1 + 2P / Q), with the rounding
// error of w = fl(1 + z) added back (c = (1 - w) + z is exact while w <
// 2^24, and at most 2^-24 for z < 1; it is clamped to that bound, which
// leaves it exact where it matters, weak messages, and harmless elsewhere).
// The factor 2 of 2P rides on the seed of each half's backward pass, so it
// costs one operation per half row, not per edge.  Per edge: exp2 and one
// reciprocal forward, one reciprocal and log2 back.
//
// FP64 uses the equivalent phi form with libm-quality exp / expm1 / log1p:
//     phi(x) = -ln tanh(x/2) = log1p(2 e^-x / (1 - e^-x)),
// prod tanh(|q|/2) = exp(-sum phi(|q|)) and 2 atanh(exp(-S)) = phi(S), so a
// combination is the sum S of phi(|q|) and the message is phi(S).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ldpc {

struct ArithF32 {
    using T = float;
    static constexpr float kIn = 1.44269504088896341f;   // natural LLR -> internal (log2 e)
    static constexpr float kOut = 0.693147180559945309f; // internal -> natural LLR (ln 2)
    static constexpr float kRmax = 28.8539008177792681f; // R_MAX = 20 in internal units

    struct Term {
        float t;  // tanh(|q| ln2 / 2), with q's sign bit
        float u;  // 1 - |t|
    };
    struct Acc {
        float P;  // product of the |t|
        float Q;  // 1 - P, formed from the u
    };
    // a (+) b = 1 - (1 - a)(1 - b) for a, b in [0, 1]
    __device__ static __forceinline__ float oplus(float a, float b) { return __builtin_fmaf(-a, b, a + b); }

    __device__ static __forceinline__ Acc identity() { return Acc{1.0f, 0.0f}; }
    __device__ static __forceinline__ Term term(float q)
    {
        const float x = __builtin_fabsf(q);
        const float e = __builtin_amdgcn_exp2f(-x);
        // d = 1 - 2^-x.  For small x the subtraction loses relative accuracy,
        // which t (a small factor of P, the size of a weak message) needs;
        // there d comes from the Taylor series of -expm1(-x ln 2) (5 terms:
        // truncation below 1e-8 relative for x < 1/8).
        // Everything is formed at half scale, d/2 and 2/(1 + e), which
        // scales by powers of two only (the same roundings) and saves the
        // doubling of e in u = 2e/(1 + e).
        float p = __builtin_fmaf(-x, 0.5f * 1.33335581e-3f, 0.5f * 9.61812911e-3f);  // ln2^5/120, ln2^4/24
        p = __builtin_fmaf(-x, p, 0.5f * 5.55041087e-2f);                             // ln2^3/6
        p = __builtin_fmaf(-x, p, 0.5f * 2.40226507e-1f);                             // ln2^2/2
        p = __builtin_fmaf(-x, p, 0.5f * 6.93147181e-1f);                             // ln2
        const float dh = (x < 0.125f) ? x * p : __builtin_fmaf(e, -0.5f, 0.5f);     // d / 2
        const float ri2 = __builtin_amdgcn_rcpf(__builtin_fmaf(e, 0.5f, 0.5f));     // 2 / (1 + e)
        Term k;
        k.t = mag_with_sign_of(dh * ri2, q);
        k.u = e * ri2;
        return k;
    }
    __device__ static __forceinline__ Acc add(Acc a, const Term &k)
    {
        return Acc{a.P * __builtin_fabsf(k.t), oplus(a.Q, k.u)};
    }
    __device__ static __forceinline__ Acc merge(Acc a, Acc b) { return Acc{a.P * b.P, oplus(a.Q, b.Q)}; }
    __device__ static __forceinline__ Acc seed(Acc a) { return Acc{a.P + a.P, a.Q}; }
    __device__ static __forceinline__ float message(Acc x)
    {
        // x.P is twice the product (seed).  Q = 0 (a degree-1 row, or every
        // other edge certain) gives z = +inf, w = +inf and log2 = +inf; c is
        // then NaN or a clamp bound, and either way r is not below R_MAX, so
        // the final select (false for NaN) returns R_MAX.  P = 0 forces Q = 1,
        // so z is never 0 * inf.
        const float z = x.P * __builtin_amdgcn_rcpf(x.Q);
        const float w = 1.0f + z;
        const float c = __builtin_amdgcn_fmed3f((1.0f - w) + z, -0x1p-24f, 0x1p-24f);
        const float r = __builtin_fmaf(c, 1.44269504088896341f, __builtin_amdgcn_logf(w));
        return r < kRmax ? r : kRmax;
    }
    __device__ static __forceinline__ uint32_t term_sign(const Term &k) { return sign_bit(k.t); }

    // The fused kernel parks a term's t in the edge's message slot and keeps u
    // in a register; kDummyParked is the parked part of a dummy edge's term
    // (q = +inf: t = 1, u = 0).
    using Keep = float;
    static constexpr float kDummyParked = 1.0f;
    __device__ static __forceinline__ float park(const Term &k) { return k.t; }
    __device__ static __forceinline__ Keep keep(const Term &k) { return k.u; }
    __device__ static __forceinline__ Term unpark(float parked, Keep kept) { return Term{parked, kept}; }

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

    using Term = double;  // phi(|q|) with q's sign bit
    using Acc = double;   // sum of phi(|q|)
    __device__ static __forceinline__ Acc identity() { return 0.0; }
    __device__ static __forceinline__ Term term(double q) { return mag_with_sign_of(phi(fabs(q)), q); }
    __device__ static __forceinline__ Acc add(Acc a, Term k) { return a + fabs(k); }
    __device__ static __forceinline__ Acc merge(Acc a, Acc b) { return a + b; }
    __device__ static __forceinline__ Acc seed(Acc a) { return a; }
    __device__ static __forceinline__ double message(Acc x)
    {
        const double r = phi(x);
        return r < kRmax ? r : kRmax;
    }
    __device__ static __forceinline__ uint32_t term_sign(Term k) { return sign_bit(k); }

    // The fused kernel parks the whole term in the edge's message slot
    // (a dummy edge, q = +inf, has phi = 0).
    struct Keep {};
    static constexpr double kDummyParked = 0.0;
    __device__ static __forceinline__ double park(Term k) { return k; }
    __device__ static __forceinline__ Keep keep(Term) { return Keep{}; }
    __device__ static __forceinline__ Term unpark(double parked, Keep) { return parked; }
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

// Exclusive combinations of one check row.  The row's d edges are split at
// h = ceil(d/2) into halves H0 = [0, h) and H1 = [h, d); for edge k in half
// H, with p_k the combination of the earlier edges of H (left to right),
// C_other the combination of the other half (left to right) and s_k the
// combination seed(C_other) grown by the later edges of H (right to left),
//     excl_k = merge(p_k, s_k).
// Fixing the order lets the fused kernel spread a row over two lanes (one
// half each, exchanging C and the sign) while the streaming kernels evaluate
// the same expression in one lane, bit for bit.

// Layered rows (Section II, Algorithm 2; both layered paths) split each half
// once more, into quarters Q0 = [0, q1), Q1 = [q1, h), Q2 = [h, q3) and
// Q3 = [q3, d), with h = ceil(d/2), q1 = ceil(h/2), q3 = h + ceil((d - h)/2).
// For edge k in Qi, excl_k = merge(p_k, s_k) as above, with p_k the
// combination of the earlier edges of Qi and s_k = seed(O_i) grown by its
// later edges, where O_i combines the other three quarters (C_j, each left
// to right) in this fixed association:
//     O_0 = merge(C_1, merge(C_2, C_3))    O_1 = merge(C_0, merge(C_2, C_3))
//     O_2 = merge(C_3, merge(C_0, C_1))    O_3 = merge(C_2, merge(C_0, C_1))
// merge is commutative bit for bit (a product, and a (+) b, whose fused
// multiply-add forms the exact product either way) but not associative.  The
// fused kernel spreads a layered row over four lanes, one quarter each, which
// halves the serial length of a layer step; the streaming layer kernel
// evaluates the same expressions in one lane.
struct Quarters {
    int q1, h, q3;
};
__host__ __device__ constexpr Quarters quarters(int d)
{
    return Quarters{((d + 1) / 2 + 1) / 2, (d + 1) / 2, (d + 1) / 2 + (d - (d + 1) / 2 + 1) / 2};
}
__host__ __device__ constexpr int quarter_of(const Quarters &q, int k)
{
    return k < q.q1 ? 0 : k < q.h ? 1 : k < q.q3 ? 2 : 3;
}

// seed(O_i) for the four quarters from their combinations C.
template <class A>
__device__ __forceinline__ void quarter_seeds(const typename A::Acc C[4], typename A::Acc S[4])
{
    const typename A::Acc c01 = A::merge(C[0], C[1]), c23 = A::merge(C[2], C[3]);
    S[0] = A::seed(A::merge(C[1], c23));
    S[1] = A::seed(A::merge(C[0], c23));
    S[2] = A::seed(A::merge(C[3], c01));
    S[3] = A::seed(A::merge(C[2], c01));
}

// Forward step for an edge with incoming message q: its term a_k, p_k = the
// half's running combination, which then grows by a_k.
template <class A>
__device__ __forceinline__ void check_forward(typename A::T q, typename A::Term &a_k, typename A::Acc &p_k,
                                              typename A::Acc &acc, uint32_t &sign)
{
    a_k = A::term(q);
    p_k = acc;
    acc = A::add(acc, a_k);
    sign ^= A::sign_bit(q);
}

// Backward step: outgoing message of an edge from its term, p_k, the half's
// running suffix s (started at seed(C_other); it then grows by this edge) and
// the row's total sign.
template <class A>
__device__ __forceinline__ typename A::T check_backward(const typename A::Term &a_k, const typename A::Acc &p_k,
                                                        typename A::Acc &s, uint32_t sign_total)
{
    const typename A::Acc ex = A::merge(p_k, s);
    s = A::add(s, a_k);
    return A::with_sign(A::message(ex), sign_total ^ A::term_sign(a_k));
}

}  // namespace ldpc
