// Device code of the min-sum check rule on the streaming layout, for both
// schedules (the same arrays and launch shapes as the sum-product kernels:
// one wavefront = one check row x 64 frames).
//
// Min-sum (arxiv 1812.06545, Section II, the rule Algorithm 1 is named
// after): r_mn = prod_{n' != n} sgn(q_mn') * min_{n' != n} |q_mn'|, here with
// |r| = max(scale * min - offset, 0), then the clamp to R_MAX.  A row keeps
// its smallest and second-smallest magnitude, the position of the smallest
// and the sign product; every message is then one select.  Minima are exact
// in any order, so every path (plain, layered, fused) gives the same
// messages for the same q.  sgn(0) = +1 (q < 0 decides the sign), as in the
// reading of the hard decision.  Offsets arrive in the kernel's units
// (natural LLR x kIn).
#pragma once

#include "flood_kernels.h"

namespace ldpc {

// Running minimum state of one row (or half row).
template <class T>
struct MinState {
    T m1, m2;       // smallest and second-smallest |q|
    int32_t idx;    // position of m1 in the row (first of equals)
    uint32_t neg;   // parity of the negative q's
};

template <class T>
__device__ __forceinline__ void min_init(MinState<T> &s)
{
    s.m1 = T(__builtin_huge_val());
    s.m2 = T(__builtin_huge_val());
    s.idx = -1;
    s.neg = 0;
}

template <class T>
__device__ __forceinline__ void min_add(MinState<T> &s, T q, int32_t k)
{
    const T a = fabs(q);
    const bool lower = a < s.m1;
    s.m2 = lower ? s.m1 : (a < s.m2 ? a : s.m2);
    s.idx = lower ? k : s.idx;
    s.m1 = lower ? a : s.m1;
    s.neg ^= static_cast<uint32_t>(q < T(0));
}

// Merge of two halves' states (the partner's is `o`); the first half's
// positions precede the second's, so ties keep the first half's position.
template <class T>
__device__ __forceinline__ void min_merge(MinState<T> &s, T o_m1, T o_m2, int32_t o_idx, uint32_t o_neg)
{
    const bool other_lower = o_m1 < s.m1;
    const T hi = other_lower ? s.m1 : o_m1;
    const T m2 = s.m2 < o_m2 ? s.m2 : o_m2;
    s.m2 = hi < m2 ? hi : m2;
    s.idx = other_lower ? o_idx : s.idx;
    s.m1 = other_lower ? o_m1 : s.m1;
    s.neg ^= o_neg;
}

// Outgoing message of edge k with incoming q_k.
template <class A>
__device__ __forceinline__ typename A::T min_message(const MinState<typename A::T> &s, typename A::T q, int32_t k,
                                                     typename A::T scale, typename A::T offset)
{
    using T = typename A::T;
    const T m = k == s.idx ? s.m2 : s.m1;
    T mag = scale * m - offset;
    mag = mag > T(0) ? mag : T(0);
    mag = mag < T(A::kRmax) ? mag : T(A::kRmax);
    const uint32_t neg = s.neg ^ static_cast<uint32_t>(q < T(0));
    return neg ? -mag : mag;
}

namespace minsum {

using flood::kWaves;
using flood::ld_lane;
using flood::ld_lane_nt;
using flood::map_block;
using flood::st_lane;
using flood::st_lane_nt;

// One row, run-time degree d <= DMAX, all loads first.  LAYERED also writes
// the posteriors L = q + r_new; otherwise ES folds the parity of the previous
// decision [L < 0] into `parity`.
template <class A, int DMAX, bool FIRST, bool ES, bool LAYERED>
__device__ __forceinline__ void ms_row(const int32_t *__restrict__ cols, int d, typename A::T *__restrict__ L,
                                       typename A::T *__restrict__ Rrow, uint32_t off, typename A::T scale,
                                       typename A::T offset, uint32_t &parity)
{
    using T = typename A::T;
    T q[DMAX], rv[DMAX];
#pragma unroll
    for (int k = 0; k < DMAX; ++k) {
        if (k < d) {
            q[k] = ld_lane(L + cols[k] * kChunk, off);
            rv[k] = FIRST ? T(0) : ld_lane_nt(Rrow + k * kChunk, off);
        }
    }
    MinState<T> st;
    min_init(st);
#pragma unroll
    for (int k = 0; k < DMAX; ++k) {
        if (k < d) {
            if (ES && !LAYERED)
                parity ^= static_cast<uint32_t>(q[k] < T(0));
            if (!FIRST)
                q[k] = q[k] - rv[k];
            min_add(st, q[k], k);
        }
    }
#pragma unroll
    for (int k = 0; k < DMAX; ++k) {
        if (k < d) {
            const T r = min_message<A>(st, q[k], k, scale, offset);
            st_lane_nt(Rrow + k * kChunk, off, r);
            if (LAYERED)
                st_lane(L + cols[k] * kChunk, off, q[k] + r);
        }
    }
}

// Flooding check kernel with the min-sum rule (Loop 2); the variable kernel
// is the sum-product path's.
template <class A, int DB, bool FIRST, bool ES>
__global__ __launch_bounds__(256) void k_check_ms(const int32_t *__restrict__ row_ptr,
                                                  const int32_t *__restrict__ col_idx, int32_t m, int32_t n, int64_t E,
                                                  int32_t groups, int32_t nchunk, typename A::T *__restrict__ R,
                                                  const typename A::T *__restrict__ L, const int32_t *__restrict__ done,
                                                  int32_t *__restrict__ unsat, typename A::T scale,
                                                  typename A::T offset)
{
    using T = typename A::T;
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
    const int lane = static_cast<int>(threadIdx.x & 63);
    int group, chunk;
    map_block(static_cast<int>(blockIdx.x), groups, nchunk, group, chunk);
    const int row = group * kWaves + wave;
    if (row >= m)
        return;
    if (ES && flood::chunk_active(done, nchunk, chunk) == 0)  // as k_check: stopped chunks skipped, stopped lanes harmless
        return;
    const uint32_t f = static_cast<uint32_t>(chunk) * 64u + static_cast<uint32_t>(lane);
    const uint32_t off = static_cast<uint32_t>(lane) * static_cast<uint32_t>(sizeof(T));
    const int32_t e0 = row_ptr[row];
    const int32_t d = __builtin_amdgcn_readfirstlane(row_ptr[row + 1] - e0);
    uint32_t parity = 0;
    T *Rrow = R + (static_cast<int64_t>(chunk) * E + e0) * kChunk;
    T *Lc = const_cast<T *>(L) + static_cast<int64_t>(chunk) * n * kChunk;
    if (d > 0)
        ms_row<A, DB, FIRST, ES, false>(col_idx + e0, d, Lc, Rrow, off, scale, offset, parity);
    if (ES && parity)
        unsat[f] = 1;
}

// Layer kernel with the min-sum rule: rows [row0, row0 + rows).
template <class A, int DB, bool FIRST, bool ES>
__global__ __launch_bounds__(256) void k_layer_ms(const int32_t *__restrict__ row_ptr,
                                                  const int32_t *__restrict__ col_idx, int32_t row0, int32_t rows,
                                                  int32_t n, int64_t E, int32_t groups, int32_t nchunk,
                                                  typename A::T *__restrict__ R, typename A::T *__restrict__ L,
                                                  const int32_t *__restrict__ done, typename A::T scale,
                                                  typename A::T offset)
{
    using T = typename A::T;
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
    const int lane = static_cast<int>(threadIdx.x & 63);
    int group, chunk;
    map_block(static_cast<int>(blockIdx.x), groups, nchunk, group, chunk);
    const int slot = group * kWaves + wave;
    if (slot >= rows)
        return;
    const int row = row0 + slot;
    if (ES && flood::chunk_active(done, nchunk, chunk) == 0)
        return;
    const uint32_t f = static_cast<uint32_t>(chunk) * 64u + static_cast<uint32_t>(lane);
    if (ES && done[f] >= 0)  // the layer updates L in place: a stopped frame is left untouched
        return;
    const uint32_t off = static_cast<uint32_t>(lane) * static_cast<uint32_t>(sizeof(T));
    const int32_t e0 = row_ptr[row];
    const int32_t d = __builtin_amdgcn_readfirstlane(row_ptr[row + 1] - e0);
    T *Rrow = R + (static_cast<int64_t>(chunk) * E + e0) * kChunk;
    T *Lc = L + static_cast<int64_t>(chunk) * n * kChunk;
    uint32_t unused = 0;
    if (d > 0)
        ms_row<A, DB, FIRST, false, true>(col_idx + e0, d, Lc, Rrow, off, scale, offset, unused);
}

}  // namespace minsum

// Arguments of one min-sum launch (flooding check or layer).
template <class A>
struct MinSumArgs {
    const int32_t *row_ptr;
    const int32_t *col_idx;
    int32_t row0, rows, m, n;
    int64_t E;
    int32_t groups, nchunk;
    typename A::T *R;
    typename A::T *L;
    const int32_t *done;
    int32_t *unsat;
    typename A::T scale, offset;
};

// Launchers for rows of degree <= DB (one definition per dtype and bucket).
template <class A, int DB>
void launch_check_ms_bucket(const MinSumArgs<A> &a, bool first, bool es, dim3 grid, hipStream_t s);
template <class A, int DB>
void launch_layer_ms_bucket(const MinSumArgs<A> &a, bool first, bool es, dim3 grid, hipStream_t s);

#define LDPC_MS_CHECK_ONE(A_, DB_, F_, E_)                                                                        \
    do {                                                                                                         \
        ProfScope ps(LDPC_KERNEL_CHECK, s);                                                                      \
        LDPC_LAUNCH(ps, (minsum::k_check_ms<A_, DB_, F_, E_>), grid, dim3(256), 0, s, a.row_ptr, a.col_idx, a.m,  \
                    a.n, a.E, a.groups, a.nchunk, a.R, a.L, a.done, a.unsat, a.scale, a.offset);                \
    } while (0)

#define LDPC_MS_LAYER_ONE(A_, DB_, F_, E_)                                                                        \
    do {                                                                                                         \
        ProfScope ps(LDPC_KERNEL_CHECK, s);                                                                      \
        LDPC_LAUNCH(ps, (minsum::k_layer_ms<A_, DB_, F_, E_>), grid, dim3(256), 0, s, a.row_ptr, a.col_idx,     \
                    a.row0, a.rows, a.n, a.E, a.groups, a.nchunk, a.R, a.L, a.done, a.scale, a.offset);        \
    } while (0)

#define LDPC_DEFINE_MS_BUCKET(A_, DB_)                                                                           \
    template <>                                                                                                 \
    void launch_check_ms_bucket<A_, DB_>(const MinSumArgs<A_> &a, bool first, bool es, dim3 grid, hipStream_t s) \
    {                                                                                                           \
        if (first && es)                                                                                        \
            LDPC_MS_CHECK_ONE(A_, DB_, true, true);                                                             \
        else if (first)                                                                                         \
            LDPC_MS_CHECK_ONE(A_, DB_, true, false);                                                            \
        else if (es)                                                                                            \
            LDPC_MS_CHECK_ONE(A_, DB_, false, true);                                                            \
        else                                                                                                    \
            LDPC_MS_CHECK_ONE(A_, DB_, false, false);                                                           \
    }                                                                                                           \
    template <>                                                                                                 \
    void launch_layer_ms_bucket<A_, DB_>(const MinSumArgs<A_> &a, bool first, bool es, dim3 grid, hipStream_t s) \
    {                                                                                                           \
        if (first && es)                                                                                        \
            LDPC_MS_LAYER_ONE(A_, DB_, true, true);                                                             \
        else if (first)                                                                                         \
            LDPC_MS_LAYER_ONE(A_, DB_, true, false);                                                            \
        else if (es)                                                                                            \
            LDPC_MS_LAYER_ONE(A_, DB_, false, true);                                                            \
        else                                                                                                    \
            LDPC_MS_LAYER_ONE(A_, DB_, false, false);                                                           \
    }

}  // namespace ldpc
