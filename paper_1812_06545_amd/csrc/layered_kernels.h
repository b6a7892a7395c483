// Device code of the layered schedule on the streaming layout (the same
// chunked frame-interleaved arrays as the flooding path: r per edge and the
// posterior L per variable, [chunk][edge or variable][64 frames]).
//
// Layered decoding (arxiv 1812.06545, Section II, Algorithm 2): check rows are
// visited one at a time in ascending order and each row's new messages update
// the posteriors of its variables at once:
//     q_mn = L_n - r_mn ;  r_mn = check rule over q_m. ;  L_n = q_mn + r_mn.
// Consecutive rows that share no variable commute, so a maximal run of them
// (a layer: a block-row of a QC code) is one launch, one wavefront per row and
// 64 frames; within a layer every L_n is read and written by one row only.
// The check rule is the flooding path's arithmetic with the layered
// combination order (four quarters, spa_math.h), the one the fused kernel's
// layered jobs use, so both layered paths give the same messages for the
// same q.
#pragma once

#include "flood_kernels.h"

namespace ldpc {
namespace layered {

using flood::kWaves;
using flood::ld_lane;
using flood::ld_lane_nt;
using flood::map_block;
using flood::st_lane;
using flood::st_lane_nt;
using flood::chunk_rsrc;
using flood::ld_gather;
using flood::st_scatter;

// One check row of compile-time degree D: all loads first, then the forward
// and backward sweeps; each new message and its posterior are stored as soon
// as they are formed.  FIRST (the first pass) reads no old messages: they
// are all 0.  Messages stream with non-temporal accesses; posteriors, which
// later layers gather, stay cached.
template <class A, int D, bool FIRST>
__device__ __forceinline__ void layer_row(const int32_t *__restrict__ cols, typename A::T *__restrict__ L, int32_t n,
                                          typename A::T *__restrict__ Rrow, uint32_t off)
{
    using T = typename A::T;
    constexpr bool kBuf = std::is_same<T, float>::value;  // posterior gathers and scatters by buffer access
    constexpr Quarters Q = quarters(D);
    const __amdgpu_buffer_rsrc_t rsrc = chunk_rsrc(L, n);
    T q[D], rv[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        if constexpr (kBuf)
            q[k] = ld_gather(rsrc, off, cols[k], T(0));
        else
            q[k] = ld_lane(L + cols[k] * kChunk, off);
        rv[k] = FIRST ? T(0) : ld_lane_nt(Rrow + k * kChunk, off);
    }
    typename A::Term a[D];
    typename A::Acc p[D];
    typename A::Acc acc[4] = {A::identity(), A::identity(), A::identity(), A::identity()};
    uint32_t sign = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        if (!FIRST)
            q[k] = q[k] - rv[k];
        check_forward<A>(q[k], a[k], p[k], acc[quarter_of(Q, k)], sign);
    }
    typename A::Acc sx[4];
    quarter_seeds<A>(acc, sx);
#pragma unroll
    for (int k = D - 1; k >= 0; --k) {
        const T r = check_backward<A>(a[k], p[k], sx[quarter_of(Q, k)], sign);
        st_lane_nt(Rrow + k * kChunk, off, r);
        if constexpr (kBuf)
            st_scatter(rsrc, off, cols[k], q[k] + r);
        else
            st_lane(L + cols[k] * kChunk, off, q[k] + r);
    }
}

// The same row for a run-time degree d <= DMAX (guarded loops; FP64 and
// degrees above the largest exact bucket).
template <class A, int DMAX, bool FIRST>
__device__ __forceinline__ void layer_row_guarded(const int32_t *__restrict__ cols, int d,
                                                  typename A::T *__restrict__ L, typename A::T *__restrict__ Rrow,
                                                  uint32_t off)
{
    using T = typename A::T;
    const Quarters Q = quarters(d);  // d is the wavefront's row's: the branches below are uniform
    T q[DMAX], rv[DMAX];
#pragma unroll
    for (int k = 0; k < DMAX; ++k) {
        if (k < d) {
            q[k] = ld_lane(L + cols[k] * kChunk, off);
            rv[k] = FIRST ? T(0) : ld_lane_nt(Rrow + k * kChunk, off);
        }
    }
    typename A::Term a[DMAX];
    typename A::Acc p[DMAX];
    // One running combination, closed into C[i] at each quarter boundary
    // (quarters may be empty: their combination is the identity).
    typename A::Acc C[4], cur = A::identity();
    uint32_t sign = 0;
#pragma unroll
    for (int k = 0; k < DMAX; ++k) {
        if (k < d) {
            if (k == Q.q1) {
                C[0] = cur;
                cur = A::identity();
            }
            if (k == Q.h) {
                C[1] = cur;
                cur = A::identity();
            }
            if (k == Q.q3) {
                C[2] = cur;
                cur = A::identity();
            }
            if (!FIRST)
                q[k] = q[k] - rv[k];
            check_forward<A>(q[k], a[k], p[k], cur, sign);
        }
    }
    if (Q.q1 >= d) {
        C[0] = cur;
        cur = A::identity();
    }
    if (Q.h >= d) {
        C[1] = cur;
        cur = A::identity();
    }
    if (Q.q3 >= d) {
        C[2] = cur;
        cur = A::identity();
    }
    C[3] = cur;
    typename A::Acc sx[4];
    quarter_seeds<A>(C, sx);
    typename A::Acc sq = sx[3];  // the running suffix, switched to each quarter's seed at its last edge
#pragma unroll
    for (int k = DMAX - 1; k >= 0; --k) {
        if (k < d) {
            if (k == Q.q3 - 1)
                sq = sx[2];
            if (k == Q.h - 1)
                sq = sx[1];
            if (k == Q.q1 - 1)
                sq = sx[0];
            const T r = check_backward<A>(a[k], p[k], sq, sign);
            st_lane_nt(Rrow + k * kChunk, off, r);
            st_lane(L + cols[k] * kChunk, off, q[k] + r);
        }
    }
}

// Exact-degree dispatch for d in [D, DB] (straight-line body per degree).
template <class A, int D, int DB, bool FIRST>
__device__ __forceinline__ void layer_row_exact(int d, const int32_t *__restrict__ cols, typename A::T *__restrict__ L,
                                                int32_t n, typename A::T *__restrict__ Rrow, uint32_t off)
{
    if constexpr (D < DB) {
        if (d == D)
            layer_row<A, D, FIRST>(cols, L, n, Rrow, off);
        else
            layer_row_exact<A, D + 1, DB, FIRST>(d, cols, L, n, Rrow, off);
    } else {
        layer_row<A, DB, FIRST>(cols, L, n, Rrow, off);
    }
}

// One layer: rows [row0, row0 + rows), one wavefront = one row x 64 frames.
// Frames already stopped (done >= 0) are left untouched.
template <class A, int DB, bool EXACT, bool FIRST, bool ES>
__global__ __launch_bounds__(256) void k_layer(const int32_t *__restrict__ row_ptr,
                                               const int32_t *__restrict__ col_idx, int32_t row0, int32_t rows,
                                               int32_t n, int64_t E, int32_t groups, int32_t nchunk,
                                               typename A::T *__restrict__ R, typename A::T *__restrict__ L,
                                               const int32_t *__restrict__ done)
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
    if (ES && done[f] >= 0)
        return;
    const uint32_t off = static_cast<uint32_t>(lane) * static_cast<uint32_t>(sizeof(T));
    const int32_t e0 = row_ptr[row];
    const int32_t d = __builtin_amdgcn_readfirstlane(row_ptr[row + 1] - e0);
    T *Rrow = R + (static_cast<int64_t>(chunk) * E + e0) * kChunk;
    T *Lc = L + static_cast<int64_t>(chunk) * n * kChunk;
    if (d > 0) {
        if constexpr (EXACT)
            layer_row_exact<A, 1, DB, FIRST>(d, col_idx + e0, Lc, n, Rrow, off);
        else
            layer_row_guarded<A, DB, FIRST>(col_idx + e0, d, Lc, Rrow, off);
    }
}

// One row of a layer spread over the four wavefronts of a workgroup, one
// quarter of the row each (the layered combination order of spa_math.h),
// 64 frames per wavefront: a layer launch then has four times the
// wavefronts, each with a quarter of the work, which evens out the launch's
// last round of resident wavefronts.  Each wavefront forms its quarter's
// combination, the four exchange them through LDS, and each finishes its
// quarter with the seed of the other three in the fixed association: the
// same expressions as layer_row in one lane, bit for bit.  The quarter body
// has DQ slots; slots past the quarter's length are skipped by a branch that
// is uniform across the wavefront (the row is the wavefront's).  FP32 rows of
// degree <= 4 DQ.
template <class A, int DQ, bool FIRST, bool ES>
__global__ __launch_bounds__(256) void k_layer_q(const int32_t *__restrict__ row_ptr,
                                                 const int32_t *__restrict__ col_idx, int32_t row0, int32_t rows,
                                                 int32_t n, int64_t E, int32_t nchunk, typename A::T *__restrict__ R,
                                                 typename A::T *__restrict__ L, const int32_t *__restrict__ done)
{
    using T = typename A::T;
    using Acc = typename A::Acc;
    __shared__ Acc sC[4][kChunk];
    __shared__ uint32_t sS[4][kChunk];
    const int part = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
    const int lane = static_cast<int>(threadIdx.x & 63);
    int group, chunk;
    map_block(static_cast<int>(blockIdx.x), rows, nchunk, group, chunk);
    if (ES && flood::chunk_active(done, nchunk, chunk) == 0)
        return;  // the whole workgroup (one chunk), before any barrier
    const uint32_t f = static_cast<uint32_t>(chunk) * 64u + static_cast<uint32_t>(lane);
    const bool live = !ES || done[f] < 0;  // a stopped frame's lanes compute but store nothing
    const uint32_t off = static_cast<uint32_t>(lane) * static_cast<uint32_t>(sizeof(T));
    const int row = row0 + group;
    const int32_t e0 = row_ptr[row];
    const int32_t d = __builtin_amdgcn_readfirstlane(row_ptr[row + 1] - e0);
    const Quarters Q = quarters(d);
    const int32_t k0 = part == 0 ? 0 : part == 1 ? Q.q1 : part == 2 ? Q.h : Q.q3;
    const int32_t dq = (part == 0 ? Q.q1 : part == 1 ? Q.h : part == 2 ? Q.q3 : d) - k0;
    const int32_t *cols = col_idx + e0 + k0;
    T *Rq = R + (static_cast<int64_t>(chunk) * E + e0 + k0) * kChunk;
    T *Lc = L + static_cast<int64_t>(chunk) * n * kChunk;
    const __amdgpu_buffer_rsrc_t rsrc = chunk_rsrc(Lc, n);
    T q[DQ], rv[DQ];
#pragma unroll
    for (int k = 0; k < DQ; ++k) {
        if (k < dq) {
            q[k] = ld_gather(rsrc, off, cols[k], T(0));
            rv[k] = FIRST ? T(0) : ld_lane_nt(Rq + k * kChunk, off);
        }
    }
    typename A::Term a[DQ];
    Acc p[DQ];
    Acc acc = A::identity();
    uint32_t sign = 0;
#pragma unroll
    for (int k = 0; k < DQ; ++k) {
        if (k < dq) {
            if (!FIRST)
                q[k] = q[k] - rv[k];
            check_forward<A>(q[k], a[k], p[k], acc, sign);
        }
    }
    sC[part][lane] = acc;
    sS[part][lane] = sign;
    __syncthreads();
    const Acc C0 = sC[0][lane], C1 = sC[1][lane], C2 = sC[2][lane], C3 = sC[3][lane];
    const uint32_t sign_total = sS[0][lane] ^ sS[1][lane] ^ sS[2][lane] ^ sS[3][lane];
    Acc other;
    if (part == 0)
        other = A::merge(C1, A::merge(C2, C3));
    else if (part == 1)
        other = A::merge(C0, A::merge(C2, C3));
    else if (part == 2)
        other = A::merge(C3, A::merge(C0, C1));
    else
        other = A::merge(C2, A::merge(C0, C1));
    Acc sx = A::seed(other);
#pragma unroll
    for (int k = DQ - 1; k >= 0; --k) {
        if (k < dq) {
            const T r = check_backward<A>(a[k], p[k], sx, sign_total);
            if (live) {
                st_lane_nt(Rq + k * kChunk, off, r);
                st_scatter(rsrc, off, cols[k], q[k] + r);
            }
        }
    }
}

}  // namespace layered

// Arguments of one layer launch.
template <class A>
struct LayerArgs {
    const int32_t *row_ptr;
    const int32_t *col_idx;
    int32_t row0, rows, n;
    int64_t E;
    int32_t groups, nchunk;
    typename A::T *R;
    typename A::T *L;
    const int32_t *done;
};

// Launcher of the layer kernel for rows of degree <= DB; each (dtype, bucket)
// is defined in its own translation unit.
template <class A, int DB, bool EXACT>
void launch_layer_bucket(const LayerArgs<A> &a, bool first, bool es, dim3 grid, hipStream_t s);

#define LDPC_LAYER_LAUNCH_ONE(A_, DB_, EX_, F_, E_)                                                              \
    do {                                                                                                         \
        ProfScope ps(LDPC_KERNEL_CHECK, s);                                                                      \
        LDPC_LAUNCH(ps, (layered::k_layer<A_, DB_, EX_, F_, E_>), grid, dim3(256), 0, s, a.row_ptr, a.col_idx,  \
                    a.row0, a.rows, a.n, a.E, a.groups, a.nchunk, a.R, a.L, a.done);                            \
    } while (0)

// FP32 exact buckets run the quarter kernel (one row per workgroup of four
// wavefronts, grid rows x chunks); the others the one-wavefront-per-row kernel.
#define LDPC_LAYER_LAUNCH_Q(A_, DB_, F_, E_)                                                                     \
    do {                                                                                                         \
        ProfScope ps(LDPC_KERNEL_CHECK, s);                                                                      \
        LDPC_LAUNCH(ps, (layered::k_layer_q<A_, (DB_) / 4, F_, E_>), qgrid, dim3(256), 0, s, a.row_ptr,          \
                    a.col_idx, a.row0, a.rows, a.n, a.E, a.nchunk, a.R, a.L, a.done);                            \
    } while (0)

#define LDPC_DEFINE_LAYER_BUCKET(A_, DB_, EX_)                                                                  \
    template <>                                                                                                 \
    void launch_layer_bucket<A_, DB_, EX_>(const LayerArgs<A_> &a, bool first, bool es, dim3 grid,              \
                                           hipStream_t s)                                                       \
    {                                                                                                           \
        if constexpr (EX_ && std::is_same<A_, ArithF32>::value) {                                              \
            const dim3 qgrid(static_cast<unsigned>(a.rows) * static_cast<unsigned>(a.nchunk));                  \
            if (first && es)                                                                                    \
                LDPC_LAYER_LAUNCH_Q(A_, DB_, true, true);                                                       \
            else if (first)                                                                                     \
                LDPC_LAYER_LAUNCH_Q(A_, DB_, true, false);                                                      \
            else if (es)                                                                                        \
                LDPC_LAYER_LAUNCH_Q(A_, DB_, false, true);                                                      \
            else                                                                                                \
                LDPC_LAYER_LAUNCH_Q(A_, DB_, false, false);                                                     \
        } else {                                                                                                \
            if (first && es)                                                                                    \
                LDPC_LAYER_LAUNCH_ONE(A_, DB_, EX_, true, true);                                                \
            else if (first)                                                                                     \
                LDPC_LAYER_LAUNCH_ONE(A_, DB_, EX_, true, false);                                               \
            else if (es)                                                                                        \
                LDPC_LAYER_LAUNCH_ONE(A_, DB_, EX_, false, true);                                               \
            else                                                                                                \
                LDPC_LAYER_LAUNCH_ONE(A_, DB_, EX_, false, false);                                              \
        }                                                                                                       \
    }

}  // namespace ldpc
