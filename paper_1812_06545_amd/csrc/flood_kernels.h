// Device code of the plain flooding path: check-node and variable-node
// kernels over the chunked frame-interleaved layout (flood.hip describes the
// layout and the schedule).  Included by the check-kernel translation units (one per
// dtype and degree bucket, compiled in parallel) and by flood.hip.
#pragma once

#include "ldpc_internal.h"
#include "spa_math.h"

namespace ldpc {
namespace flood {

constexpr int kWaves = 4;  // wavefronts (rows or columns) per 256-thread block

// Frame state with early stop: done[f] (f < frames padded to whole chunks)
// is the iteration at which frame f stopped, -1 while it runs; done[Fp + c]
// counts the frames of chunk c still running (written by the variable
// kernel, or by the retire kernel of the layered schedule), so that work on
// a chunk whose frames have all stopped is skipped with one wave-uniform load.
__device__ __forceinline__ int32_t chunk_active(const int32_t *__restrict__ done, int32_t nchunk, int chunk)
{
    return done[nchunk * kChunk + chunk];
}

// Block -> (group of kWaves rows, frame chunk).  Workgroups are dispatched to
// the 8 XCDs round-robin; when the chunk count allows it, XCD x gets chunks
// x, x+8, ... and sweeps every row of one chunk before the next, so that the
// chunk's posterior slice (n x 64 values) stays resident in that XCD's L2
// while all rows gather from it.
__device__ __forceinline__ void map_block(int b, int groups, int nchunk, int &group, int &chunk)
{
    if ((nchunk & 7) == 0) {
        const int xcd = b & 7, j = b >> 3;
        chunk = (j / groups) * 8 + xcd;
        group = j % groups;
    } else {
        chunk = b / groups;
        group = b % groups;
    }
}

// Access `lane_off` bytes past a wave-uniform base pointer: the base stays in
// scalar registers and one 32-bit lane offset serves every access.
template <class T>
__device__ __forceinline__ T ld_lane(const T *base, uint32_t lane_off)
{
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + lane_off);
}
template <class T>
__device__ __forceinline__ void st_lane(T *base, uint32_t lane_off, T v)
{
    *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + lane_off) = v;
}
// Gathers of a chunk's posteriors through one buffer resource: the lane
// offset is the vector offset and the row's column (times the column
// stride) the scalar offset, so no gathered load needs vector address
// arithmetic.  The resource covers exactly the chunk's n x 64 posteriors
// (a load outside it would return 0; none is made).
constexpr int32_t kBufferWord3 = 0x00020000;  // raw 32-bit access, gfx9-family layout
template <class T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t chunk_rsrc(const T *base, int32_t n)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<T *>(base), 0, n * kChunk * static_cast<int32_t>(sizeof(T)),
                                             kBufferWord3);
}
__device__ __forceinline__ float ld_gather(__amdgpu_buffer_rsrc_t rsrc, uint32_t lane_off, int32_t col, float)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(
                                         rsrc, static_cast<int32_t>(lane_off), col * kChunk * 4, 0));
}
__device__ __forceinline__ void st_scatter(__amdgpu_buffer_rsrc_t rsrc, uint32_t lane_off, int32_t col, float v)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), rsrc, static_cast<int32_t>(lane_off),
                                          col * kChunk * 4, 0);
}

// Non-temporal forms for the streamed messages r (read once and written once
// per launch, no reuse inside it); the gathered posteriors keep the cached forms.
template <class T>
__device__ __forceinline__ T ld_lane_nt(const T *base, uint32_t lane_off)
{
    return __builtin_nontemporal_load(reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + lane_off));
}
template <class T>
__device__ __forceinline__ void st_lane_nt(T *base, uint32_t lane_off, T v)
{
    __builtin_nontemporal_store(v, reinterpret_cast<T *>(reinterpret_cast<char *>(base) + lane_off));
}

// One check row of compile-time degree D: all 2D loads are issued before any
// arithmetic (the wave waits once per row, and straight-line code lets each
// edge start as soon as its own loads land).  Both halves of the row are
// evaluated here (two independent chains).
template <class A, int D, bool FIRST, bool ES>
__device__ __forceinline__ void check_row(const int32_t *__restrict__ cols, const typename A::T *__restrict__ L,
                                          int32_t n, typename A::T *__restrict__ Rrow, uint32_t off,
                                          uint32_t &parity)
{
    using T = typename A::T;
    constexpr int H = (D + 1) / 2;
    const __amdgpu_buffer_rsrc_t rsrc = chunk_rsrc(L, n);
    T lv[D], rv[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        if constexpr (std::is_same<T, float>::value)
            lv[k] = ld_gather(rsrc, off, cols[k], T(0));
        else
            lv[k] = ld_lane(L + cols[k] * kChunk, off);
        rv[k] = FIRST ? T(0) : ld_lane_nt(Rrow + k * kChunk, off);
    }
    typename A::Term a[D];
    typename A::Acc p[D];
    typename A::Acc acc0 = A::identity(), acc1 = A::identity();
    uint32_t sign = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        if (ES)
            parity ^= static_cast<uint32_t>(lv[k] < T(0));
        const T q = FIRST ? lv[k] : lv[k] - rv[k];
        check_forward<A>(q, a[k], p[k], k < H ? acc0 : acc1, sign);
    }
    typename A::Acc s0 = A::seed(acc1), s1 = A::seed(acc0);
#pragma unroll
    for (int k = D - 1; k >= 0; --k) {
        const T r = k < H ? check_backward<A>(a[k], p[k], s0, sign) : check_backward<A>(a[k], p[k], s1, sign);
        st_lane_nt(Rrow + k * kChunk, off, r);
    }
}

// The same row for a run-time degree d <= DMAX (guarded loops; used for FP64
// and for degrees above the largest exact bucket).
template <class A, int DMAX, bool FIRST, bool ES>
__device__ __forceinline__ void check_row_guarded(const int32_t *__restrict__ cols, int d,
                                                  const typename A::T *__restrict__ L, typename A::T *__restrict__ Rrow,
                                                  uint32_t off, uint32_t &parity)
{
    using T = typename A::T;
    const int h = (d + 1) / 2;
    T lv[DMAX], rv[DMAX];
#pragma unroll
    for (int k = 0; k < DMAX; ++k) {
        if (k < d) {
            lv[k] = ld_lane(L + cols[k] * kChunk, off);
            rv[k] = FIRST ? T(0) : ld_lane_nt(Rrow + k * kChunk, off);
        }
    }
    typename A::Term a[DMAX];
    typename A::Acc p[DMAX];
    typename A::Acc acc0 = A::identity(), acc1 = A::identity();
    uint32_t sign = 0;
#pragma unroll
    for (int k = 0; k < DMAX; ++k) {
        if (k < d) {
            if (ES)
                parity ^= static_cast<uint32_t>(lv[k] < T(0));
            const T q = FIRST ? lv[k] : lv[k] - rv[k];
            if (k < h)
                check_forward<A>(q, a[k], p[k], acc0, sign);
            else
                check_forward<A>(q, a[k], p[k], acc1, sign);
        }
    }
    typename A::Acc s0 = A::seed(acc1), s1 = A::seed(acc0);
#pragma unroll
    for (int k = DMAX - 1; k >= 0; --k) {
        if (k < d) {
            const T r = k < h ? check_backward<A>(a[k], p[k], s0, sign)
                              : check_backward<A>(a[k], p[k], s1, sign);
            st_lane_nt(Rrow + k * kChunk, off, r);
        }
    }
}

// Exact-degree dispatch for d in [D, DB]: one straight-line body per degree,
// so no unrolled loop carries guards (a guard makes every array element a
// control-flow merge and inflates register use).  A kernel's register budget
// is that of its largest body, hence one kernel per degree bucket DB.
template <class A, int D, int DB, bool FIRST, bool ES>
__device__ __forceinline__ void check_row_exact(int d, const int32_t *__restrict__ cols,
                                                const typename A::T *__restrict__ L, int32_t n,
                                                typename A::T *__restrict__ Rrow, uint32_t off, uint32_t &parity)
{
    if constexpr (D < DB) {
        if (d == D)
            check_row<A, D, FIRST, ES>(cols, L, n, Rrow, off, parity);
        else
            check_row_exact<A, D + 1, DB, FIRST, ES>(d, cols, L, n, Rrow, off, parity);
    } else {
        check_row<A, DB, FIRST, ES>(cols, L, n, Rrow, off, parity);
    }
}

// Check-node kernel (Loop 2): one wavefront = one check row x 64 frames.
// Rows must have degree <= DB.  EXACT selects straight-line bodies per degree.
template <class A, int DB, bool EXACT, bool FIRST, bool ES>
__global__ __launch_bounds__(256) void k_check(const int32_t *__restrict__ row_ptr,
                                               const int32_t *__restrict__ col_idx, int32_t m, int32_t n, int64_t E,
                                               int32_t groups, int32_t nchunk, typename A::T *__restrict__ R,
                                               const typename A::T *__restrict__ L, const int32_t *__restrict__ done,
                                               int32_t *__restrict__ unsat)
{
    using T = typename A::T;
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
    const int lane = static_cast<int>(threadIdx.x & 63);
    int group, chunk;
    map_block(static_cast<int>(blockIdx.x), groups, nchunk, group, chunk);
    const int row = group * kWaves + wave;
    if (row >= m)
        return;
    // A chunk whose frames have all stopped is skipped whole (one wave-uniform
    // load).  Otherwise every lane is computed: a stopped frame's posterior is
    // frozen (the variable kernel leaves it) and its messages are never read
    // again, and computing its lane costs no extra traffic, since the chunk's
    // 256-byte segments are read anyway.
    if (ES && chunk_active(done, nchunk, chunk) == 0)
        return;
    const uint32_t f = static_cast<uint32_t>(chunk) * 64u + static_cast<uint32_t>(lane);
    const uint32_t off = static_cast<uint32_t>(lane) * static_cast<uint32_t>(sizeof(T));
    const int32_t e0 = row_ptr[row];
    const int32_t d = __builtin_amdgcn_readfirstlane(row_ptr[row + 1] - e0);
    uint32_t parity = 0;
    T *Rrow = R + (static_cast<int64_t>(chunk) * E + e0) * kChunk;
    const T *Lc = L + static_cast<int64_t>(chunk) * n * kChunk;
    if (d > 0) {
        if constexpr (EXACT)
            check_row_exact<A, 1, DB, FIRST, ES>(d, col_idx + e0, Lc, n, Rrow, off, parity);
        else
            check_row_guarded<A, DB, FIRST, ES>(col_idx + e0, d, Lc, Rrow, off, parity);
    }
    if (ES && parity)
        unsat[f] = 1;
}

// L = Lch + sum of the column's r in ascending row order, for a column of
// compile-time degree D (loads first, then the ordered sum).
template <class A, int D>
__device__ __forceinline__ typename A::T column_sum(typename A::T acc, const int32_t *__restrict__ edges,
                                                    const typename A::T *__restrict__ R, uint32_t off)
{
    using T = typename A::T;
    T rv[D > 0 ? D : 1];
#pragma unroll
    for (int k = 0; k < D; ++k)
        rv[k] = ld_lane(R + edges[k] * kChunk, off);
#pragma unroll
    for (int k = 0; k < D; ++k)
        acc += rv[k];
    return acc;
}

template <class A, int D>
__device__ __forceinline__ typename A::T column_sum_exact(int dv, typename A::T acc, const int32_t *__restrict__ edges,
                                                          const typename A::T *__restrict__ R, uint32_t off)
{
    if constexpr (D <= 16) {
        if (dv == D)
            return column_sum<A, D>(acc, edges, R, off);
        return column_sum_exact<A, D + 1>(dv, acc, edges, R, off);
    } else {
        for (int32_t k = 0; k < dv; ++k)  // rare high-degree columns
            acc += ld_lane(R + edges[k] * kChunk, off);
        return acc;
    }
}

// Variable-node kernel (Loops 3 and 4): one wavefront = one variable x 64
// frames.  The hard decision is the sign of the stored posterior.  One item
// is one block's worth of work, kWaves columns of one frame chunk; the
// chunk's running count has been tested by the caller.
template <class A, bool ES>
__device__ __forceinline__ void variable_item(int group, int chunk, const int32_t *__restrict__ col_ptr,
                                              const int32_t *__restrict__ col_edge, int32_t n, int64_t E,
                                              int32_t nchunk, const typename A::T *__restrict__ R,
                                              const typename A::T *__restrict__ Lch, typename A::T *__restrict__ L,
                                              int32_t *__restrict__ done, const int32_t *__restrict__ unsat,
                                              int32_t t_prev)
{
    using T = typename A::T;
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
    const int lane = static_cast<int>(threadIdx.x & 63);
    const int col = group * kWaves + wave;
    if (col >= n)
        return;
    const uint32_t f = static_cast<uint32_t>(chunk) * 64u + static_cast<uint32_t>(lane);
    const uint32_t off = static_cast<uint32_t>(lane) * static_cast<uint32_t>(sizeof(T));
    const int32_t k0 = col_ptr[col];
    const int32_t dv = __builtin_amdgcn_readfirstlane(col_ptr[col + 1] - k0);
    const int64_t vo = (static_cast<int64_t>(chunk) * n + col) * kChunk;
    const T *Rc = R + static_cast<int64_t>(chunk) * E * kChunk;
    // With early stop the frame's state is loaded beside the column's values
    // (both words, so that neither load waits for the other).
    int32_t dn = -1, us = 1;
    if constexpr (ES) {
        dn = done[f];
        us = unsat[f];
    }
    const T acc = ld_lane(Lch + vo, off);
    const T v = column_sum_exact<A, 0>(dv, acc, col_edge + k0, Rc, off);
    if (ES) {
        // A frame runs iteration t unless it stopped earlier or its decision
        // x^(t-1) satisfies every row (it stops at t-1).  The column-0 wave of
        // each chunk records the stops and the chunk's count of running frames.
        const bool running = (dn < 0) & (us != 0);
        if (col == 0) {
            if (dn < 0 && !running)
                done[f] = t_prev;
            const uint64_t live = __ballot(running);
            if (lane == 0)
                done[nchunk * kChunk + chunk] = __popcll(live);
        }
        if (!running)
            return;
    }
    st_lane(L + vo, off, v);
}

// Without early stop the grid holds one block per item.  With early stop it
// holds at most the blocks the device keeps resident at once (stride_grid, a
// multiple of 8, so that item b still runs on XCD b mod 8), which stride over
// the items in order: the items in flight form one window moving through the
// item order, as under the hardware's own dispatch, and a launch over stopped
// chunks costs those blocks' passes over the item list instead of the
// dispatch of one block per column group and chunk.  A block tests a chunk's
// running count when its items move to another chunk.  The count may drop
// to 0 during the launch (the column-0 wave writes it); a block that still
// holds the older count computes the item, whose frames have all stopped and
// store nothing, and one that reads the 0 skips it: the same result.
// Measured on MI355X (stair64800, 256 frames): a launch over four running
// chunks took 69-70 us instead of 91, one after every frame stopped 13 us
// instead of 20.  Without early stop the strided form was 3% slower than one
// block per item, and a strided check kernel 13% slower per launch (a
// block's items are fixed, so the CUs of an XCD cannot even out its row
// groups' run times as the dispatcher does).
template <class A, bool ES>
__global__ __launch_bounds__(256) void k_variable(const int32_t *__restrict__ col_ptr,
                                                  const int32_t *__restrict__ col_edge, int32_t n, int64_t E,
                                                  int32_t groups, int32_t nchunk, const typename A::T *__restrict__ R,
                                                  const typename A::T *__restrict__ Lch, typename A::T *__restrict__ L,
                                                  int32_t *__restrict__ done, const int32_t *__restrict__ unsat,
                                                  int32_t t_prev)
{
    int group, chunk;
    if constexpr (ES) {
        const int items = groups * nchunk;
        int tested = -1, running = 0;
        for (int b = static_cast<int>(blockIdx.x); b < items; b += static_cast<int>(gridDim.x)) {
            map_block(b, groups, nchunk, group, chunk);
            if (chunk != tested) {
                tested = chunk;
                running = chunk_active(done, nchunk, chunk);
            }
            if (running != 0)
                variable_item<A, ES>(group, chunk, col_ptr, col_edge, n, E, nchunk, R, Lch, L, done, unsat, t_prev);
        }
    } else {
        map_block(static_cast<int>(blockIdx.x), groups, nchunk, group, chunk);
        variable_item<A, ES>(group, chunk, col_ptr, col_edge, n, E, nchunk, R, Lch, L, done, unsat, t_prev);
    }
}

}  // namespace flood

// Arguments of one check-node launch.
template <class A>
struct CheckArgs {
    const int32_t *row_ptr;
    const int32_t *col_idx;
    int32_t m, n;
    int64_t E;
    int32_t groups, nchunk;
    typename A::T *R;
    const typename A::T *L;
    const int32_t *done;
    int32_t *unsat;
};

// Grid of a launch whose 256-thread blocks stride over `items` items: as many
// blocks of kernel fn as the current device keeps resident at once (rounded
// down to a multiple of 8), or `items` if that is fewer.  The occupancy query
// and the CU count are cached per (kernel, device) in a fixed-size table; if
// either query fails the grid is `items` (one block per item).
unsigned stride_grid(const void *fn, unsigned items);

// Launcher of the check kernel for rows of degree <= DB; each (dtype, bucket)
// is defined in its own translation unit.
template <class A, int DB, bool EXACT>
void launch_check_bucket(const CheckArgs<A> &a, bool first, bool es, dim3 grid, hipStream_t s);

#define LDPC_CHECK_LAUNCH_ONE(A_, DB_, EX_, F_, E_)                                                              \
    do {                                                                                                         \
        ProfScope ps(LDPC_KERNEL_CHECK, s);                                                                      \
        LDPC_LAUNCH(ps, (flood::k_check<A_, DB_, EX_, F_, E_>), grid, dim3(256), 0, s, a.row_ptr, a.col_idx, a.m, \
                    a.n, a.E, a.groups, a.nchunk, a.R, a.L, a.done, a.unsat);                                   \
    } while (0)

#define LDPC_DEFINE_CHECK_BUCKET(A_, DB_, EX_)                                                                  \
    template <>                                                                                                 \
    void launch_check_bucket<A_, DB_, EX_>(const CheckArgs<A_> &a, bool first, bool es, dim3 grid,              \
                                           hipStream_t s)                                                       \
    {                                                                                                           \
        if (first && es)                                                                                        \
            LDPC_CHECK_LAUNCH_ONE(A_, DB_, EX_, true, true);                                                    \
        else if (first)                                                                                         \
            LDPC_CHECK_LAUNCH_ONE(A_, DB_, EX_, true, false);                                                   \
        else if (es)                                                                                            \
            LDPC_CHECK_LAUNCH_ONE(A_, DB_, EX_, false, true);                                                   \
        else                                                                                                    \
            LDPC_CHECK_LAUNCH_ONE(A_, DB_, EX_, false, false);                                                  \
    }

}  // namespace ldpc
