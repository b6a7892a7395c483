// Plain flooding path: one check-node and one variable-node kernel per
// iteration, with every message of every frame streamed through HBM.
//
// Schedule (arxiv 1812.06545, Section II, two-phase message passing and
// Algorithm 1): iteration t runs Loop 2 (all check nodes) as one launch, then
// Loops 3 and 4 (all variable nodes; the hard decision is the sign of the
// stored posterior) as a second launch; the launch boundary is the global
// barrier the flooding schedule needs.
//
// Data layout (frame-interleaved, the idea of Section III-B's interleaving
// kernels): frames are padded to a multiple of 64 and grouped in chunks of 64;
// every per-edge or per-variable array is stored [chunk][edge or
// variable][64 frames].  A wavefront holds one check row (or one variable)
// for the 64 frames of a chunk: each lane is a frame, every load and store is
// a 256-byte (FP32) contiguous segment, the row's CSR indices are
// wave-uniform scalar loads, and all data of a chunk (E + 2n segments) is one
// contiguous region, which keeps DRAM pages and address translations local
// while an XCD works through the chunk.
//
// Stored state per frame: r (one message per edge), the posterior L (one per
// variable) and the scaled channel values Lch.  The check kernel forms
// q = L - r_old on the fly (Loop 3's extrinsic message), so q is never
// written back; per iteration the HBM traffic is
//   check:    read r, gather L (served from L2), write r
//   variable: read r, read Lch, write L.
//
// Early stop: the check kernel of iteration t also forms the syndrome of the
// previous hard decision x^(t-1) = [L^(t-1) < 0] from the L values it
// gathers anyway, and marks unsatisfied frames.  The variable kernel of
// iteration t then retires a frame whose syndrome was zero (iters = t-1) and
// leaves its posterior untouched.  No host synchronisation is needed.
//
// The layered schedule (LDPC_LAYERED) runs on the same arrays: r per edge,
// starting at 0, and L, starting at Lch.  An iteration is one launch per layer
// (layered_kernels.h); with early stop a syndrome kernel and a retire kernel
// test x^(t-1) = [L < 0] before pass t, since inside a pass the rows see
// different posteriors and cannot test one decision together.
//
// With LDPC_MIN_SUM the check rule is min-sum (minsum_kernels.h) on either
// schedule; the variable kernel, the syndrome and the retire kernels are
// shared.
#include <algorithm>
#include <cmath>
#include <mutex>

#include "flood_kernels.h"
#include "layered_kernels.h"
#include "minsum_kernels.h"

namespace ldpc {

unsigned stride_grid(const void *fn, unsigned items)
{
    struct Entry {
        const void *fn;
        int dev;
        unsigned blocks;
    };
    constexpr int kEntries = 64;
    static std::mutex mu;
    static Entry cache[kEntries];
    static int used = 0;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return items;
    unsigned blocks = 0;
    {
        std::lock_guard<std::mutex> lk(mu);
        for (int i = 0; i < used && blocks == 0; ++i)
            if (cache[i].fn == fn && cache[i].dev == dev)
                blocks = cache[i].blocks;
    }
    if (blocks == 0) {
        int per_cu = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, 0) != hipSuccess || per_cu < 1 ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) {
            (void)hipGetLastError();  // the failed query, not a launch, set it
            return items;
        }
        blocks = std::max(8u, static_cast<unsigned>(per_cu * cus) & ~7u);
        std::lock_guard<std::mutex> lk(mu);
        if (used < kEntries)
            cache[used++] = Entry{fn, dev, blocks};
    }
    return std::min(items, blocks);
}

namespace {

using namespace flood;

// [frames][n] -> [chunk][n][64] through a 64x64 LDS tile; padding frames get LLR 1.
template <class A>
__global__ __launch_bounds__(256) void k_ingest(const typename A::T *__restrict__ llr, int32_t F, int32_t n,
                                                typename A::T *__restrict__ Lch, typename A::T *__restrict__ L)
{
    using T = typename A::T;
    __shared__ T tile[64][65];
    const int c0 = blockIdx.x * 64, f0 = blockIdx.y * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int i = ty; i < 64; i += 4) {
        const int f = f0 + i, c = c0 + tx;
        T v = T(1);
        if (f < F && c < n)
            v = llr[static_cast<int64_t>(f) * n + c];
        tile[i][tx] = v * T(A::kIn);
    }
    __syncthreads();
    for (int i = ty; i < 64; i += 4) {
        const int c = c0 + i;
        if (c < n) {
            const T v = tile[tx][i];
            const int64_t o = (static_cast<int64_t>(blockIdx.y) * n + c) * kChunk + tx;
            Lch[o] = v;
            L[o] = v;
        }
    }
}

// done[f] = -1 (running) for every frame, done[Fp + c] = 64 running frames
// per chunk, unsat = 0.
__global__ __launch_bounds__(256) void k_frames_init(int64_t Fp, int32_t *__restrict__ done,
                                                     int32_t *__restrict__ unsat, int64_t unsat_words)
{
    const int64_t nchunk = Fp / kChunk;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < Fp + nchunk + unsat_words;
         i += stride) {
        if (i < Fp)
            done[i] = -1;
        else if (i < Fp + nchunk)
            done[i] = kChunk;
        else
            unsat[i - Fp - nchunk] = 0;
    }
}

// [chunk][n][64] -> bits / posterior [frames][n]; iters.  A frame that ran no
// iteration reports the caller's LLRs bit-exactly as its posterior.
template <class A>
__global__ __launch_bounds__(256) void k_output(const typename A::T *__restrict__ L,
                                                const typename A::T *__restrict__ llr,
                                                const int32_t *__restrict__ done, int32_t F, int32_t n,
                                                int32_t max_iter, int32_t es, uint8_t *__restrict__ bits,
                                                int32_t *__restrict__ iters, typename A::T *__restrict__ posterior)
{
    using T = typename A::T;
    __shared__ T tile[64][65];
    __shared__ int32_t it[64];
    const int c0 = blockIdx.x * 64, f0 = blockIdx.y * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    if (threadIdx.x < 64) {
        const int64_t f = f0 + threadIdx.x;
        const int32_t v = (es && done[f] >= 0) ? done[f] : max_iter;
        it[threadIdx.x] = v;
        if (blockIdx.x == 0 && f < F)
            iters[f] = v;
    }
    for (int i = ty; i < 64; i += 4) {
        const int c = c0 + i;
        tile[i][tx] = c < n ? L[(static_cast<int64_t>(blockIdx.y) * n + c) * kChunk + tx] : T(0);
    }
    __syncthreads();
    for (int i = ty; i < 64; i += 4) {
        const int f = f0 + i, c = c0 + tx;
        if (f < F && c < n) {
            const T v = tile[tx][i];
            const int64_t o = static_cast<int64_t>(f) * n + c;
            bits[o] = static_cast<uint8_t>(v < T(0));
            if (posterior)
                posterior[o] = it[i] == 0 ? llr[o] : v * T(A::kOut);
        }
    }
}

// Syndrome of the hard decision [L < 0]: one wavefront = one row x 64
// frames; an unsatisfied row marks its frames in `unsat`.
template <class A>
__global__ __launch_bounds__(256) void k_syndrome(const int32_t *__restrict__ row_ptr,
                                                  const int32_t *__restrict__ col_idx, int32_t m, int32_t n,
                                                  int32_t groups, int32_t nchunk, const typename A::T *__restrict__ L,
                                                  const int32_t *__restrict__ done, int32_t *__restrict__ unsat)
{
    using T = typename A::T;
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
    const int lane = static_cast<int>(threadIdx.x & 63);
    int group, chunk;
    map_block(static_cast<int>(blockIdx.x), groups, nchunk, group, chunk);
    const int row = group * kWaves + wave;
    if (row >= m)
        return;
    if (chunk_active(done, nchunk, chunk) == 0)
        return;
    const uint32_t f = static_cast<uint32_t>(chunk) * 64u + static_cast<uint32_t>(lane);
    if (done[f] >= 0)
        return;
    const uint32_t off = static_cast<uint32_t>(lane) * static_cast<uint32_t>(sizeof(T));
    const int32_t e0 = row_ptr[row];
    const int32_t d = __builtin_amdgcn_readfirstlane(row_ptr[row + 1] - e0);
    const T *Lc = L + static_cast<int64_t>(chunk) * n * kChunk;
    uint32_t parity = 0;
#pragma unroll 8
    for (int32_t k = 0; k < d; ++k)
        parity ^= static_cast<uint32_t>(ld_lane(Lc + col_idx[e0 + k] * kChunk, off) < T(0));
    if (parity)
        unsat[f] = 1;
}

// A frame still running whose decision x^t satisfies every row stops at t
// (and leaves its chunk's count of running frames).
__global__ __launch_bounds__(256) void k_retire(int64_t Fp, int32_t *__restrict__ done,
                                                const int32_t *__restrict__ unsat, int32_t t)
{
    const int64_t f = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (f < Fp && done[f] < 0 && unsat[f] == 0) {
        done[f] = t;
        atomicSub(&done[Fp + f / kChunk], 1);
    }
}

struct Carve {
    char *p;
    template <class U>
    U *take(size_t count)
    {
        U *r = reinterpret_cast<U *>(p);
        p += align_up(count * sizeof(U), 256);
        return r;
    }
};

template <class A>
size_t ws_bytes(const ldpc_code_s *c, int64_t Fp, int32_t max_iter)
{
    using T = typename A::T;
    size_t b = 0;
    b += align_up(static_cast<size_t>(c->E) * Fp * sizeof(T), 256);
    b += 2 * align_up(static_cast<size_t>(c->n) * Fp * sizeof(T), 256);
    b += align_up(static_cast<size_t>(Fp + Fp / kChunk) * sizeof(int32_t), 256);  // done, chunk counts
    b += align_up(static_cast<size_t>(std::max(max_iter, 1)) * Fp * sizeof(int32_t), 256);
    return b;
}

// Smallest kernel bucket that holds every row of the code.
template <class A>
void launch_check(const ldpc_code_s *c, bool first, bool es, dim3 grid, hipStream_t s, const CheckArgs<A> &a);

template <>
void launch_check<ArithF32>(const ldpc_code_s *c, bool first, bool es, dim3 grid, hipStream_t s,
                            const CheckArgs<ArithF32> &a)
{
    const int d = c->max_row_deg;
    if (d <= 8)
        launch_check_bucket<ArithF32, 8, true>(a, first, es, grid, s);
    else if (d <= 16)
        launch_check_bucket<ArithF32, 16, true>(a, first, es, grid, s);
    else if (d <= 24)
        launch_check_bucket<ArithF32, 24, true>(a, first, es, grid, s);
    else if (d <= 32)
        launch_check_bucket<ArithF32, 32, true>(a, first, es, grid, s);
    else
        launch_check_bucket<ArithF32, 64, false>(a, first, es, grid, s);
}

template <>
void launch_check<ArithF64>(const ldpc_code_s *c, bool first, bool es, dim3 grid, hipStream_t s,
                            const CheckArgs<ArithF64> &a)
{
    const int d = c->max_row_deg;
    if (d <= 8)
        launch_check_bucket<ArithF64, 8, false>(a, first, es, grid, s);
    else if (d <= 16)
        launch_check_bucket<ArithF64, 16, false>(a, first, es, grid, s);
    else if (d <= 32)
        launch_check_bucket<ArithF64, 32, false>(a, first, es, grid, s);
    else
        launch_check_bucket<ArithF64, 64, false>(a, first, es, grid, s);
}

// Smallest layer-kernel bucket that holds every row of layer l.
template <class A>
void launch_layer(int32_t dmax, bool first, bool es, dim3 grid, hipStream_t s, const LayerArgs<A> &a);

template <>
void launch_layer<ArithF32>(int32_t d, bool first, bool es, dim3 grid, hipStream_t s, const LayerArgs<ArithF32> &a)
{
    if (d <= 8)
        launch_layer_bucket<ArithF32, 8, true>(a, first, es, grid, s);
    else if (d <= 16)
        launch_layer_bucket<ArithF32, 16, true>(a, first, es, grid, s);
    else if (d <= 24)
        launch_layer_bucket<ArithF32, 24, true>(a, first, es, grid, s);
    else if (d <= 32)
        launch_layer_bucket<ArithF32, 32, true>(a, first, es, grid, s);
    else
        launch_layer_bucket<ArithF32, 64, false>(a, first, es, grid, s);
}

template <>
void launch_layer<ArithF64>(int32_t d, bool first, bool es, dim3 grid, hipStream_t s, const LayerArgs<ArithF64> &a)
{
    if (d <= 8)
        launch_layer_bucket<ArithF64, 8, false>(a, first, es, grid, s);
    else if (d <= 16)
        launch_layer_bucket<ArithF64, 16, false>(a, first, es, grid, s);
    else if (d <= 32)
        launch_layer_bucket<ArithF64, 32, false>(a, first, es, grid, s);
    else
        launch_layer_bucket<ArithF64, 64, false>(a, first, es, grid, s);
}

// Min-sum bucket of a row degree: 8, 16, 32 or 64.
template <class A>
void launch_ms(int32_t d, bool layered, bool first, bool es, dim3 grid, hipStream_t s, const MinSumArgs<A> &a)
{
    if (d <= 8)
        layered ? launch_layer_ms_bucket<A, 8>(a, first, es, grid, s) : launch_check_ms_bucket<A, 8>(a, first, es, grid, s);
    else if (d <= 16)
        layered ? launch_layer_ms_bucket<A, 16>(a, first, es, grid, s)
                : launch_check_ms_bucket<A, 16>(a, first, es, grid, s);
    else if (d <= 32)
        layered ? launch_layer_ms_bucket<A, 32>(a, first, es, grid, s)
                : launch_check_ms_bucket<A, 32>(a, first, es, grid, s);
    else
        layered ? launch_layer_ms_bucket<A, 64>(a, first, es, grid, s)
                : launch_check_ms_bucket<A, 64>(a, first, es, grid, s);
}

template <class A>
ldpc_status decode_impl(const ldpc_code_s *c, int32_t frames, int32_t max_iter, uint32_t flags, const void *llr_v,
                        uint8_t *bits, int32_t *iters, void *post_v, void *ws, hipStream_t s, double ms_scale,
                        double ms_offset)
{
    using T = typename A::T;
    const int64_t Fp = frames_padded(frames);
    const int32_t nchunk = static_cast<int32_t>(Fp / kChunk);
    const bool es = (flags & LDPC_EARLY_STOP) != 0;
    const T *llr = static_cast<const T *>(llr_v);
    T *post = static_cast<T *>(post_v);

    Carve cv{static_cast<char *>(ws)};
    T *R = cv.take<T>(static_cast<size_t>(c->E) * Fp);
    T *L = cv.take<T>(static_cast<size_t>(c->n) * Fp);
    T *Lch = cv.take<T>(static_cast<size_t>(c->n) * Fp);
    int32_t *done = cv.take<int32_t>(Fp + nchunk);  // per frame, then per chunk (flood_kernels.h)
    int32_t *unsat = cv.take<int32_t>(static_cast<size_t>(std::max(max_iter, 1)) * Fp);

    // The frame state is read only with early stop (every read is under the
    // kernels' ES flag), so only then is it initialised.
    if (es) {
        const int64_t unsat_words = static_cast<int64_t>(max_iter) * Fp;
        const int init_blocks = static_cast<int>(std::min<int64_t>((Fp + nchunk + unsat_words + 255) / 256, 4096));
        ProfScope ps(LDPC_KERNEL_OTHER, s);
        LDPC_LAUNCH(ps, k_frames_init, dim3(init_blocks), dim3(256), 0, s, Fp, done, unsat, unsat_words);
    }
    const dim3 tiles((c->n + 63) / 64, nchunk);
    {
        ProfScope ps(LDPC_KERNEL_INGEST, s);
        LDPC_LAUNCH(ps, (k_ingest<A>), tiles, dim3(256), 0, s, llr, frames, c->n, Lch, L);
    }

    const int32_t rgroups = (c->m + kWaves - 1) / kWaves;
    const int32_t cgroups = (c->n + kWaves - 1) / kWaves;
    const dim3 rgrid(static_cast<unsigned>(rgroups) * nchunk), cgrid(static_cast<unsigned>(cgroups) * nchunk);
    // With early stop the variable kernel's resident blocks stride over its
    // items (flood_kernels.h); every other launch has one block per item.
    const dim3 cgrid_es(es ? stride_grid(reinterpret_cast<const void *>(&k_variable<A, true>), cgrid.x) : cgrid.x);
    const bool layered = (flags & LDPC_LAYERED) != 0;
    const bool ms = (flags & LDPC_MIN_SUM) != 0;
    const T scale = static_cast<T>(ms_scale), offset = static_cast<T>(ms_offset * A::kIn);
    for (int32_t t = 1; t <= max_iter && layered; ++t) {
        const bool first = (t == 1);
        if (es && c->m > 0) {
            int32_t *unsat_t = unsat + static_cast<int64_t>(t - 1) * Fp;
            {
                ProfScope ps(LDPC_KERNEL_OTHER, s);
                LDPC_LAUNCH(ps, (k_syndrome<A>), rgrid, dim3(256), 0, s, c->row_ptr, c->col_idx, c->m, c->n,
                                   rgroups, nchunk, L, done, unsat_t);
            }
            ProfScope ps(LDPC_KERNEL_OTHER, s);
            LDPC_LAUNCH(ps, k_retire, dim3(static_cast<unsigned>((Fp + 255) / 256)), dim3(256), 0, s, Fp, done,
                               unsat_t, t - 1);
        }
        for (size_t l = 0; l + 1 < c->layer_ptr.size(); ++l) {
            const int32_t row0 = c->layer_ptr[l], rows = c->layer_ptr[l + 1] - row0;
            const int32_t groups = (rows + kWaves - 1) / kWaves;
            const dim3 grid(static_cast<unsigned>(groups) * nchunk);
            if (ms) {
                const MinSumArgs<A> ma{c->row_ptr, c->col_idx, row0, rows, c->m, c->n, c->E, groups, nchunk,
                                       R, L, done, nullptr, scale, offset};
                launch_ms<A>(c->layer_dmax[l], true, first, es, grid, s, ma);
            } else {
                const LayerArgs<A> la{c->row_ptr, c->col_idx, row0, rows, c->n, c->E, groups, nchunk, R, L, done};
                launch_layer<A>(c->layer_dmax[l], first, es, grid, s, la);
            }
        }
    }
    for (int32_t t = 1; t <= max_iter && !layered; ++t) {
        const bool first = (t == 1);
        int32_t *unsat_t = unsat + static_cast<int64_t>(t - 1) * Fp;
        if (ms) {
            const MinSumArgs<A> ma{c->row_ptr, c->col_idx, 0, c->m, c->m, c->n, c->E, rgroups, nchunk,
                                   R, L, done, unsat_t, scale, offset};
            launch_ms<A>(c->max_row_deg, false, first, es, rgrid, s, ma);
        } else {
            const CheckArgs<A> ca{c->row_ptr, c->col_idx, c->m, c->n, c->E, rgroups, nchunk, R, L, done, unsat_t};
            launch_check<A>(c, first, es, rgrid, s, ca);
        }
        ProfScope ps(LDPC_KERNEL_VARIABLE, s);
        if (es)
            LDPC_LAUNCH(ps, (k_variable<A, true>), cgrid_es, dim3(256), 0, s, c->col_ptr, c->col_edge, c->n, c->E,
                               cgroups, nchunk, R, Lch, L, done, unsat_t, t - 1);
        else
            LDPC_LAUNCH(ps, (k_variable<A, false>), cgrid, dim3(256), 0, s, c->col_ptr, c->col_edge, c->n, c->E,
                               cgroups, nchunk, R, Lch, L, done, unsat_t, t - 1);
    }
    {
        ProfScope ps(LDPC_KERNEL_OUTPUT, s);
        LDPC_LAUNCH(ps, (k_output<A>), tiles, dim3(256), 0, s, L, llr, done, frames, c->n, max_iter,
                           static_cast<int32_t>(es), bits, iters, post);
    }
    return hipGetLastError() == hipSuccess ? LDPC_OK : LDPC_EDEVICE;
}

}  // namespace

size_t stream_workspace_bytes(const ldpc_code_s *c, ldpc_dtype dt, int32_t frames, int32_t max_iter)
{
    const int64_t Fp = frames_padded(frames);
    return dt == LDPC_F64 ? ws_bytes<ArithF64>(c, Fp, max_iter) : ws_bytes<ArithF32>(c, Fp, max_iter);
}

ldpc_status stream_decode(const ldpc_code_s *c, ldpc_dtype dt, int32_t frames, int32_t max_iter, uint32_t flags,
                          const void *llr, uint8_t *bits, int32_t *iters, void *posterior, void *ws,
                          hipStream_t stream, double ms_scale, double ms_offset)
{
    if (dt == LDPC_F64)
        return decode_impl<ArithF64>(c, frames, max_iter, flags, llr, bits, iters, posterior, ws, stream, ms_scale,
                                     ms_offset);
    return decode_impl<ArithF32>(c, frames, max_iter, flags, llr, bits, iters, posterior, ws, stream, ms_scale,
                                 ms_offset);
}

bool minsum_params_ok(double scale, double offset)
{
    return std::isfinite(scale) && scale > 0.0 && std::isfinite(offset) && offset >= 0.0;
}

}  // namespace ldpc

extern "C" ldpc_status ldpc_workspace_bytes(ldpc_code code, ldpc_dtype dtype, int32_t frames, int32_t max_iter,
                                            size_t *bytes)
try {
    if (!code || !bytes || frames < 0 || frames > LDPC_MAX_FRAMES || max_iter < 0 ||
        (dtype != LDPC_F32 && dtype != LDPC_F64))
        return LDPC_EINVAL;
    *bytes = ldpc::stream_workspace_bytes(code, dtype, frames, max_iter);
    return LDPC_OK;
} catch (...) {
    return ldpc::status_of_exception();
}

extern "C" ldpc_status ldpc_decode(ldpc_code code, ldpc_dtype dtype, int32_t frames, int32_t max_iter,
                                   uint32_t flags, const void *llr, uint8_t *bits, int32_t *iters, void *posterior,
                                   void *workspace, size_t workspace_bytes, void *stream)
try {
    return ldpc_decode_minsum(code, dtype, frames, max_iter, flags, 1.0f, 0.0f, llr, bits, iters, posterior,
                              workspace, workspace_bytes, stream);
} catch (...) {
    return ldpc::status_of_exception();
}

extern "C" ldpc_status ldpc_decode_minsum(ldpc_code code, ldpc_dtype dtype, int32_t frames, int32_t max_iter,
                                          uint32_t flags, float ms_scale, float ms_offset, const void *llr,
                                          uint8_t *bits, int32_t *iters, void *posterior, void *workspace,
                                          size_t workspace_bytes, void *stream)
try {
    if (!code || frames < 0 || frames > LDPC_MAX_FRAMES || max_iter < 0 ||
        (flags & ~(LDPC_EARLY_STOP | LDPC_LAYERED | LDPC_MIN_SUM)) != 0 || (dtype != LDPC_F32 && dtype != LDPC_F64) ||
        !ldpc::minsum_params_ok(ms_scale, ms_offset))
        return LDPC_EINVAL;
    if (frames == 0)
        return LDPC_OK;
    if (!llr || !bits || !iters || !workspace)
        return LDPC_EINVAL;
    if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
        return LDPC_EINVAL;
    if (workspace_bytes < ldpc::stream_workspace_bytes(code, dtype, frames, max_iter))
        return LDPC_EINVAL;
    if (!ldpc::code_on_current_device(code))
        return LDPC_EINVAL;
    return ldpc::stream_decode(code, dtype, frames, max_iter, flags, llr, bits, iters, posterior, workspace,
                               static_cast<hipStream_t>(stream), ms_scale, ms_offset);
} catch (...) {
    return ldpc::status_of_exception();
}
