// Internal declarations shared by the libldpc translation units.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <new>
#include <stdexcept>
#include <system_error>
#include <vector>

#include "ldpc.h"

#define LDPC_HIP_OR_RETURN(expr)                 \
    do {                                         \
        hipError_t ldpc_e_ = (expr);             \
        if (ldpc_e_ != hipSuccess)               \
            return LDPC_EDEVICE;                 \
    } while (0)

namespace ldpc {

// No C++ exception crosses the C interface: every entry point is a
// function-try-block whose handler calls this (inside the handler, so the
// exception in flight is rethrown and classified).  Host allocation and
// thread-creation failures become LDPC_ENOMEM; nothing else is expected to
// throw, and anything that does is reported as LDPC_EDEVICE.
inline ldpc_status status_of_exception() noexcept
{
    try {
        throw;
    } catch (const std::bad_alloc &) {
        return LDPC_ENOMEM;
    } catch (const std::length_error &) {
        return LDPC_ENOMEM;
    } catch (const std::system_error &) {
        return LDPC_ENOMEM;
    } catch (...) {
        return LDPC_EDEVICE;
    }
}

}  // namespace ldpc

// A code handle: H in device memory, in two layouts.
//   CSR/CSC (every code): edges numbered in CSR order (rows ascending,
//   columns ascending inside a row); col_edge lists each column's edges in
//   ascending row order.  Used by the per-iteration streaming kernels.
//   Circulant-block tables (QC codes only): blocks numbered row-major over
//   the base matrix; the edge of block b in check row i*Z + r is b*Z + r.
//   Used by the fused frame-resident kernel.
struct ldpc_code_s {
    int device = 0;
    int32_t m = 0, n = 0;
    int64_t E = 0;
    int32_t max_row_deg = 0, max_col_deg = 0;
    void *d_mem = nullptr;
    const int32_t *row_ptr = nullptr;   // m + 1
    const int32_t *col_idx = nullptr;   // E
    const int32_t *col_ptr = nullptr;   // n + 1
    const int32_t *col_edge = nullptr;  // E
    // circulant-block tables (is_qc)
    bool is_qc = false;
    int32_t mb = 0, nb = 0, Z = 0, nblocks = 0;
    int32_t max_brow_deg = 0, max_bcol_deg = 0;
    // qc_tab layout (int32 words):
    //   [0, mb]                 row_blk_start   (first block of block-row i; mb+1 entries)
    //   [mb+1, +nblocks)        blk_col         (base column j of block b)
    //   [.., +nblocks)          blk_shift       (shift s of block b)
    //   [.., +nb+1)             col_blk_start   (nb+1 entries)
    //   [.., +nblocks)          col_blk         (blocks of base column j, ascending block-row)
    const int32_t *qc_tab = nullptr;
    int32_t qc_words = 0;
    std::vector<int32_t> h_qc_tab;
    // Thread-slot tables of the fused kernel (every code).  Check rows are
    // visited in "slot" order: for QC codes block-rows sorted by decreasing
    // degree (rows of one block-row consecutive), otherwise natural order;
    // brow_order[i] is the block-row in sorted position i (QC only).
    // row_gmax[g]: largest row degree among slots 32g .. 32g+31 (one
    // wavefront's rows: the fused kernel gives each row two lanes);
    // col_gmax[g]: largest column degree among columns 64g .. 64g+63.
    const int32_t *brow_order = nullptr;
    const int32_t *row_gmax = nullptr;
    const int32_t *col_gmax = nullptr;
    // Half-row words of the fused kernel's circulant view (QC codes whose
    // sizes fit the fields, else null): word 2 sr + h describes half h of
    // row slot sr as (first block of the half) | (its length) << 13 |
    // (the row's index within its block-row) << 19.
    const uint32_t *half_rows = nullptr;
    // Layers of the layered schedule (host): maximal runs of consecutive rows,
    // in ascending order, in which no two rows share a variable.  Layer l is
    // rows [layer_ptr[l], layer_ptr[l+1]); layer_dmax[l] its largest degree.
    std::vector<int32_t> layer_ptr, layer_dmax;
    const int32_t *d_layer_ptr = nullptr;  // device copy of layer_ptr
    // Hash of the code's shape (sizes, lifting size, row and column degree
    // histograms): the key of tuning choices, which depend on shape only.
    uint64_t shape_hash = 0;
};

namespace ldpc {

constexpr int kChunk = 64;  // frames per wavefront in the streaming layout

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }
inline int64_t frames_padded(int64_t frames) { return (frames + kChunk - 1) / kChunk * kChunk; }

bool code_on_current_device(const ldpc_code_s *c);

// Timing of one kernel launch when profiling is on (and the stream is not
// being captured): the scope hands out a start and a stop event that the
// launch carries itself (LDPC_LAUNCH, i.e. hipExtLaunchKernelGGL), so the
// runtime stamps the kernel's own start and end and no separate event
// packet sits between dependent launches; the scope files the pair on exit.
// Otherwise both events are null and LDPC_LAUNCH is a plain launch.
class ProfScope {
  public:
    // enabled = false: no timing for this launch, whatever the global setting.
    ProfScope(ldpc_kernel_kind kind, hipStream_t stream, bool enabled = true);
    ~ProfScope();
    ProfScope(const ProfScope &) = delete;
    ProfScope &operator=(const ProfScope &) = delete;
    hipEvent_t start() const { return start_; }
    hipEvent_t stop() const { return stop_; }

  private:
    int kind_ = -1;
    hipEvent_t start_ = nullptr, stop_ = nullptr;
};

#define LDPC_LAUNCH(ps, kernel, grid, block, shmem, stream, ...)                                                  \
    do {                                                                                                         \
        if ((ps).start())                                                                                        \
            hipExtLaunchKernelGGL(kernel, grid, block, shmem, stream, (ps).start(), (ps).stop(), 0u, __VA_ARGS__); \
        else                                                                                                     \
            hipLaunchKernelGGL(kernel, grid, block, shmem, stream, __VA_ARGS__);                                \
    } while (0)

// Copies bytes (a multiple of 16, both pointers 16-byte aligned) with the
// streaming copy kernel on `stream`; either side may be pinned host memory
// mapped for the device.
ldpc_status launch_copy16(void *dst, const void *src, size_t bytes, hipStream_t stream);
// The same copy on a grid of at most max_blocks workgroups of 256 threads,
// for copies that cross the host link while other kernels run.
ldpc_status launch_link_copy16(void *dst, const void *src, size_t bytes, int32_t max_blocks, hipStream_t stream);

// Workspace bytes of one fused launch of ldpc_decode_batch (its job table
// and work counter).  A batch of J jobs needs at most J such launches.
size_t fused_group_bytes();

// Streaming (per-iteration) path.
size_t stream_workspace_bytes(const ldpc_code_s *c, ldpc_dtype dt, int32_t frames, int32_t max_iter);
// ms_scale / ms_offset: the min-sum magnitude correction (used with
// LDPC_MIN_SUM; natural-LLR units).
ldpc_status stream_decode(const ldpc_code_s *c, ldpc_dtype dt, int32_t frames, int32_t max_iter, uint32_t flags,
                          const void *llr, uint8_t *bits, int32_t *iters, void *posterior, void *ws,
                          hipStream_t stream, double ms_scale, double ms_offset);
// scale finite and > 0, offset finite and >= 0.
bool minsum_params_ok(double scale, double offset);

}  // namespace ldpc
