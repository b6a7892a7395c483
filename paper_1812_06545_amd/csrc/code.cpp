// Code handles: validation of H and its device-resident layouts.
//
// H (arxiv 1812.06545, Section II) arrives as CSR or as a quasi-cyclic base
// matrix of circulant shifts.  Both are canonicalised to CSR with columns
// ascending inside each row, and the transposed view (each column's edges in
// ascending row order) is built once; everything is uploaded in a single
// device allocation and never changes afterwards.
#include <algorithm>
#include <cstring>
#include <vector>

#include "ldpc_internal.h"

namespace {

struct HostLayout {
    int32_t m = 0, n = 0;
    std::vector<int32_t> row_ptr, col_idx, col_ptr, col_edge;
    int32_t max_row_deg = 0, max_col_deg = 0;
};

ldpc_status build_host_layout(int32_t m, int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                              HostLayout &h)
{
    if (m < 1 || n < 1 || !row_ptr)
        return LDPC_EINVAL;
    if (row_ptr[0] != 0)
        return LDPC_EINVAL;
    for (int32_t i = 0; i < m; ++i)
        if (row_ptr[i + 1] < row_ptr[i])
            return LDPC_EINVAL;
    const int64_t E = row_ptr[m];
    if (E > 0 && !col_idx)
        return LDPC_EINVAL;
    // The kernels index a 64-frame chunk's messages and posteriors with
    // 32-bit byte and element offsets (edge x 64, variable x 64 x 8 bytes).
    if (E > LDPC_MAX_EDGES || n > LDPC_MAX_VARIABLES)
        return LDPC_EUNSUPPORTED;
    h.m = m;
    h.n = n;
    h.row_ptr.assign(row_ptr, row_ptr + m + 1);
    h.col_idx.resize(E);
    for (int32_t i = 0; i < m; ++i) {
        const int32_t b = row_ptr[i], e = row_ptr[i + 1];
        for (int32_t k = b; k < e; ++k) {
            if (col_idx[k] < 0 || col_idx[k] >= n)
                return LDPC_EINVAL;
            h.col_idx[k] = col_idx[k];
        }
        std::sort(h.col_idx.begin() + b, h.col_idx.begin() + e);
        for (int32_t k = b + 1; k < e; ++k)
            if (h.col_idx[k] == h.col_idx[k - 1])
                return LDPC_EINVAL;  // duplicate edge
        h.max_row_deg = std::max(h.max_row_deg, e - b);
    }
    if (h.max_row_deg > LDPC_MAX_ROW_DEGREE)
        return LDPC_EUNSUPPORTED;
    h.col_ptr.assign(n + 1, 0);
    for (int64_t k = 0; k < E; ++k)
        h.col_ptr[h.col_idx[k] + 1]++;
    for (int32_t j = 0; j < n; ++j) {
        h.max_col_deg = std::max(h.max_col_deg, h.col_ptr[j + 1]);
        h.col_ptr[j + 1] += h.col_ptr[j];
    }
    h.col_edge.resize(E);
    std::vector<int32_t> fill(n, 0);
    for (int32_t i = 0; i < m; ++i)
        for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
            const int32_t j = h.col_idx[k];
            h.col_edge[h.col_ptr[j] + fill[j]++] = k;
        }
    return LDPC_OK;
}

// Slot tables of the fused kernel (see ldpc_code_s).  brow_order is empty
// for codes without a circulant-block structure.
void slot_tables(const HostLayout &h, const std::vector<int32_t> &row_blk_start, int32_t Z,
                 std::vector<int32_t> &brow_order, std::vector<int32_t> &row_gmax, std::vector<int32_t> &col_gmax)
{
    std::vector<int32_t> row_deg(h.m);
    if (!row_blk_start.empty()) {
        const int32_t mb = static_cast<int32_t>(row_blk_start.size()) - 1;
        brow_order.resize(mb);
        for (int32_t i = 0; i < mb; ++i)
            brow_order[i] = i;
        std::stable_sort(brow_order.begin(), brow_order.end(), [&](int32_t a, int32_t b) {
            return row_blk_start[a + 1] - row_blk_start[a] > row_blk_start[b + 1] - row_blk_start[b];
        });
        for (int32_t si = 0; si < mb; ++si)
            for (int32_t r = 0; r < Z; ++r)
                row_deg[si * Z + r] = row_blk_start[brow_order[si] + 1] - row_blk_start[brow_order[si]];
    } else {
        for (int32_t i = 0; i < h.m; ++i)
            row_deg[i] = h.row_ptr[i + 1] - h.row_ptr[i];
    }
    row_gmax.assign((h.m + 31) / 32, 0);
    for (int32_t i = 0; i < h.m; ++i)
        row_gmax[i / 32] = std::max(row_gmax[i / 32], row_deg[i]);
    col_gmax.assign((h.n + 63) / 64, 0);
    for (int32_t j = 0; j < h.n; ++j)
        col_gmax[j / 64] = std::max(col_gmax[j / 64], h.col_ptr[j + 1] - h.col_ptr[j]);
}

// Half-row words of the fused kernel's circulant view (see ldpc_code_s):
// row slot sr is row r = sr mod Z of block-row brow_order[sr / Z], whose
// blocks are b0 .. b0 + d - 1; its first half holds ceil(d / 2) blocks from
// b0, its second the rest.  Empty when there is no circulant view or a
// field would overflow (13 bits of block index, 6 of length, 13 of row).
std::vector<int32_t> half_row_words(const std::vector<int32_t> &row_blk_start, const std::vector<int32_t> &brow_order,
                                    int32_t Z, int32_t m)
{
    std::vector<int32_t> out;
    if (row_blk_start.empty() || brow_order.empty() || Z < 1 || Z >= (1 << 13) || row_blk_start.back() >= (1 << 13))
        return out;
    out.resize(2 * static_cast<size_t>(m));
    for (int32_t sr = 0; sr < m; ++sr) {
        const int32_t i = brow_order[sr / Z], r = sr % Z;
        const int32_t b0 = row_blk_start[i], d = row_blk_start[i + 1] - b0, h = (d + 1) / 2;
        if (h >= (1 << 6))
            return {};
        for (int32_t half = 0; half < 2; ++half) {
            const uint32_t k0 = half ? h : 0, dh = half ? d - h : h;
            const uint32_t w = (static_cast<uint32_t>(b0) + k0) | dh << 13 | static_cast<uint32_t>(r) << 19;
            out[2 * static_cast<size_t>(sr) + half] = static_cast<int32_t>(w);
        }
    }
    return out;
}

// Greedy layers over the rows in ascending order: a row opens a new layer
// when it shares a variable with a row of the current one.  Visiting the
// layers in order, each as a parallel step, equals visiting the rows one at a
// time in order.
void layer_tables(const HostLayout &h, std::vector<int32_t> &layer_ptr, std::vector<int32_t> &layer_dmax)
{
    std::vector<int32_t> mark(h.n, -1);
    int32_t cur = 0;
    layer_ptr.assign(1, 0);
    layer_dmax.assign(1, 0);
    for (int32_t i = 0; i < h.m; ++i) {
        const int32_t b = h.row_ptr[i], e = h.row_ptr[i + 1];
        bool clash = false;
        for (int32_t k = b; k < e && !clash; ++k)
            clash = mark[h.col_idx[k]] == cur;
        if (clash) {
            ++cur;
            layer_ptr.push_back(i);
            layer_dmax.push_back(0);
        }
        for (int32_t k = b; k < e; ++k)
            mark[h.col_idx[k]] = cur;
        layer_dmax.back() = std::max(layer_dmax.back(), e - b);
    }
    layer_ptr.push_back(h.m);
    if (h.m == 0) {
        layer_ptr.assign(1, 0);
        layer_dmax.clear();
    }
}

// FNV-1a over the code's sizes, lifting size and row and column degree
// histograms: codes of one shape (whatever their edge placement) share it.
uint64_t shape_hash(const HostLayout &h, int32_t Z)
{
    uint64_t x = 1469598103934665603ull;
    auto mix = [&x](uint64_t v) {
        for (int b = 0; b < 8; ++b) {
            x ^= (v >> (8 * b)) & 0xffu;
            x *= 1099511628211ull;
        }
    };
    mix(static_cast<uint64_t>(h.m));
    mix(static_cast<uint64_t>(h.n));
    mix(static_cast<uint64_t>(h.col_idx.size()));
    mix(static_cast<uint64_t>(Z));
    std::vector<int64_t> rows(h.max_row_deg + 1, 0), cols(h.max_col_deg + 1, 0);
    for (int32_t i = 0; i < h.m; ++i)
        rows[h.row_ptr[i + 1] - h.row_ptr[i]]++;
    for (int32_t j = 0; j < h.n; ++j)
        cols[h.col_ptr[j + 1] - h.col_ptr[j]]++;
    for (int64_t v : rows)
        mix(static_cast<uint64_t>(v));
    mix(~0ull);
    for (int64_t v : cols)
        mix(static_cast<uint64_t>(v));
    return x;
}

ldpc_status upload(const HostLayout &h, const std::vector<int32_t> *qc_tab, const std::vector<int32_t> &row_blk_start,
                   int32_t Z, ldpc_code_s *c)
{
    layer_tables(h, c->layer_ptr, c->layer_dmax);
    std::vector<int32_t> brow_order, row_gmax, col_gmax;
    slot_tables(h, row_blk_start, Z, brow_order, row_gmax, col_gmax);
    const std::vector<int32_t> halves = half_row_words(row_blk_start, brow_order, Z, h.m);
    const size_t words = h.row_ptr.size() + h.col_idx.size() + h.col_ptr.size() + h.col_edge.size() +
                         (qc_tab ? qc_tab->size() : 0) + brow_order.size() + row_gmax.size() + col_gmax.size() +
                         c->layer_ptr.size() + halves.size();
    std::vector<int32_t> blob;
    blob.reserve(words);
    auto put = [&](const std::vector<int32_t> &v) {
        const size_t off = blob.size();
        blob.insert(blob.end(), v.begin(), v.end());
        return off;
    };
    const size_t o_rp = put(h.row_ptr), o_ci = put(h.col_idx), o_cp = put(h.col_ptr), o_ce = put(h.col_edge);
    const size_t o_qc = qc_tab ? put(*qc_tab) : 0;
    const size_t o_bo = put(brow_order), o_rg = put(row_gmax), o_cg = put(col_gmax), o_lp = put(c->layer_ptr);
    const size_t o_hr = put(halves);
    void *d = nullptr;
    if (hipMalloc(&d, std::max<size_t>(blob.size(), 1) * sizeof(int32_t)) != hipSuccess)
        return LDPC_ENOMEM;
    if (hipMemcpy(d, blob.data(), blob.size() * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(d);
        return LDPC_EDEVICE;
    }
    const int32_t *base = static_cast<const int32_t *>(d);
    c->d_mem = d;
    c->row_ptr = base + o_rp;
    c->col_idx = base + o_ci;
    c->col_ptr = base + o_cp;
    c->col_edge = base + o_ce;
    c->qc_tab = qc_tab ? base + o_qc : nullptr;
    c->brow_order = brow_order.empty() ? nullptr : base + o_bo;
    c->row_gmax = base + o_rg;
    c->col_gmax = base + o_cg;
    c->d_layer_ptr = base + o_lp;
    c->half_rows = halves.empty() ? nullptr : reinterpret_cast<const uint32_t *>(base + o_hr);
    c->m = h.m;
    c->n = h.n;
    c->E = static_cast<int64_t>(h.col_idx.size());
    c->max_row_deg = h.max_row_deg;
    c->max_col_deg = h.max_col_deg;
    c->shape_hash = shape_hash(h, Z);
    return LDPC_OK;
}

}  // namespace

bool ldpc::code_on_current_device(const ldpc_code_s *c)
{
    int dev = -1;
    return hipGetDevice(&dev) == hipSuccess && dev == c->device;
}

extern "C" const char *ldpc_status_str(ldpc_status s)
{
    switch (s) {
    case LDPC_OK: return "ok";
    case LDPC_EINVAL: return "invalid argument";
    case LDPC_ENOMEM: return "out of memory";
    case LDPC_EDEVICE: return "HIP runtime error";
    case LDPC_EBUSY: return "busy";
    case LDPC_EUNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

extern "C" ldpc_status ldpc_code_from_csr(int32_t m, int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                                          ldpc_code *out)
try {
    if (!out)
        return LDPC_EINVAL;
    HostLayout h;
    ldpc_status st = build_host_layout(m, n, row_ptr, col_idx, h);
    if (st != LDPC_OK)
        return st;
    auto *c = new (std::nothrow) ldpc_code_s();
    if (!c)
        return LDPC_ENOMEM;
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return LDPC_EDEVICE;
    }
    st = upload(h, nullptr, {}, 0, c);
    if (st != LDPC_OK) {
        delete c;
        return st;
    }
    *out = c;
    return LDPC_OK;
} catch (...) {
    return ldpc::status_of_exception();
}

extern "C" ldpc_status ldpc_code_from_qc(int32_t mb, int32_t nb, int32_t Z, const int32_t *shifts, ldpc_code *out)
try {
    if (!out || !shifts || mb < 1 || nb < 1 || Z < 1)
        return LDPC_EINVAL;
    if (static_cast<int64_t>(mb) * Z > INT32_MAX / 2 || static_cast<int64_t>(nb) * Z > INT32_MAX / 2)
        return LDPC_EUNSUPPORTED;
    for (int64_t k = 0; k < static_cast<int64_t>(mb) * nb; ++k)
        if (shifts[k] < -1 || shifts[k] >= Z)
            return LDPC_EINVAL;
    // CSR of the lifted matrix: row i*Z + r has, for each non-empty block
    // (i, j) in ascending j, the column j*Z + (r + s) mod Z.
    const int32_t m = mb * Z, n = nb * Z;
    std::vector<int32_t> row_ptr(m + 1, 0), col_idx;
    std::vector<int32_t> row_blk_start(mb + 1, 0), blk_col, blk_shift;
    for (int32_t i = 0; i < mb; ++i) {
        for (int32_t j = 0; j < nb; ++j)
            if (shifts[i * nb + j] >= 0) {
                blk_col.push_back(j);
                blk_shift.push_back(shifts[i * nb + j]);
            }
        row_blk_start[i + 1] = static_cast<int32_t>(blk_col.size());
    }
    const int32_t nblocks = static_cast<int32_t>(blk_col.size());
    col_idx.reserve(static_cast<size_t>(nblocks) * Z);
    for (int32_t i = 0; i < mb; ++i)
        for (int32_t r = 0; r < Z; ++r) {
            for (int32_t b = row_blk_start[i]; b < row_blk_start[i + 1]; ++b)
                col_idx.push_back(blk_col[b] * Z + (r + blk_shift[b]) % Z);
            row_ptr[i * Z + r + 1] = static_cast<int32_t>(col_idx.size());
        }
    HostLayout h;
    ldpc_status st = build_host_layout(m, n, row_ptr.data(), col_idx.data(), h);
    if (st != LDPC_OK)
        return st;
    std::vector<int32_t> col_blk_start(nb + 1, 0), col_blk;
    int32_t max_bcol = 0, max_brow = 0;
    for (int32_t j = 0; j < nb; ++j) {
        for (int32_t i = 0; i < mb; ++i)
            for (int32_t b = row_blk_start[i]; b < row_blk_start[i + 1]; ++b)
                if (blk_col[b] == j)
                    col_blk.push_back(b);
        col_blk_start[j + 1] = static_cast<int32_t>(col_blk.size());
        max_bcol = std::max(max_bcol, col_blk_start[j + 1] - col_blk_start[j]);
    }
    for (int32_t i = 0; i < mb; ++i)
        max_brow = std::max(max_brow, row_blk_start[i + 1] - row_blk_start[i]);
    std::vector<int32_t> tab;
    tab.insert(tab.end(), row_blk_start.begin(), row_blk_start.end());
    tab.insert(tab.end(), blk_col.begin(), blk_col.end());
    tab.insert(tab.end(), blk_shift.begin(), blk_shift.end());
    tab.insert(tab.end(), col_blk_start.begin(), col_blk_start.end());
    tab.insert(tab.end(), col_blk.begin(), col_blk.end());

    auto *c = new (std::nothrow) ldpc_code_s();
    if (!c)
        return LDPC_ENOMEM;
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return LDPC_EDEVICE;
    }
    st = upload(h, &tab, row_blk_start, Z, c);
    if (st != LDPC_OK) {
        delete c;
        return st;
    }
    c->is_qc = true;
    c->mb = mb;
    c->nb = nb;
    c->Z = Z;
    c->nblocks = nblocks;
    c->max_brow_deg = max_brow;
    c->max_bcol_deg = max_bcol;
    c->qc_words = static_cast<int32_t>(tab.size());
    c->h_qc_tab = std::move(tab);
    *out = c;
    return LDPC_OK;
} catch (...) {
    return ldpc::status_of_exception();
}

extern "C" ldpc_status ldpc_code_info(ldpc_code code, int32_t *m, int32_t *n, int64_t *edges)
try {
    if (!code)
        return LDPC_EINVAL;
    if (m)
        *m = code->m;
    if (n)
        *n = code->n;
    if (edges)
        *edges = code->E;
    return LDPC_OK;
} catch (...) {
    return ldpc::status_of_exception();
}

extern "C" ldpc_status ldpc_code_layers(ldpc_code code, int32_t *nlayers, int32_t *min_rows, int32_t *max_rows)
try {
    if (!code)
        return LDPC_EINVAL;
    const int32_t L = static_cast<int32_t>(code->layer_dmax.size());
    int32_t lo = L ? INT32_MAX : 0, hi = 0;
    for (int32_t l = 0; l < L; ++l) {
        const int32_t r = code->layer_ptr[l + 1] - code->layer_ptr[l];
        lo = std::min(lo, r);
        hi = std::max(hi, r);
    }
    if (nlayers)
        *nlayers = L;
    if (min_rows)
        *min_rows = lo;
    if (max_rows)
        *max_rows = hi;
    return LDPC_OK;
} catch (...) {
    return ldpc::status_of_exception();
}

extern "C" void ldpc_code_destroy(ldpc_code code)
try {
    if (!code)
        return;
    if (code->d_mem) {
        int prev = -1;
        (void)hipGetDevice(&prev);
        (void)hipSetDevice(code->device);
        (void)hipFree(code->d_mem);
        if (prev >= 0)
            (void)hipSetDevice(prev);
    }
    delete code;
} catch (...) {
}
