// Fused frame-resident decoder: one workgroup decodes one frame through all
// of its iterations with the frame's messages held in LDS, on the flooding
// schedule or (jobs with LDPC_LAYERED) the layered one.
//
// Schedule (arxiv 1812.06545, Section II; Algorithm 1): the same flooding
// two-phase iteration as the plain path, but the global barrier between the
// check-node and variable-node phases becomes a workgroup barrier, because
// the frames are independent (the frame-level parallelism of Section III-A)
// and one workgroup owns a whole frame.  HBM traffic per frame is the channel
// LLRs (read once per iteration, from L2 after the first) and the outputs.
//
// Persistent launch: workgroups pull (job, frame) items from a device counter
// until the queue is empty, so one launch decodes a batch of jobs of
// different codes, lengths and rates, and a frame that stops early frees its
// workgroup for the next item.
//
// Thread mapping: check rows are visited in slot order (for QC codes
// block-rows sorted by decreasing degree).  A wavefront's 64 rows may differ
// in degree; the wave runs the straight-line body of its largest degree and
// pads shorter rows with dummy edges carrying q = +inf, whose term is exactly
// the identity of the row's combination and whose sign is +, so every real
// message is computed with exactly the operations and rounding of the plain
// path (bit-identical results).
//
// LDS per workgroup (FrameLayout; all accesses by byte offset from its
// start): the posterior L of every variable, a word holding +inf, one
// dummy-edge slot per thread, r for every edge, and the code's tables
// (circulant codes: row and column views, and spare zero words after the
// column view so that a column body may read past its own entries).
//
// Circulant codes keep their messages in a rotated layout: the message of
// row r of block b, whose shift is s_b, sits at b*Z + ((r + s_b) mod Z),
// the offset of the edge's column inside its block-column.  A row then
// finds its message and its posterior from one offset, and a column finds
// the messages of its blocks without any modular arithmetic.
#pragma once

#include <mutex>
#include <type_traits>
#include <vector>

#include "ldpc_internal.h"
#include "minsum_kernels.h"
#include "spa_math.h"

namespace ldpc {
namespace fused {

constexpr int kMaxCodes = 16;
constexpr int kMaxJobs = 24;

// Kernel-argument copy of a code's device layout.
struct Code {
    int32_t m, n, E, Z, nblocks;
    int32_t mb, nb, qc, words;  // qc: use the circulant view (words: QC table words, 0 otherwise)
    uint32_t zmagic;            // ceil(2^32 / Z): x / Z = mulhi(x, zmagic) for x * Z < 2^32 (qc only, Z >= 2)
    const int32_t *tab, *row_ptr, *col_idx, *col_ptr, *col_edge, *brow_order, *row_gmax, *col_gmax;
    const int32_t *layer_ptr;  // layered schedule, CSR view: layer l = rows [layer_ptr[l], layer_ptr[l+1])
    int32_t nlayers;
    const uint32_t *half_rows;  // circulant view: word 2 sr + h = half h of row slot sr (or null)
};

struct Job {
    int32_t code, frames, max_iter;
    uint32_t flags;
    float ms_scale, ms_offset;  // min-sum correction (LDPC_MIN_SUM), natural LLR units
    int64_t item_begin;
    const void *llr;
    uint8_t *bits;
    int32_t *iters;
    void *post;
};

struct Batch {
    int32_t njobs, ncodes;
    int64_t nitems;
    int32_t emax, nmax, words_max, mb_max;
    Code codes[kMaxCodes];
    Job jobs[kMaxJobs];
};

// One message-sized LDS word per thread (up to 512) after the +inf word: the
// target of dummy-edge stores, so that a half row's stores need no
// exec-mask branch and its loads can all be issued first.
constexpr int kDummySlots = 512;
// Zero words after the circulant column table: a column body of length D
// reads table slots k0 .. k0 + D - 1 whatever the column's degree, which for
// the last block-columns runs up to D - 1 words past the table's end.  A zero
// word decodes to an offset inside the posteriors, a valid LDS address.
// Exact column bodies go up to degree 16.
constexpr int kColSpare = 16;

__host__ __device__ inline uint32_t align16(size_t x) { return static_cast<uint32_t>((x + 15) / 16 * 16); }

// Byte layout of a workgroup's LDS for `frames` frames (1, or 2 for the
// pair kernel) of the launch's largest n and E.  Frame k's region starts at
// k * span; inside it (offsets from its start):
//   [0, n)              posteriors L (message-sized words)
//   n                   +inf: dummy edges read their posterior there
//   n + 1 + t           dummy slot of thread t
//   r0 ..               messages r, one word per edge
// and the code's tables (int32 words) follow the last frame, at t0.
struct FrameLayout {
    uint32_t r0, span, t0;
    size_t bytes;
};
__host__ __device__ inline FrameLayout frame_layout(int64_t E, int32_t n, int32_t words, int32_t nblocks, int32_t mb,
                                                    size_t tsize, int frames = 1)
{
    FrameLayout f;
    f.r0 = align16((static_cast<size_t>(n) + 1 + kDummySlots) * tsize);
    f.span = align16(f.r0 + static_cast<size_t>(E) * tsize);
    f.t0 = f.span * static_cast<uint32_t>(frames);
    f.bytes = f.t0 + static_cast<size_t>(words + 2 * nblocks + mb + kColSpare) * sizeof(int32_t);
    return f;
}

// LDS bytes a workgroup needs for `frames` frames of this code.
__host__ __device__ inline size_t frame_lds_bytes(int64_t E, int32_t n, int32_t words, int32_t nblocks, int32_t mb,
                                                  size_t tsize, int frames = 1)
{
    return frame_layout(E, n, words, nblocks, mb, tsize, frames).bytes;
}

// Loads and stores of LDS words by byte offset from the frame's base.
template <class T>
__device__ __forceinline__ T lds_ld(const unsigned char *base, uint32_t off)
{
    return *reinterpret_cast<const T *>(base + off);
}
template <class T>
__device__ __forceinline__ void lds_st(unsigned char *base, uint32_t off, T v)
{
    *reinterpret_cast<T *>(base + off) = v;
}

__device__ __forceinline__ int32_t div_z(int32_t x, uint32_t zmagic)
{
    return static_cast<int32_t>(__umulhi(static_cast<uint32_t>(x), zmagic));
}

// Byte offsets of the messages and posteriors of one half row.
//   QC:  slot k of a half row starting at block b0 + k0:
//        c = tsize * ((r + s) mod Z) for that block's shift s,
//        message b * Z * tsize + c (rotated layout), posterior j * Z * tsize + c
//   CSR: slot k is edge e0 + k0 + k (CSR order), posterior col_idx[e]
struct RowQC {
    // The row table in LDS is followed by at least kColSpare readable words
    // (the block-row order, the column table and its spare words), so
    // offsets(k) may be read for any k < kColSpare past a row's blocks: the
    // offsets are then some values, which the caller discards.
    static constexpr bool kReadPast = true;
    uint32_t r_t;          // tsize * r
    uint32_t z_t;          // tsize * Z
    uint32_t base;         // r0 + tsize * Z * (first block of this half)
    const uint32_t *pack;  // LDS, from this half's first block: (tsize * j * Z) | (tsize * s) << 16
    __device__ __forceinline__ void offsets(int k, uint32_t &ri, uint32_t &ci) const
    {
        const uint32_t w = pack[k];
        const uint32_t c = r_t + (w >> 16);                             // in [0, 2 z_t): min picks c or c - z_t
        const uint32_t cm = __builtin_elementwise_min(c, c - z_t);
        ci = (w & 0xffffu) + cm;
        ri = base + static_cast<uint32_t>(k) * z_t + cm;
    }
};

template <int TS>
struct RowCSR {
    static constexpr bool kReadPast = false;  // col_idx ends with the last row
    uint32_t base;        // r0 + TS * (e0 + k0)
    const int32_t *cols;  // global: col_idx + e0 + k0
    __device__ __forceinline__ void offsets(int k, uint32_t &ri, uint32_t &ci) const
    {
        ri = base + static_cast<uint32_t>(k * TS);
        ci = static_cast<uint32_t>(cols[k] * TS);
    }
};

// Offsets of slot k of a half row: the real edge's, or, for a slot past its
// edges (a dummy), this thread's dummy slot and the +inf word.  Where the row
// view allows it the table is read unconditionally, so the load needs no
// exec-mask branch.
template <class Row>
__device__ __forceinline__ void slot_offsets(const Row &row, int k, bool real, uint32_t dslot, uint32_t inf_off,
                                             uint32_t &ri, uint32_t &ci)
{
    if constexpr (Row::kReadPast) {
        static_assert(kColSpare >= 16, "half rows up to 16 slots read past the row table");
        uint32_t a, b;
        row.offsets(k, a, b);
        ri = real ? a : dslot;
        ci = real ? b : inf_off;
    } else {
        if (real) {
            row.offsets(k, ri, ci);
        } else {
            ri = dslot;
            ci = inf_off;
        }
    }
}

// Per-thread places every half row of a frame shares: this thread's dummy
// slot and the +inf word (byte offsets).
struct Slots {
    uint32_t dslot, inf_off;
};

// Value of the partner lane (lane ^ 32): the other half of the same row.
// Rows are laid out so that lanes 0..31 of a wavefront hold the first halves
// of 32 consecutive rows and lanes 32..63 their second halves.
__device__ __forceinline__ uint32_t pair_swap(uint32_t v)
{
    return static_cast<uint32_t>(__shfl_xor(static_cast<int>(v), 32));
}
__device__ __forceinline__ float pair_swap(float v) { return __shfl_xor(v, 32); }
__device__ __forceinline__ double pair_swap(double v) { return __shfl_xor(v, 32); }
__device__ __forceinline__ ArithF32::Acc pair_swap(const ArithF32::Acc &v)
{
    return ArithF32::Acc{pair_swap(v.P), pair_swap(v.Q)};
}

// Value of lane ^ 16: the sibling quarter of a layered row, whose four
// quarters sit in lanes l, l + 16, l + 32 and l + 48 (l < 16).
__device__ __forceinline__ uint32_t quad_swap(uint32_t v)
{
    return static_cast<uint32_t>(__shfl_xor(static_cast<int>(v), 16));
}
__device__ __forceinline__ double quad_swap(double v) { return __shfl_xor(v, 16); }
__device__ __forceinline__ ArithF32::Acc quad_swap(const ArithF32::Acc &v)
{
    return ArithF32::Acc{__shfl_xor(v.P, 16), __shfl_xor(v.Q, 16)};
}

// One half of a check row, run-time length dh <= D, as the straight-line
// body of length D: this lane owns dh edges of the row (the first half, or
// the second), its partner lane the other half.  Slots j >= dh are
// dummies: they enter as q = +inf, whose terms are the exact identity of the
// combination (t = 1, u = 0 in FP32; phi = 0 in FP64) with a + sign; they
// read the +inf posterior word and this thread's dummy slot, and write only
// to the dummy slot.  All of the half row's offsets and loads are issued
// before its arithmetic.  The forward pass parks (part of) a_k in the edge's
// own r slot (free once q_k is formed, owned by this lane alone) instead of
// a register array; after the partner's half combination and sign are
// exchanged, the backward pass reads a_k back and overwrites the slot with
// the new message.
// TAIL: the caller has checked that every lane of the wave has dh >= D - 1,
// so only the last slot can be a dummy.
template <class A, int D, bool PAR, bool TAIL, class Row>
__device__ __forceinline__ void fused_half_row(const Row &row, int dh, unsigned char *__restrict__ s, Slots sl,
                                               uint32_t &parity)
{
    using T = typename A::T;
    typename A::Acc p[D];
    typename A::Keep kp[D];
    typename A::Acc acc = A::identity();
    uint32_t sign = 0, par = 0;
    uint32_t ri[D], ci[D];
#pragma unroll
    for (int j = 0; j < D; ++j)
        slot_offsets(row, j, (TAIL && j < D - 1) || j < dh, sl.dslot, sl.inf_off, ri[j], ci[j]);
    T lv[D], rv[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
        lv[j] = lds_ld<T>(s, ci[j]);
        rv[j] = lds_ld<T>(s, ri[j]);
    }
    // A dummy edge reads l = +inf; its slot holds a finite value (a parked
    // term or a clamped message) written by this thread in an earlier
    // iteration, so q = +inf and the edge adds nothing to the parity.
#pragma unroll
    for (int j = 0; j < D; ++j) {
        const T l = lv[j];
        if constexpr (PAR)
            par ^= static_cast<uint32_t>(l < T(0));
        const T q = l - rv[j];
        typename A::Term a_k;
        check_forward<A>(q, a_k, p[j], acc, sign);
        kp[j] = A::keep(a_k);
        lds_st<T>(s, ri[j], A::park(a_k));
    }
    const typename A::Acc s_other = pair_swap(acc);
    const uint32_t sign_total = sign ^ pair_swap(sign);
    if constexpr (PAR)
        parity |= par ^ pair_swap(par);  // a lane may hold several rows: any unsatisfied row counts
    typename A::Acc sx = A::seed(s_other);
    // Every parked value is read before the first message is stored: a
    // dummy's slot then still holds the parked dummy term (kDummyParked,
    // written by the forward pass), which needs no per-slot select.
    T pv[D];
#pragma unroll
    for (int j = 0; j < D; ++j)
        pv[j] = lds_ld<T>(s, ri[j]);
#pragma unroll
    for (int j = D - 1; j >= 0; --j) {
        const T parked = pv[j];
        const typename A::Term a_k = A::unpark(parked, kp[j]);
        const T r = check_backward<A>(a_k, p[j], sx, sign_total);
        lds_st<T>(s, ri[j], r);
    }
}

// An exact-length body.  For jobs without early stop (no syndrome), when the
// wave's half rows are all D or D - 1 long (a wave within one block-row, or
// across two of close degrees: the common case), one whose slots need no
// dummy select but the last.  (With the syndrome the same body measured
// slower on most codes, so early-stop jobs keep the general one.)
template <class A, int D, bool PAR, class Row>
__device__ __forceinline__ void fused_row_exact(const Row &row, int dh, unsigned char *__restrict__ s, Slots sl,
                                                uint32_t &parity)
{
    if constexpr (!PAR && D > 1) {
        if (__all(dh >= D - 1)) {
            fused_half_row<A, D, PAR, true>(row, dh, s, sl, parity);
            return;
        }
    }
    fused_half_row<A, D, PAR, false>(row, dh, s, sl, parity);
}

// Body selection by the wave's largest half length: exact-length bodies for
// FP32 circulant codes, the hot case; one padded body of length DB for FP64
// and for CSR codes (fewer instantiations, same results).
template <class A, int D, int DB, bool PAR, class Row>
__device__ __forceinline__ void fused_row_dispatch(int hwave, const Row &row, int dh, unsigned char *__restrict__ s,
                                                   Slots sl, uint32_t &parity)
{
    constexpr bool exact = std::is_same<A, ArithF32>::value && std::is_same<Row, RowQC>::value;
    if constexpr (!exact) {
        fused_half_row<A, DB, PAR, false>(row, dh, s, sl, parity);
    } else if constexpr (D < DB) {
        if (hwave == D)
            fused_row_exact<A, D, PAR>(row, dh, s, sl, parity);
        else
            fused_row_dispatch<A, D + 1, DB, PAR>(hwave, row, dh, s, sl, parity);
    } else {
        fused_row_exact<A, DB, PAR>(row, dh, s, sl, parity);
    }
}

// One quarter of a layered check row (Section II, Algorithm 2, with the
// layered combination order of spa_math.h): as layered_half_row, over this
// lane's quarter (run-time length dq <= D); the quarter combinations are
// exchanged in two steps, with the sibling quarter (lane ^ 16) and then
// between the halves (lane ^ 32), which gives every lane O_i in the same
// association as the streaming layer kernel.
template <class A, int D, class Row>
__device__ __forceinline__ void layered_quarter_row(const Row &row, int dq, unsigned char *__restrict__ s, Slots sl)
{
    using T = typename A::T;
    typename A::Acc p[D];
    typename A::Keep kp[D];
    typename A::Acc acc = A::identity();
    uint32_t sign = 0;
    uint32_t ri[D], ci[D];
#pragma unroll
    for (int j = 0; j < D; ++j)
        slot_offsets(row, j, j < dq, sl.dslot, sl.inf_off, ri[j], ci[j]);
    T lv[D], rv[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
        lv[j] = lds_ld<T>(s, ci[j]);
        rv[j] = lds_ld<T>(s, ri[j]);
    }
#pragma unroll
    for (int j = 0; j < D; ++j) {
        const T q = lv[j] - rv[j];  // +inf for a dummy
        typename A::Term a_k;
        check_forward<A>(q, a_k, p[j], acc, sign);
        kp[j] = A::keep(a_k);
        lds_st<T>(s, ri[j], A::park(a_k));
        lds_st<T>(s, ci[j], q);
    }
    const typename A::Acc c_sib = quad_swap(acc);
    const typename A::Acc c_other = pair_swap(A::merge(acc, c_sib));  // the other half's combination
    typename A::Acc sx = A::seed(A::merge(c_sib, c_other));
    const uint32_t sign_half = sign ^ quad_swap(sign);
    const uint32_t sign_total = sign_half ^ pair_swap(sign_half);
#pragma unroll
    for (int j = D - 1; j >= 0; --j) {
        const bool real = j < dq;
        const T parked = lds_ld<T>(s, ri[j]);  // a dummy's slot is valid; its value may be a later dummy's message
        const typename A::Term a_k = A::unpark(real ? parked : T(A::kDummyParked), kp[j]);
        const T r = check_backward<A>(a_k, p[j], sx, sign_total);
        const T q = lds_ld<T>(s, ci[j]);
        lds_st<T>(s, ri[j], r);
        lds_st<T>(s, ci[j], q + r);
    }
}

template <class A, int D, int DB, class Row>
__device__ __forceinline__ void layered_quarter_dispatch(int qwave, const Row &row, int dq,
                                                         unsigned char *__restrict__ s, Slots sl)
{
    constexpr bool exact = std::is_same<A, ArithF32>::value && std::is_same<Row, RowQC>::value;
    if constexpr (!exact) {
        layered_quarter_row<A, DB>(row, dq, s, sl);
    } else if constexpr (D < DB) {
        if (qwave == D)
            layered_quarter_row<A, D>(row, dq, s, sl);
        else
            layered_quarter_dispatch<A, D + 1, DB>(qwave, row, dq, s, sl);
    } else {
        layered_quarter_row<A, DB>(row, dq, s, sl);
    }
}

// This lane's quarter of a row of degree d: its first position k0 and length.
__device__ __forceinline__ void quarter_span(int32_t d, int part, int32_t &k0, int32_t &dq)
{
    const Quarters Q = quarters(d);
    k0 = part == 0 ? 0 : part == 1 ? Q.q1 : part == 2 ? Q.h : Q.q3;
    dq = (part == 0 ? Q.q1 : part == 1 ? Q.h : part == 2 ? Q.q3 : d) - k0;
}

// One half of a check row under the min-sum rule, flooding or (LAYERED)
// layered, padded body of length D: each lane keeps the running minimum
// state of its half, the partner lanes merge theirs, and every real edge gets
// one select.  k0 is the half's first position in the row (positions identify
// the smallest message).  Flooding folds the parity of the previous decision
// into `parity` (as fused_half_row); layered writes L = q + r at once.
template <class A, int D, bool LAYERED, class Row>
__device__ __forceinline__ void ms_half_row(const Row &row, int k0, int dh, unsigned char *__restrict__ s, Slots sl,
                                            uint32_t &parity, typename A::T scale, typename A::T offset)
{
    using T = typename A::T;
    T q[D];
    MinState<T> st;
    min_init(st);
    uint32_t par = 0;
    // dummy edges enter as q = +inf, which leaves the minimum state
    // unchanged, and store their messages in this thread's dummy slot; they
    // read (and, layered, write back) the +inf posterior word, as in
    // fused_half_row: a min-sum message is clamped too, so the dummy slot
    // always holds a finite value
    uint32_t ri[D], ci[D];
#pragma unroll
    for (int j = 0; j < D; ++j)
        slot_offsets(row, j, j < dh, sl.dslot, sl.inf_off, ri[j], ci[j]);
    T lv[D], rv[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
        lv[j] = lds_ld<T>(s, ci[j]);
        rv[j] = lds_ld<T>(s, ri[j]);
    }
#pragma unroll
    for (int j = 0; j < D; ++j) {
        if (!LAYERED)
            par ^= static_cast<uint32_t>(lv[j] < T(0));
        q[j] = lv[j] - rv[j];
        min_add(st, q[j], k0 + j);
    }
    const T o_m1 = pair_swap(st.m1), o_m2 = pair_swap(st.m2);
    const int32_t o_idx = static_cast<int32_t>(pair_swap(static_cast<uint32_t>(st.idx)));
    const uint32_t o_neg = pair_swap(st.neg);
    min_merge(st, o_m1, o_m2, o_idx, o_neg);
    if (!LAYERED)
        parity |= par ^ pair_swap(par);
#pragma unroll
    for (int j = 0; j < D; ++j) {
        const T r = min_message<A>(st, q[j], k0 + j, scale, offset);
        lds_st<T>(s, ri[j], r);
        if (LAYERED)
            lds_st<T>(s, ci[j], q[j] + r);
    }
}

// Column sum L = Lch + sum of r in ascending row order, run-time degree dv <= D
// (dummy edges read a valid word and are not added).  SAFE0: every table
// slot up to D - 1 past the column's start is readable and decodes to a valid
// offset (the circulant tables in LDS end with kColSpare zero words), so all
// D slots are read unconditionally at constant offsets; otherwise dummies
// read offset 0.  edge(k) is the byte offset of the column's k-th message.
template <class A, int D, bool SAFE0, bool FULL, class Edge>
__device__ __forceinline__ typename A::T fused_col(const Edge &edge, int dv, typename A::T acc,
                                                   const unsigned char *__restrict__ s)
{
    using T = typename A::T;
    static_assert(!SAFE0 || D <= kColSpare, "column body longer than the spare words cover");
    T rv[D > 0 ? D : 1];
#pragma unroll
    for (int k = 0; k < D; ++k)
        rv[k] = SAFE0 || FULL ? lds_ld<T>(s, edge(k)) : lds_ld<T>(s, k < dv ? edge(k) : 0u);
#pragma unroll
    for (int k = 0; k < D; ++k)
        acc = FULL || k < dv ? acc + rv[k] : acc;
    return acc;
}

template <class A, int D, bool SAFE0, class Edge>
__device__ __forceinline__ typename A::T fused_col_dispatch(int dwave, const Edge &edge, int dv, typename A::T acc,
                                                            const unsigned char *__restrict__ s)
{
    using T = typename A::T;
    if constexpr (!std::is_same<A, ArithF32>::value) {
        for (int k = 0; k < dv; ++k)
            acc += lds_ld<T>(s, edge(k));
        return acc;
    } else if constexpr (D <= kColSpare) {
        if (dwave == D) {
            // FULL: every column of the wave has degree D (no slot to skip)
            if (__all(dv == D))
                return fused_col<A, D, SAFE0, true>(edge, dv, acc, s);
            return fused_col<A, D, SAFE0, false>(edge, dv, acc, s);
        }
        return fused_col_dispatch<A, D + 1, SAFE0>(dwave, edge, dv, acc, s);
    } else {
        for (int k = 0; k < dv; ++k)
            acc += lds_ld<T>(s, edge(k));
        return acc;
    }
}

// Places of one frame's data in LDS, for the launch.
struct FrameView {
    unsigned char *s;      // the frame's LDS (posteriors at offset 0)
    uint32_t r0;           // byte offset of the messages
    const int32_t *tab;    // the code's tables (raw QC tables, then the views below)
    Slots slots;
};

// Messages r start at 0 (before the first iteration, or pass, there are
// none), and so does this thread's dummy slot: the first iteration then
// forms q = L - 0 = L exactly, as the streaming kernels' first iteration,
// with the same code as every later one.
template <class T>
__device__ __forceinline__ void start_messages(const Code &c, const FrameView &fv)
{
    T *sR = reinterpret_cast<T *>(fv.s + fv.r0);
    for (int e = static_cast<int>(threadIdx.x); e < c.E; e += static_cast<int>(blockDim.x))
        sR[e] = T(0);
    lds_st<T>(fv.s, fv.slots.dslot, T(0));
}

// QC table views in LDS (raw tables of `words` words first):
//   [words, +nblocks)             row view: pack word of block b
//   [.., +mb)                     brow_order
//   [.., +nblocks)                column view: r0 + tsize * Z * b for block-column slot w
//   [.., +kColSpare)              zero words
// Kernel instances: one for any batch, and two compiled with one schedule's
// sum-product rows on circulant views only (no min-sum, no CSR rows, no
// other schedule), for batches whose jobs all allow it.
enum Instance { kAnyJob = 0, kFloodQC = 1, kLayeredQC = 2, kMinSumQC = 3 };

// QCF: every job of the launch is sum-product flooding on a circulant view
// (no min-sum or CSR rows compiled in); MSQ: every job is min-sum flooding on
// a circulant view (no sum-product or CSR rows compiled in).
template <class A, int DB, bool QCF = false, bool MSQ = false>
__device__ __forceinline__ void decode_frame(const Code &c, const Job &job, int64_t f, const FrameView &fv)
{
    using T = typename A::T;
    constexpr uint32_t TS = sizeof(T);
    const int tid = static_cast<int>(threadIdx.x), NT = static_cast<int>(blockDim.x);
    const int32_t m = c.m, n = c.n, Z = c.Z;
    const T *llr = static_cast<const T *>(job.llr) + f * n;
    unsigned char *s = fv.s;
    T *sL = reinterpret_cast<T *>(s);
    const int32_t *rbs = fv.tab;
    const int32_t *cbs = fv.tab + (c.mb + 1) + 2 * c.nblocks;
    const uint32_t *pack = reinterpret_cast<const uint32_t *>(fv.tab + c.words);
    const int32_t *border = fv.tab + c.words + c.nblocks;
    const uint32_t *cpack = reinterpret_cast<const uint32_t *>(border + c.mb);
    const uint32_t z_t = TS * static_cast<uint32_t>(Z);

    for (int j = tid; j < n; j += NT)
        sL[j] = llr[j] * T(A::kIn);
    start_messages<T>(c, fv);
    __syncthreads();

    const bool es = (job.flags & LDPC_EARLY_STOP) != 0;
    const bool ms = MSQ || (!QCF && (job.flags & LDPC_MIN_SUM) != 0);
    const T ms_scale = static_cast<T>(job.ms_scale), ms_offset = static_cast<T>(job.ms_offset * A::kIn);
    int32_t it = job.max_iter;
    for (int32_t t = 1; t <= job.max_iter; ++t) {
        uint32_t parity = 0;
        // two lanes per check row: in each wavefront, lane l < 32 takes the
        // first half of slot rb + l and lane l + 32 its second half
        const int lane = tid & 63, half = lane >> 5;
        for (int rb = (tid >> 6) * 32; rb < m; rb += (NT >> 6) * 32) {
            const int dwave = c.row_gmax[__builtin_amdgcn_readfirstlane(rb) >> 5];
            const int sr = rb + (lane & 31);
            if (dwave == 0 || sr >= m)
                continue;
            const int hwave = (dwave + 1) >> 1;
            if constexpr (QCF) {
                // the half row's first block, length and row in one word
                const uint32_t w = c.half_rows[2 * sr + half];
                const uint32_t bk = w & 0x1fffu, r = w >> 19;
                const int32_t dh = static_cast<int32_t>((w >> 13) & 63u);
                const RowQC row{TS * r, z_t, fv.r0 + z_t * bk, pack + bk};
                if (es)
                    fused_row_dispatch<A, 1, DB / 2, true>(hwave, row, dh, s, fv.slots, parity);
                else
                    fused_row_dispatch<A, 1, DB / 2, false>(hwave, row, dh, s, fv.slots, parity);
            } else if (c.qc) {
                const int32_t si = div_z(sr, c.zmagic);
                const int32_t r = sr - si * Z;
                const int32_t i = border[si];
                const int32_t b0 = rbs[i], d = rbs[i + 1] - b0, h = (d + 1) >> 1;
                const int32_t k0 = half ? h : 0, dh = half ? d - h : h;
                const RowQC row{TS * static_cast<uint32_t>(r), z_t, fv.r0 + z_t * static_cast<uint32_t>(b0 + k0),
                                pack + b0 + k0};
                if (ms)
                    ms_half_row<A, DB / 2, false>(row, k0, dh, s, fv.slots, parity, ms_scale, ms_offset);
                else if constexpr (!MSQ) {
                    if (es)
                        fused_row_dispatch<A, 1, DB / 2, true>(hwave, row, dh, s, fv.slots, parity);
                    else
                        fused_row_dispatch<A, 1, DB / 2, false>(hwave, row, dh, s, fv.slots, parity);
                }
            } else if constexpr (!MSQ) {
                const int32_t e0 = c.row_ptr[sr], d = c.row_ptr[sr + 1] - e0, h = (d + 1) >> 1;
                const int32_t k0 = half ? h : 0, dh = half ? d - h : h;
                const RowCSR<TS> row{fv.r0 + TS * static_cast<uint32_t>(e0 + k0), c.col_idx + e0 + k0};
                if (ms)
                    ms_half_row<A, DB / 2, false>(row, k0, dh, s, fv.slots, parity, ms_scale, ms_offset);
                else if (es)
                    fused_row_dispatch<A, 1, DB / 2, true>(hwave, row, dh, s, fv.slots, parity);
                else
                    fused_row_dispatch<A, 1, DB / 2, false>(hwave, row, dh, s, fv.slots, parity);
            }
        }
        // The syndrome of x^(t-1) is formed only under early stop (min-sum
        // rows form it always, unused without).
        if (es) {
            if (!__syncthreads_or(static_cast<int>(parity))) {  // a codeword: stop at t-1, keep L^(t-1)
                it = t - 1;
                break;
            }
        } else {
            __syncthreads();
        }
        for (int j = tid; j < n; j += NT) {
            const int dwave = c.col_gmax[__builtin_amdgcn_readfirstlane(j) >> 6];
            const T acc = llr[j] * T(A::kIn);
            T v;
            if (QCF || MSQ || c.qc) {
                const int32_t bj = div_z(j, c.zmagic);
                const uint32_t cc_t = TS * static_cast<uint32_t>(j - bj * Z);
                const int32_t k0 = cbs[bj];
                auto edge = [&](int k) { return cpack[k0 + k] + cc_t; };
                v = fused_col_dispatch<A, 0, true>(dwave, edge, cbs[bj + 1] - k0, acc, s);
            } else {
                const int32_t k0 = c.col_ptr[j];
                auto edge = [&](int k) { return fv.r0 + TS * static_cast<uint32_t>(c.col_edge[k0 + k]); };
                v = fused_col_dispatch<A, 0, false>(dwave, edge, c.col_ptr[j + 1] - k0, acc, s);
            }
            sL[j] = v;
        }
        __syncthreads();
    }
    uint8_t *bits = job.bits + f * n;
    T *post = job.post ? static_cast<T *>(job.post) + f * n : nullptr;
    for (int j = tid; j < n; j += NT) {
        const T v = sL[j];
        bits[j] = static_cast<uint8_t>(v < T(0));
        if (post)
            post[j] = it == 0 ? llr[j] : v * T(A::kOut);
    }
    if (tid == 0)
        job.iters[f] = it;
}

// One frame under the layered schedule: check rows are visited in ascending
// order, one layer at a time (QC codes: one block-row, Z rows; other codes:
// the code's layer table), the rows of a layer in parallel with two lanes
// each and a workgroup barrier between layers.  With early stop the syndrome
// of [L < 0] is tested before the first pass and after every pass but the
// last.  Each row's arithmetic is the plain layered path's, bit for bit.
// QCL: every job of the launch is sum-product layered on a circulant view
// (no min-sum or CSR rows compiled in).
template <class A, int DB, bool QCL = false>
__device__ __forceinline__ void decode_frame_layered(const Code &c, const Job &job, int64_t f, const FrameView &fv)
{
    using T = typename A::T;
    constexpr uint32_t TS = sizeof(T);
    const int tid = static_cast<int>(threadIdx.x), NT = static_cast<int>(blockDim.x);
    const int lane = tid & 63, half = lane >> 5, wave = tid >> 6, nwaves = NT >> 6;
    const int32_t m = c.m, n = c.n, Z = c.Z;
    const T *llr = static_cast<const T *>(job.llr) + f * n;
    unsigned char *s = fv.s;
    T *sL = reinterpret_cast<T *>(s);
    const int32_t *rbs = fv.tab;
    const uint32_t *pack = reinterpret_cast<const uint32_t *>(fv.tab + c.words);
    const uint32_t z_t = TS * static_cast<uint32_t>(Z);

    for (int j = tid; j < n; j += NT)
        sL[j] = llr[j] * T(A::kIn);
    start_messages<T>(c, fv);
    __syncthreads();

    // View of one half of row sr (natural order).
    auto qc_half = [&](int32_t i, int32_t r, int32_t &d, int32_t &k0, int32_t &dh) {
        const int32_t b0 = rbs[i];
        d = rbs[i + 1] - b0;
        const int32_t h = (d + 1) >> 1;
        k0 = half ? h : 0;
        dh = half ? d - h : h;
        return RowQC{TS * static_cast<uint32_t>(r), z_t, fv.r0 + z_t * static_cast<uint32_t>(b0 + k0), pack + b0 + k0};
    };

    // 1 if some row is unsatisfied by [sL < 0]: each lane takes one half of a
    // row, partner lanes combine their parities.  A wavefront stops at its
    // first group of 32 rows holding an unsatisfied one (the answer is then
    // known; in most passes that is the first group).
    auto unsatisfied = [&]() -> int {
        uint32_t bad = 0;
        for (int rb = wave * 32; rb < m && !__any(static_cast<int>(bad)); rb += nwaves * 32) {
            const int sr = rb + (lane & 31);
            uint32_t par = 0;
            if (sr < m) {
                if (QCL || c.qc) {
                    const int32_t si = div_z(sr, c.zmagic);
                    int32_t d, k0, dh;
                    const RowQC row = qc_half(si, sr - si * Z, d, k0, dh);
                    for (int32_t k = 0; k < dh; ++k) {
                        uint32_t ri, ci;
                        row.offsets(k, ri, ci);
                        par ^= static_cast<uint32_t>(lds_ld<T>(s, ci) < T(0));
                    }
                } else {
                    const int32_t e0 = c.row_ptr[sr], d = c.row_ptr[sr + 1] - e0, h = (d + 1) >> 1;
                    const int32_t k0 = half ? h : 0, dh = half ? d - h : h;
                    for (int32_t k = 0; k < dh; ++k)
                        par ^= static_cast<uint32_t>(sL[c.col_idx[e0 + k0 + k]] < T(0));
                }
            }
            bad |= par ^ pair_swap(par);
        }
        return __syncthreads_or(static_cast<int>(bad));
    };

    const bool es = (job.flags & LDPC_EARLY_STOP) != 0;
    const bool ms = !QCL && (job.flags & LDPC_MIN_SUM) != 0;
    const T ms_scale = static_cast<T>(job.ms_scale), ms_offset = static_cast<T>(job.ms_offset * A::kIn);
    uint32_t no_parity = 0;
    int32_t it = job.max_iter;
    if (es && !unsatisfied()) {
        it = 0;
    } else {
        for (int32_t t = 1; t <= job.max_iter; ++t) {
            // min-sum rows: two lanes each (32 rows per wavefront); sum-product
            // rows: four lanes each (16 rows per wavefront)
            const int rows_per_wave = ms ? 32 : 16;
            const int part = lane >> 4;
            if (QCL || c.qc) {
                for (int32_t i = 0; i < c.mb; ++i) {
                    for (int rb = wave * rows_per_wave; rb < Z; rb += nwaves * rows_per_wave) {
                        const int r = rb + (lane & (rows_per_wave - 1));
                        if (r >= Z)
                            continue;
                        if (ms) {
                            int32_t d, k0, dh;
                            const RowQC row = qc_half(i, r, d, k0, dh);
                            if (d > 0)
                                ms_half_row<A, DB / 2, true>(row, k0, dh, s, fv.slots, no_parity, ms_scale,
                                                             ms_offset);
                        } else {
                            const int32_t b0 = rbs[i], d = rbs[i + 1] - b0;
                            if (d == 0)
                                continue;
                            int32_t k0, dq;
                            quarter_span(d, part, k0, dq);
                            const RowQC row{TS * static_cast<uint32_t>(r), z_t,
                                            fv.r0 + z_t * static_cast<uint32_t>(b0 + k0), pack + b0 + k0};
                            layered_quarter_dispatch<A, 1, DB / 4>(quarters(d).q1, row, dq, s, fv.slots);
                        }
                    }
                    __syncthreads();
                }
            } else {
                for (int32_t l = 0; l < c.nlayers; ++l) {
                    const int32_t row0 = c.layer_ptr[l], rows = c.layer_ptr[l + 1] - row0;
                    for (int rb = wave * rows_per_wave; rb < rows; rb += nwaves * rows_per_wave) {
                        const int slot = rb + (lane & (rows_per_wave - 1));
                        if (slot >= rows)
                            continue;
                        const int32_t e0 = c.row_ptr[row0 + slot], d = c.row_ptr[row0 + slot + 1] - e0;
                        if (d == 0)
                            continue;
                        if (ms) {
                            const int32_t h = (d + 1) >> 1;
                            const int32_t k0 = half ? h : 0, dh = half ? d - h : h;
                            const RowCSR<TS> row{fv.r0 + TS * static_cast<uint32_t>(e0 + k0), c.col_idx + e0 + k0};
                            ms_half_row<A, DB / 2, true>(row, k0, dh, s, fv.slots, no_parity, ms_scale, ms_offset);
                        } else {
                            int32_t k0, dq;
                            quarter_span(d, part, k0, dq);
                            const RowCSR<TS> row{fv.r0 + TS * static_cast<uint32_t>(e0 + k0), c.col_idx + e0 + k0};
                            layered_quarter_dispatch<A, 1, DB / 4>(quarters(d).q1, row, dq, s, fv.slots);
                        }
                    }
                    __syncthreads();
                }
            }
            if (es && t < job.max_iter && !unsatisfied()) {
                it = t;
                break;
            }
        }
    }
    uint8_t *bits = job.bits + f * n;
    T *post = job.post ? static_cast<T *>(job.post) + f * n : nullptr;
    for (int j = tid; j < n; j += NT) {
        const T v = sL[j];
        bits[j] = static_cast<uint8_t>(v < T(0));
        if (post)
            post[j] = it == 0 ? llr[j] : v * T(A::kOut);
    }
    if (tid == 0)
        job.iters[f] = it;
}

// The code's tables in LDS (see decode_frame): the raw QC tables, then the
// row view (pack words), the block-row order, the column view (message
// offsets from a frame's base) and the spare zero words.  Ends with a
// workgroup barrier.
template <uint32_t TS>
__device__ __forceinline__ void load_tables(const Code &c, int32_t *__restrict__ sTab, uint32_t r0)
{
    for (int w = threadIdx.x; w < c.words; w += blockDim.x)
        sTab[w] = c.tab[w];
    if (c.qc) {
        const uint32_t Z = static_cast<uint32_t>(c.Z);
        const int32_t *bcol = c.tab + (c.mb + 1);
        const int32_t *bsh = bcol + c.nblocks;
        for (int w = threadIdx.x; w < c.nblocks; w += blockDim.x)
            sTab[c.words + w] = static_cast<int32_t>((TS * static_cast<uint32_t>(bcol[w]) * Z) |
                                                     ((TS * static_cast<uint32_t>(bsh[w])) << 16));
        for (int w = threadIdx.x; w < c.mb; w += blockDim.x)
            sTab[c.words + c.nblocks + w] = c.brow_order[w];
        // the column phase's view: block-column slot w holds block cb[w]
        const int32_t *cb = bsh + c.nblocks + (c.nb + 1);
        for (int w = threadIdx.x; w < c.nblocks; w += blockDim.x)
            sTab[c.words + c.nblocks + c.mb + w] = static_cast<int32_t>(r0 + TS * Z * static_cast<uint32_t>(cb[w]));
        if (threadIdx.x < kColSpare)  // readable words past the column table's end
            sTab[c.words + 2 * c.nblocks + c.mb + threadIdx.x] = 0;
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Two frames per workgroup (flooding, sum-product): every lane runs its half
// rows and columns for two frames of one job at once, so the offsets, table
// reads, dummy handling and loop bookkeeping of a slot serve both frames.
// Each frame's arithmetic, in its own LDS region, is exactly the one-frame
// kernel's (and so the plain path's), bit for bit.

// fused_half_row for frames at s0 and s1 (see there).
template <class A, int D, class Row>
__device__ __forceinline__ void fused_half_row2(const Row &row, int dh, unsigned char *__restrict__ s0,
                                                unsigned char *__restrict__ s1, Slots sl, uint32_t &parity0,
                                                uint32_t &parity1)
{
    using T = typename A::T;
    typename A::Acc p0[D], p1[D];
    typename A::Keep kp0[D], kp1[D];
    typename A::Acc acc0 = A::identity(), acc1 = A::identity();
    uint32_t sign0 = 0, sign1 = 0, par0 = 0, par1 = 0;
    uint32_t ri[D], ci[D];
#pragma unroll
    for (int j = 0; j < D; ++j)
        slot_offsets(row, j, j < dh, sl.dslot, sl.inf_off, ri[j], ci[j]);
    T lv0[D], rv0[D], lv1[D], rv1[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
        lv0[j] = lds_ld<T>(s0, ci[j]);
        rv0[j] = lds_ld<T>(s0, ri[j]);
        lv1[j] = lds_ld<T>(s1, ci[j]);
        rv1[j] = lds_ld<T>(s1, ri[j]);
    }
#pragma unroll
    for (int j = 0; j < D; ++j) {
        par0 ^= static_cast<uint32_t>(lv0[j] < T(0));
        par1 ^= static_cast<uint32_t>(lv1[j] < T(0));
        typename A::Term a0, a1;
        check_forward<A>(lv0[j] - rv0[j], a0, p0[j], acc0, sign0);
        check_forward<A>(lv1[j] - rv1[j], a1, p1[j], acc1, sign1);
        kp0[j] = A::keep(a0);
        kp1[j] = A::keep(a1);
        lds_st<T>(s0, ri[j], A::park(a0));
        lds_st<T>(s1, ri[j], A::park(a1));
    }
    const typename A::Acc o0 = pair_swap(acc0), o1 = pair_swap(acc1);
    const uint32_t st0 = sign0 ^ pair_swap(sign0), st1 = sign1 ^ pair_swap(sign1);
    parity0 |= par0 ^ pair_swap(par0);
    parity1 |= par1 ^ pair_swap(par1);
    typename A::Acc x0 = A::seed(o0), x1 = A::seed(o1);
    // Every parked value is read before the first message is stored: a
    // dummy's slot then still holds the parked dummy term (kDummyParked,
    // written by the forward pass), which needs no per-slot select.
    T v0[D], v1[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
        v0[j] = lds_ld<T>(s0, ri[j]);
        v1[j] = lds_ld<T>(s1, ri[j]);
    }
#pragma unroll
    for (int j = D - 1; j >= 0; --j) {
        const typename A::Term a0 = A::unpark(v0[j], kp0[j]);
        const typename A::Term a1 = A::unpark(v1[j], kp1[j]);
        const T r0 = check_backward<A>(a0, p0[j], x0, st0);
        const T r1 = check_backward<A>(a1, p1[j], x1, st1);
        lds_st<T>(s0, ri[j], r0);
        lds_st<T>(s1, ri[j], r1);
    }
}

template <class A, int D, int DB, class Row>
__device__ __forceinline__ void fused_row_dispatch2(int hwave, const Row &row, int dh, unsigned char *__restrict__ s0,
                                                    unsigned char *__restrict__ s1, Slots sl, uint32_t &parity0,
                                                    uint32_t &parity1)
{
    constexpr bool exact = std::is_same<Row, RowQC>::value;
    if constexpr (!exact) {
        fused_half_row2<A, DB>(row, dh, s0, s1, sl, parity0, parity1);
    } else if constexpr (D < DB) {
        if (hwave == D)
            fused_half_row2<A, D>(row, dh, s0, s1, sl, parity0, parity1);
        else
            fused_row_dispatch2<A, D + 1, DB>(hwave, row, dh, s0, s1, sl, parity0, parity1);
    } else {
        fused_half_row2<A, DB>(row, dh, s0, s1, sl, parity0, parity1);
    }
}

// fused_col for frames at s0 and s1.
template <class A, int D, bool SAFE0, class Edge>
__device__ __forceinline__ void fused_col2(const Edge &edge, int dv, typename A::T &acc0, typename A::T &acc1,
                                           const unsigned char *__restrict__ s0, const unsigned char *__restrict__ s1)
{
    using T = typename A::T;
    static_assert(!SAFE0 || D <= kColSpare, "column body longer than the spare words cover");
    T rv0[D > 0 ? D : 1], rv1[D > 0 ? D : 1];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const uint32_t o = SAFE0 ? edge(k) : (k < dv ? edge(k) : 0u);
        rv0[k] = lds_ld<T>(s0, o);
        rv1[k] = lds_ld<T>(s1, o);
    }
#pragma unroll
    for (int k = 0; k < D; ++k) {
        acc0 = k < dv ? acc0 + rv0[k] : acc0;
        acc1 = k < dv ? acc1 + rv1[k] : acc1;
    }
}

template <class A, int D, bool SAFE0, class Edge>
__device__ __forceinline__ void fused_col_dispatch2(int dwave, const Edge &edge, int dv, typename A::T &acc0,
                                                    typename A::T &acc1, const unsigned char *__restrict__ s0,
                                                    const unsigned char *__restrict__ s1)
{
    using T = typename A::T;
    if constexpr (SAFE0 && D <= kColSpare) {
        if (dwave == D)
            return fused_col2<A, D, SAFE0>(edge, dv, acc0, acc1, s0, s1);
        return fused_col_dispatch2<A, D + 1, SAFE0>(dwave, edge, dv, acc0, acc1, s0, s1);
    } else {
        for (int k = 0; k < dv; ++k) {
            const uint32_t o = edge(k);
            acc0 += lds_ld<T>(s0, o);
            acc1 += lds_ld<T>(s1, o);
        }
    }
}

// Frames f0 and f0 + 1 of a flooding sum-product job (with has1 false only
// frame f0: the second region then decodes a copy of it, whose results are
// not written).  Early stop is per frame: a frame whose decision is a
// codeword keeps its posteriors from then on (its column updates are
// skipped) and leaves the loop's work to the other frame.
template <class A, int DB>
__device__ __forceinline__ void decode_frame_pair(const Code &c, const Job &job, int64_t f0, bool has1,
                                                  const FrameView &fv0, const FrameView &fv1)
{
    using T = typename A::T;
    constexpr uint32_t TS = sizeof(T);
    const int tid = static_cast<int>(threadIdx.x), NT = static_cast<int>(blockDim.x);
    const int32_t m = c.m, n = c.n, Z = c.Z;
    const T *llr0 = static_cast<const T *>(job.llr) + f0 * n;
    const T *llr1 = has1 ? llr0 + n : llr0;
    unsigned char *s0 = fv0.s, *s1 = fv1.s;
    T *sL0 = reinterpret_cast<T *>(s0), *sL1 = reinterpret_cast<T *>(s1);
    const int32_t *rbs = fv0.tab;
    const int32_t *cbs = fv0.tab + (c.mb + 1) + 2 * c.nblocks;
    const uint32_t *pack = reinterpret_cast<const uint32_t *>(fv0.tab + c.words);
    const int32_t *border = fv0.tab + c.words + c.nblocks;
    const uint32_t *cpack = reinterpret_cast<const uint32_t *>(border + c.mb);
    const uint32_t z_t = TS * static_cast<uint32_t>(Z);

    for (int j = tid; j < n; j += NT) {
        sL0[j] = llr0[j] * T(A::kIn);
        sL1[j] = llr1[j] * T(A::kIn);
    }
    start_messages<T>(c, fv0);
    start_messages<T>(c, fv1);
    __syncthreads();

    const bool es = (job.flags & LDPC_EARLY_STOP) != 0;
    int32_t it0 = job.max_iter, it1 = job.max_iter;
    bool run0 = true, run1 = true;
    for (int32_t t = 1; t <= job.max_iter; ++t) {
        uint32_t parity0 = 0, parity1 = 0;
        const int lane = tid & 63, half = lane >> 5;
        for (int rb = (tid >> 6) * 32; rb < m; rb += (NT >> 6) * 32) {
            const int dwave = c.row_gmax[__builtin_amdgcn_readfirstlane(rb) >> 5];
            const int sr = rb + (lane & 31);
            if (dwave == 0 || sr >= m)
                continue;
            const int hwave = (dwave + 1) >> 1;
            if (c.qc) {
                const int32_t si = div_z(sr, c.zmagic);
                const int32_t r = sr - si * Z;
                const int32_t i = border[si];
                const int32_t b0 = rbs[i], d = rbs[i + 1] - b0, h = (d + 1) >> 1;
                const int32_t k0 = half ? h : 0, dh = half ? d - h : h;
                const RowQC row{TS * static_cast<uint32_t>(r), z_t, fv0.r0 + z_t * static_cast<uint32_t>(b0 + k0),
                                pack + b0 + k0};
                fused_row_dispatch2<A, 1, DB / 2>(hwave, row, dh, s0, s1, fv0.slots, parity0, parity1);
            } else {
                const int32_t e0 = c.row_ptr[sr], d = c.row_ptr[sr + 1] - e0, h = (d + 1) >> 1;
                const int32_t k0 = half ? h : 0, dh = half ? d - h : h;
                const RowCSR<TS> row{fv0.r0 + TS * static_cast<uint32_t>(e0 + k0), c.col_idx + e0 + k0};
                fused_row_dispatch2<A, 1, DB / 2>(hwave, row, dh, s0, s1, fv0.slots, parity0, parity1);
            }
        }
        const int unsat0 = __syncthreads_or(static_cast<int>(parity0));
        const int unsat1 = __syncthreads_or(static_cast<int>(parity1));
        if (es) {  // as decode_frame, per frame: x^(t-1) a codeword -> stop at t-1, keep L^(t-1)
            if (run0 && !unsat0) {
                it0 = t - 1;
                run0 = false;
            }
            if (run1 && !unsat1) {
                it1 = t - 1;
                run1 = false;
            }
            if (!run0 && !run1)
                break;
        }
        for (int j = tid; j < n; j += NT) {
            const int dwave = c.col_gmax[__builtin_amdgcn_readfirstlane(j) >> 6];
            T v0 = llr0[j] * T(A::kIn), v1 = llr1[j] * T(A::kIn);
            if (c.qc) {
                const int32_t bj = div_z(j, c.zmagic);
                const uint32_t cc_t = TS * static_cast<uint32_t>(j - bj * Z);
                const int32_t k0 = cbs[bj];
                auto edge = [&](int k) { return cpack[k0 + k] + cc_t; };
                fused_col_dispatch2<A, 0, true>(dwave, edge, cbs[bj + 1] - k0, v0, v1, s0, s1);
            } else {
                const int32_t k0 = c.col_ptr[j];
                auto edge = [&](int k) { return fv0.r0 + TS * static_cast<uint32_t>(c.col_edge[k0 + k]); };
                fused_col_dispatch2<A, 0, false>(dwave, edge, c.col_ptr[j + 1] - k0, v0, v1, s0, s1);
            }
            if (run0)
                sL0[j] = v0;
            if (run1)
                sL1[j] = v1;
        }
        __syncthreads();
    }
    uint8_t *bits = job.bits + f0 * n;
    T *post = job.post ? static_cast<T *>(job.post) + f0 * n : nullptr;
    for (int j = tid; j < n; j += NT) {
        const T v = sL0[j];
        bits[j] = static_cast<uint8_t>(v < T(0));
        if (post)
            post[j] = it0 == 0 ? llr0[j] : v * T(A::kOut);
        if (has1) {
            const T w = sL1[j];
            bits[n + j] = static_cast<uint8_t>(w < T(0));
            if (post)
                post[n + j] = it1 == 0 ? llr1[j] : w * T(A::kOut);
        }
    }
    if (tid == 0) {
        job.iters[f0] = it0;
        if (has1)
            job.iters[f0 + 1] = it1;
    }
}

// Persistent batch kernel over frame pairs: flooding sum-product jobs only,
// item i of a job being its frames 2i and 2i + 1.  Two frames' LDS (qc1944:
// 152 KB) allow one 512-thread workgroup per CU, so the bodies may use 256
// VGPRs (2 waves per SIMD).
template <class A, int DB>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2))) void k_fused_pair(const Batch *__restrict__ batch, unsigned long long *counter)
{
    using T = typename A::T;
    constexpr uint32_t TS = sizeof(T);
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ long long s_item;
    const Batch &b = *batch;
    const FrameLayout lay = frame_layout(b.emax, b.nmax, 0, 0, 0, TS, 2);
    int32_t *sTab = reinterpret_cast<int32_t *>(smem + lay.t0);
    const uint32_t nmax = static_cast<uint32_t>(b.nmax);
    const Slots slots{TS * (nmax + 1 + threadIdx.x), TS * nmax};
    const FrameView fv0{smem, lay.r0, sTab, slots}, fv1{smem + lay.span, lay.r0, sTab, slots};
    if (threadIdx.x == 0) {  // published by the first barrier of the item loop
        reinterpret_cast<T *>(fv0.s)[nmax] = T(__builtin_huge_val());
        reinterpret_cast<T *>(fv1.s)[nmax] = T(__builtin_huge_val());
    }
    int cur_code = -1;
    for (;;) {
        if (threadIdx.x == 0)
            s_item = static_cast<long long>(atomicAdd(counter, 1ull));
        __syncthreads();
        const int64_t item = s_item;
        __syncthreads();
        if (item >= b.nitems)
            break;
        int j = 0;
        while (j + 1 < b.njobs && b.jobs[j + 1].item_begin <= item)
            ++j;
        const Job &job = b.jobs[j];
        const Code &c = b.codes[job.code];
        if (job.code != cur_code) {
            cur_code = job.code;
            load_tables<TS>(c, sTab, lay.r0);
        }
        const int64_t f0 = 2 * (item - job.item_begin);
        decode_frame_pair<A, DB>(c, job, f0, f0 + 1 < job.frames, fv0, fv1);
        __syncthreads();
    }
}

// Persistent batch kernel: workgroups take (job, frame) items from *counter.
// 512-thread workgroups, two per CU for n = 1944 (LDS bound): FP32 bodies are
// held to 128 VGPRs so both fit (4 waves per SIMD); FP64 bodies get 256.
template <class A>
constexpr int kFusedWavesPerEU = std::is_same<A, ArithF32>::value ? 4 : 2;

template <class A, int DB, int INST = kAnyJob>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(kFusedWavesPerEU<A>))) void k_fused(const Batch *__restrict__ batch, unsigned long long *counter)
{
    using T = typename A::T;
    constexpr uint32_t TS = sizeof(T);
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ long long s_item;
    const Batch &b = *batch;
    const FrameLayout lay = frame_layout(b.emax, b.nmax, 0, 0, 0, TS);
    int32_t *sTab = reinterpret_cast<int32_t *>(smem + lay.t0);
    const uint32_t nmax = static_cast<uint32_t>(b.nmax);
    const FrameView fv{smem, lay.r0, sTab, Slots{TS * (nmax + 1 + threadIdx.x), TS * nmax}};
    if (threadIdx.x == 0)  // published by the first barrier of the item loop
        reinterpret_cast<T *>(smem)[nmax] = T(__builtin_huge_val());
    int cur_code = -1;
    for (;;) {
        if (threadIdx.x == 0)
            s_item = static_cast<long long>(atomicAdd(counter, 1ull));
        __syncthreads();
        const int64_t item = s_item;
        __syncthreads();
        if (item >= b.nitems)
            break;
        int j = 0;
        while (j + 1 < b.njobs && b.jobs[j + 1].item_begin <= item)
            ++j;
        const Job &job = b.jobs[j];
        const Code &c = b.codes[job.code];
        if (job.code != cur_code) {
            cur_code = job.code;
            load_tables<TS>(c, sTab, lay.r0);
        }
        if (INST == kLayeredQC || (INST == kAnyJob && (job.flags & LDPC_LAYERED)))
            decode_frame_layered<A, DB, INST == kLayeredQC>(c, job, item - job.item_begin, fv);
        else
            decode_frame<A, DB, INST == kFloodQC, INST == kMinSumQC>(c, job, item - job.item_begin, fv);
        __syncthreads();
    }
}

// The instance of k_fused that runs every job of the batch: kFloodQC or
// kLayeredQC when all jobs are sum-product (no LDPC_MIN_SUM) on codes with a
// circulant view and all take that schedule, kMinSumQC when all are min-sum
// flooding on such codes, else kAnyJob.
inline Instance batch_instance(const Batch &b)
{
    if (b.njobs == 0)
        return kAnyJob;
    for (int32_t k = 0; k < b.ncodes; ++k)
        if (!b.codes[k].qc)
            return kAnyJob;
    const uint32_t first = b.jobs[0].flags & (LDPC_LAYERED | LDPC_MIN_SUM);
    for (int32_t k = 0; k < b.njobs; ++k)
        if ((b.jobs[k].flags & (LDPC_LAYERED | LDPC_MIN_SUM)) != first)
            return kAnyJob;
    if (first == LDPC_MIN_SUM)
        return kMinSumQC;
    if (first != 0 && first != LDPC_LAYERED)
        return kAnyJob;  // layered min-sum
    if (first)
        return kLayeredQC;
    for (int32_t k = 0; k < b.ncodes; ++k)  // the flooding instance reads the half-row words
        if (b.codes[k].half_rows == nullptr)
            return kAnyJob;
    return kFloodQC;
}

}  // namespace fused

namespace fused {

// Workgroups per CU and CU count for a launch of kernel fn with this LDS size
// and block size on the current device.  The runtime calls behind them (the
// kernel's LDS limit, the occupancy query, the device attribute) run once per
// (kernel, device, LDS bytes, threads) and are cached, not repeated on every
// launch; the LDS limit is only ever raised.  The caches are fixed-size
// tables (no heap allocation on any call): when the shape table is full it
// starts over, and a kernel missing from the full limit table has its limit
// set on every launch of a new shape.
inline ldpc_status launch_shape(const void *fn, size_t lds, int threads, int &per_cu, int &cus)
{
    struct Shape {
        const void *fn;
        int dev;
        size_t lds;
        int threads, per_cu, cus;
    };
    struct Limit {
        const void *fn;
        int dev;
        size_t lds;
    };
    constexpr int kShapes = 256, kLimits = 128;
    static std::mutex mu;
    static Shape shapes[kShapes];
    static Limit limits[kLimits];
    static int nshapes = 0, nlimits = 0;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return LDPC_EDEVICE;
    std::lock_guard<std::mutex> lk(mu);
    for (int i = 0; i < nshapes; ++i) {
        const Shape &e = shapes[i];
        if (e.fn == fn && e.dev == dev && e.lds == lds && e.threads == threads) {
            per_cu = e.per_cu;
            cus = e.cus;
            return LDPC_OK;
        }
    }
    Limit *lim = nullptr;
    for (int i = 0; i < nlimits; ++i)
        if (limits[i].fn == fn && limits[i].dev == dev)
            lim = &limits[i];
    if (lim == nullptr || lim->lds < lds) {
        if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)) != hipSuccess)
            return LDPC_EUNSUPPORTED;
        if (lim != nullptr)
            lim->lds = lds;
        else if (nlimits < kLimits)
            limits[nlimits++] = Limit{fn, dev, lds};
    }
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, lds) != hipSuccess || per_cu < 1)
        return LDPC_EUNSUPPORTED;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return LDPC_EDEVICE;
    if (nshapes == kShapes)  // batches of many different code mixes: start over
        nshapes = 0;
    shapes[nshapes++] = Shape{fn, dev, lds, threads, per_cu, cus};
    return LDPC_OK;
}

}  // namespace fused

// Launcher of the fused kernel for codes of row degree <= DB (one
// translation unit per dtype and bucket).
// The caller has already written the batch table to d_batch and reset *counter.
// fpw: frames per workgroup, 1 (k_fused) or 2 (k_fused_pair, FP32 flooding
// sum-product jobs only; the batch's items are then frame pairs).
// profile = false keeps the launch out of ldpc_profile_* timing (whose event
// pool may create events).
template <class A, int DB>
ldpc_status launch_fused_bucket(const fused::Batch &batch, fused::Batch *d_batch, unsigned long long *counter,
                                size_t lds_bytes, int threads, int fpw, hipStream_t s, bool profile);

template <class K>
ldpc_status launch_fused_kernel(K kern, const fused::Batch &batch, fused::Batch *d_batch, unsigned long long *counter,
                                size_t lds_bytes, int threads, hipStream_t s, bool profile)
{
    int per_cu = 0, cus = 0;
    const ldpc_status shape_rc =
        fused::launch_shape(reinterpret_cast<const void *>(kern), lds_bytes, threads, per_cu, cus);
    if (shape_rc != LDPC_OK)
        return shape_rc;
    const int64_t grid = std::min<int64_t>(batch.nitems, static_cast<int64_t>(per_cu) * cus);
    ProfScope ps(LDPC_KERNEL_FUSED, s, profile);
    LDPC_LAUNCH(ps, kern, dim3(static_cast<unsigned>(grid)), dim3(threads), static_cast<uint32_t>(lds_bytes), s,
                d_batch, counter);
    return hipGetLastError() == hipSuccess ? LDPC_OK : LDPC_EDEVICE;
}

#define LDPC_DEFINE_FUSED_BUCKET(A_, DB_)                                                                        \
    template <>                                                                                                  \
    ldpc_status launch_fused_bucket<A_, DB_>(const fused::Batch &batch, fused::Batch *d_batch,                  \
                                             unsigned long long *counter, size_t lds_bytes, int threads,        \
                                             int fpw, hipStream_t s, bool profile)                               \
    {                                                                                                            \
        if constexpr (std::is_same<A_, ArithF32>::value) {                                                       \
            if (fpw == 2)                                                                                        \
                return launch_fused_kernel(fused::k_fused_pair<A_, DB_>, batch, d_batch, counter, lds_bytes,    \
                                           threads, s, profile);                                                 \
            const fused::Instance inst_ = fpw == 1 ? fused::batch_instance(batch) : fused::kAnyJob;              \
            if (inst_ == fused::kFloodQC)                                                                        \
                return launch_fused_kernel(fused::k_fused<A_, DB_, fused::kFloodQC>, batch, d_batch, counter,   \
                                           lds_bytes, threads, s, profile);                                      \
            if (inst_ == fused::kLayeredQC)                                                                      \
                return launch_fused_kernel(fused::k_fused<A_, DB_, fused::kLayeredQC>, batch, d_batch, counter, \
                                           lds_bytes, threads, s, profile);                                      \
            if (inst_ == fused::kMinSumQC)                                                                       \
                return launch_fused_kernel(fused::k_fused<A_, DB_, fused::kMinSumQC>, batch, d_batch, counter,  \
                                           lds_bytes, threads, s, profile);                                      \
        }                                                                                                        \
        if (fpw != 1)                                                                                            \
            return LDPC_EUNSUPPORTED;                                                                            \
        return launch_fused_kernel(fused::k_fused<A_, DB_>, batch, d_batch, counter, lds_bytes, threads, s,     \
                                   profile);                                                                     \
    }

}  // namespace ldpc
