/*
 * ldpc.h - C ABI of libldpc: LDPC belief-propagation decoding (sum-product
 * or min-sum; flooding or layered schedule) on AMD Instinct MI355X (gfx950).
 *
 * The operation (arxiv 1812.06545, Section II): a binary LDPC code is given by
 * its sparse m x n parity-check matrix H (H[i][j] = 1 joins check node i to
 * variable node j of the Tanner graph).  Given channel log-likelihood ratios
 * L_ch (LLR = ln P(bit=0)/P(bit=1), so a negative value favours 1) for many
 * frames, the decoder runs belief propagation (the sum-product algorithm of
 * Section I) on a flooding (two-phase) schedule, Algorithm 1's loop order:
 *   Loop 1  q_mn = L_ch,n
 *   Loop 2  r_mn = 2 atanh( prod_{n' in N(m), n' != n} tanh(q_mn' / 2) ),
 *           clamped to [-LDPC_R_MAX, LDPC_R_MAX]
 *   Loop 3  L_n = L_ch,n + sum_{m in M(n)} r_mn ;  q_mn = L_n - r_mn
 *   Loop 4  x_n = 1 if L_n < 0 else 0
 * for t = 1 .. max_iter.  With LDPC_EARLY_STOP the syndrome H x (mod 2) is
 * tested before iteration 1 and after every Loop 4; a frame stops at the
 * first all-zero syndrome.  The per-frame iteration count is the number of
 * iterations run (0 when the channel decision already is a codeword;
 * max_iter when the syndrome never clears or early stop is off).
 *
 * With LDPC_LAYERED the decoder runs the layered schedule instead (Section
 * II, Algorithm 2): r = 0 and L = L_ch initially; one iteration visits the
 * check rows one at a time in ascending index order, and visiting row m sets
 *   q_mn = L_n - r_mn ;  r_mn = the Loop 2 rule over q_m. ;  L_n = q_mn + r_mn
 * for every n in N(m), so each row sees the updates of the rows before it.
 * The hard decision, syndrome test and iteration count are as above, per pass
 * over the rows.  Rows in a maximal run of consecutive rows that share no
 * variable (a layer; a block-row of a QC code) run in parallel, which does
 * not change the result.  To decode in another row order, permute the rows
 * of H.
 *
 * With LDPC_MIN_SUM the Loop 2 rule is min-sum (Section II: Algorithm 1 is
 * named the min-sum algorithm), on either schedule:
 *   r_mn = prod_{n' != n} sgn(q_mn') * min(max(scale * min_{n' != n} |q_mn'| - offset, 0), LDPC_R_MAX)
 * with sgn(0) = +1; scale = 1 and offset = 0 is plain min-sum, scale < 1
 * normalised and offset > 0 offset min-sum (ldpc_decode_minsum; ldpc_decode
 * uses 1 and 0).  A check of degree 1 sends +LDPC_R_MAX.
 *
 * Conventions for every call:
 *   - Frame buffers are row-major [frames][n]: frame f, bit j at f*n + j.
 *   - "device" pointers are HIP device memory of the device the code handle
 *     was created on, which must be the current device at the call.
 *   - Decoding calls are asynchronous on the given hipStream_t (passed as
 *     void*; NULL = the null stream).  They return after enqueueing.
 *   - Argument errors are detected before anything is enqueued: the call
 *     returns LDPC_EINVAL (or LDPC_EUNSUPPORTED) and writes nothing.
 *   - A HIP launch failure returns LDPC_EDEVICE; faults during execution
 *     surface at the caller's next synchronisation.
 *   - frames == 0 is a no-op returning LDPC_OK.
 *   - LLR inputs must be finite.
 *   - The caller owns every frame buffer, workspace and stream; the library
 *     owns code handles (device-resident, immutable after creation, safe to
 *     share between threads) and plans.
 */
#ifndef LDPC_H
#define LDPC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#pragma GCC visibility push(default)
#endif

typedef enum {
    LDPC_OK = 0,
    LDPC_EINVAL = -1,       /* invalid argument; nothing was enqueued or written */
    LDPC_ENOMEM = -2,       /* device or host allocation (or host thread creation) failed */
    LDPC_EDEVICE = -3,      /* HIP runtime error, or an unexpected internal failure */
    LDPC_EBUSY = -4,        /* resource temporarily unavailable (server full) */
    LDPC_EUNSUPPORTED = -5  /* valid but outside this build's limits */
} ldpc_status;

/* Every function reports failure through its status; no C++ exception
 * leaves the library. */

typedef enum { LDPC_F32 = 0, LDPC_F64 = 1 } ldpc_dtype;

#define LDPC_EARLY_STOP 1u  /* flag: stop a frame at its first zero syndrome */
#define LDPC_LAYERED 2u     /* flag: layered schedule (ldpc_decode and ldpc_decode_batch jobs) */
#define LDPC_MIN_SUM 4u     /* flag: min-sum check rule instead of sum-product */

/* Clamp on check-to-variable messages (the paper gives none; 20 keeps the
 * FP64 tanh/atanh evaluation accurate). */
#define LDPC_R_MAX 20.0

/* Limits of this build.  Edges and variables are bounded so that the
 * kernels' 32-bit offsets into a 64-frame chunk (edge x 64 values, variable
 * x 64 doubles) cannot overflow. */
#define LDPC_MAX_ROW_DEGREE 64
#define LDPC_MAX_FRAMES (1 << 24)
#define LDPC_MAX_EDGES ((1 << 25) - 1)
#define LDPC_MAX_VARIABLES ((1 << 22) - 1)

typedef struct ldpc_code_s *ldpc_code;

/* Human-readable name of a status code (static storage).  Not an operation of
 * the paper: the error convention of this library. */
const char *ldpc_status_str(ldpc_status status);

/*
 * Create a code from H in CSR form (Section II: the H-matrix / Tanner graph).
 *   m, n     rows (check nodes) >= 1 and columns (variable nodes) >= 1
 *   row_ptr  host, m+1 entries, row_ptr[0] = 0, non-decreasing
 *   col_idx  host, row_ptr[m] entries; columns of row i in
 *            col_idx[row_ptr[i] .. row_ptr[i+1]); any order, no duplicates
 * The matrix is copied to the current device; the caller keeps its arrays.
 * Rows may be empty (always satisfied); columns may be empty (L = L_ch).
 * Errors: EINVAL for bad sizes, out-of-range or duplicate columns, NULL
 * pointers; EUNSUPPORTED for a row degree above LDPC_MAX_ROW_DEGREE, more
 * than LDPC_MAX_EDGES edges or more than LDPC_MAX_VARIABLES columns;
 * ENOMEM / EDEVICE on allocation or copy failure.  *out is set only on OK.
 */
ldpc_status ldpc_code_from_csr(int32_t m, int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                               ldpc_code *out);

/*
 * Create a quasi-cyclic code from an mb x nb base matrix of circulant shifts
 * (host, row-major, -1 = all-zero block, otherwise 0 <= shift < Z).  Block
 * (i, j) with shift s joins check row i*Z + r to variable column
 * j*Z + ((r + s) mod Z), r = 0 .. Z-1; so m = mb*Z, n = nb*Z.
 * Errors as ldpc_code_from_csr, plus EINVAL for shifts outside [-1, Z).
 * QC codes additionally get the circulant-block layout used by the fused
 * (frame-resident) kernels.
 */
ldpc_status ldpc_code_from_qc(int32_t mb, int32_t nb, int32_t Z, const int32_t *shifts, ldpc_code *out);

/* Sizes of a code (Section II: m check nodes, n variable nodes, one Tanner
 * graph edge per 1 of H): m, n and the number of edges.  Any output may be NULL. */
ldpc_status ldpc_code_info(ldpc_code code, int32_t *m, int32_t *n, int64_t *edges);

/* Layers of the layered schedule (Section II, Algorithm 2): the rows in
 * ascending order, split into maximal runs in which no two rows share a
 * variable; each layer is one parallel step.  Outputs the number of layers and
 * the fewest and most rows in a layer (0, 0, 0 for a code without rows).  Any
 * output may be NULL. */
ldpc_status ldpc_code_layers(ldpc_code code, int32_t *nlayers, int32_t *min_rows, int32_t *max_rows);

/* Release a code (library bookkeeping, no paper passage).  The caller must
 * ensure no enqueued work still uses it.  NULL is ignored. */
void ldpc_code_destroy(ldpc_code code);

/*
 * Workspace needed by ldpc_decode for `frames` frames of `code` in `dtype`
 * with at most `max_iter` iterations.  Frames are padded to a multiple of 64;
 * the messages are stored edge-major with frames innermost (the interleaved
 * frame layout of Section III-B: the same node of consecutive frames side by
 * side).
 */
ldpc_status ldpc_workspace_bytes(ldpc_code code, ldpc_dtype dtype, int32_t frames, int32_t max_iter,
                                 size_t *bytes);

/*
 * Decode `frames` frames with per-iteration kernel launches (the plain
 * path, messages streamed through device memory): flooding runs one
 * check-node and one variable-node kernel per iteration (Section II,
 * Algorithm 1: Loop 2, then Loops 3 and 4; the launch boundary is the
 * two-phase barrier); layered (LDPC_LAYERED; Algorithm 2) one kernel per
 * layer, plus a syndrome kernel per iteration with early stop.  The frames
 * are interleaved on the device as in Section III-B.
 *   dtype      LDPC_F32 (llr/posterior are float) or LDPC_F64 (double)
 *   max_iter   >= 0; 0 returns the hard decision of llr, iters 0, posterior = llr
 *   flags      any of LDPC_EARLY_STOP, LDPC_LAYERED, LDPC_MIN_SUM (or 0)
 *   llr        device, [frames][n] of dtype, read only
 *   bits       device, [frames][n] uint8 0/1 (written)
 *   iters      device, [frames] int32 (written)
 *   posterior  device, [frames][n] of dtype, or NULL (written if non-NULL)
 *   workspace  device, at least ldpc_workspace_bytes(...) bytes, 256-byte aligned
 *   stream     hipStream_t or NULL
 */
ldpc_status ldpc_decode(ldpc_code code, ldpc_dtype dtype, int32_t frames, int32_t max_iter, uint32_t flags,
                        const void *llr, uint8_t *bits, int32_t *iters, void *posterior, void *workspace,
                        size_t workspace_bytes, void *stream);

/*
 * ldpc_decode with the min-sum magnitude correction given (Section II: the
 * min-sum rule Algorithm 1 is named after): with LDPC_MIN_SUM
 * in flags, |r| = max(ms_scale * min - ms_offset, 0) before the clamp
 * (ms_offset in natural LLR units).  EINVAL unless ms_scale is finite and
 * > 0 and ms_offset finite and >= 0 (checked whatever the flags).
 */
ldpc_status ldpc_decode_minsum(ldpc_code code, ldpc_dtype dtype, int32_t frames, int32_t max_iter, uint32_t flags,
                               float ms_scale, float ms_offset, const void *llr, uint8_t *bits, int32_t *iters,
                               void *posterior, void *workspace, size_t workspace_bytes, void *stream);

/* One decoding job of a batch (Section III-A: one code's frames, decoded
 * alike): same meaning as the ldpc_decode arguments. */
typedef struct {
    ldpc_code code;
    int32_t frames;
    int32_t max_iter;
    uint32_t flags;
    const void *llr;
    uint8_t *bits;
    int32_t *iters;
    void *posterior; /* may be NULL */
    float ms_scale;  /* min-sum correction (used with LDPC_MIN_SUM), as in ldpc_decode_minsum: */
    float ms_offset; /* scale > 0 (1 = plain min-sum), offset >= 0 */
} ldpc_job;

/*
 * Workspace for ldpc_decode_batch over these jobs (all of one dtype): the job
 * tables of its persistent launches (Section III-A), and the streaming
 * workspace of the largest job that takes the plain path.
 */
ldpc_status ldpc_batch_workspace_bytes(const ldpc_job *jobs, int32_t njobs, ldpc_dtype dtype, size_t *bytes);

/*
 * Decode a batch of jobs of possibly different codes, lengths and rates
 * (Section III-A: frame-level parallelism, the same decoding carried out
 * for many frames at once, a workgroup per frame here; Section III-C: work
 * from several sources kept in flight together, here in one launch).
 * Jobs whose code fits the fused frame-resident kernel (messages of one
 * frame held in LDS) run together in ONE persistent launch whose workgroups
 * pull (job, frame) items from a device-side queue; each workgroup runs every
 * iteration of its frame, with per-frame early stop, on the schedule its job's
 * flags select (flooding or LDPC_LAYERED: block-rows, or the code's layers,
 * one at a time with a workgroup barrier between them).  Jobs whose code
 * does not fit run through the plain per-iteration kernels on the same
 * stream.
 * Each frame's result is identical to decoding that frame alone.
 * Errors as ldpc_decode; jobs with frames == 0 are skipped.
 */
ldpc_status ldpc_decode_batch(const ldpc_job *jobs, int32_t njobs, ldpc_dtype dtype, void *workspace,
                              size_t workspace_bytes, void *stream);

/*
 * ldpc_decode_batch for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation.  Same jobs, results (bit for bit) and errors as
 * ldpc_decode_batch, without a workspace: the batch tables and work counters
 * live in a static device array of the library (LDPC_NOALLOC_MAX_GROUPS
 * slices of about 4 KiB each, about 64 KiB, held on every device the call
 * runs on until the process ends).  The call allocates nothing, on the
 * device or the host, and creates no events (ldpc_profile_* does not time
 * it).  Every job's code must fit the fused kernel (ldpc_batch_fits_fused)
 * and the jobs must pack into at most LDPC_NOALLOC_MAX_GROUPS launches (24
 * jobs and 16 codes per launch, fewer if the codes' LDS needs add up, and
 * one launch per tuned workgroup size and frames per workgroup among them);
 * otherwise LDPC_EUNSUPPORTED and nothing is enqueued.  The array is shared
 * by every call on a device: calls whose work overlaps on one device
 * (different streams, or threads) race on it and must be serialised by the
 * caller, e.g. by using one stream.  Each launch rewrites its slice (table
 * and counter) with a kernel before using it, so nothing must be cleared
 * between calls.
 */
#define LDPC_NOALLOC_MAX_GROUPS 16
ldpc_status ldpc_decode_batch_noalloc(const ldpc_job *jobs, int32_t njobs, ldpc_dtype dtype, void *stream);

/*
 * Plans: the launch sequence of ldpc_decode_batch for these jobs, captured
 * once in a HIP graph (kernel nodes only) and replayed by ldpc_plan_launch
 * (Section III-C: the paper's streams re-issue the same per-batch kernel
 * sequence for every batch; a plan records it once and replays it).
 * The job buffers and the workspace are fixed at creation and must outlive
 * the plan; each launch decodes whatever the LLR buffers hold when it runs,
 * with results identical to ldpc_decode_batch on the same inputs.  Creation
 * captures on a private stream and enqueues nothing.  Errors as
 * ldpc_decode_batch; EDEVICE if capture or instantiation fails.
 */
typedef struct ldpc_plan_s *ldpc_plan;
ldpc_status ldpc_plan_create(const ldpc_job *jobs, int32_t njobs, ldpc_dtype dtype, void *workspace,
                             size_t workspace_bytes, ldpc_plan *out);
ldpc_status ldpc_plan_launch(ldpc_plan plan, void *stream);
void ldpc_plan_destroy(ldpc_plan plan);

/*
 * Serving: continuous batching of decode requests (one request = 1 or more
 * frames of one code), the concurrency of Section III-C (several host
 * threads keeping their own frames in flight on the GPU) re-designed: requests
 * of any thread join the next launch group as memory and slots free up.  A scheduler thread owned by the server admits queued
 * requests, first come first served, whenever arena memory (fixed at
 * creation, sized by mem_budget_bytes) and one of max_inflight launch slots
 * are free; each admitted group's LLRs are packed contiguously in pinned host
 * memory, ordered by code (then iteration limit, flags and whether
 * posteriors are wanted; FIFO within each) so that neighbouring requests
 * decoded alike form one job, moved to the device by one copy kernel and
 * decoded by one ldpc_decode_batch call on the slot's own stream (so a group
 * admitted while others run overlaps with them on the device); the decode
 * kernel writes the results into pinned host memory, from which the
 * scheduler fills the requester's buffers and marks the request done.  The
 * requester's LLRs are read when the group is admitted, so they must stay
 * valid until the request completes.  Every frame's result equals decoding it
 * alone.
 * While groups are in flight the scheduler thread polls their completion by
 * spinning (one host core busy), not by timed sleeps: waking a sleeping
 * thread can take milliseconds, which every request in flight would wait out.
 * With LDPC_SERVER_TRACE set to a file name, scheduler steps slower than
 * 0.5 ms are appended to that file when the server is destroyed (where the
 * step's time went, the thread's CPU time, its context switches).
 * Codes must fit the fused kernel (ldpc_batch_fits_fused), all FP32.
 */
typedef struct ldpc_server_s *ldpc_server;

typedef struct {
    int32_t ncodes;            /* number of codes served (<= 64) */
    const ldpc_code *codes;    /* request code_id indexes this array; handles must outlive the server */
    size_t mem_budget_bytes;   /* arena for in-flight requests: about budget/10 coded bits (frames x n) at once,
                                  each 4 bytes of device memory (LLR) and 9 of pinned host memory */
    int32_t max_inflight;      /* concurrent launch groups (streams), 1 .. 8 */
    int32_t max_group_frames;  /* cap on frames per launch group (bounds latency), >= 1; each launch slot
                                  also reserves about 4.4 KiB of device memory per frame of this cap for
                                  the launch tables of the group's fused launches */
    int32_t max_queue;         /* queued requests beyond which submit returns LDPC_EBUSY, >= 1 */
} ldpc_server_cfg;

typedef struct {
    int64_t submitted, completed, cancelled, failed, launches;
    int64_t frames_completed, bits_completed; /* coded bits = frames * n */
    double p50_ms, p99_ms, p999_ms, max_ms;    /* latency: completion - arrival, over completed requests */
    double mean_group_frames;
    int64_t max_queue_depth;
    /* where the slowest request (the one of max_ms) spent its time: */
    double worst_submit_ms;   /* arrival -> submit call */
    double worst_queue_ms;    /* submit -> its group admitted by the scheduler */
    double worst_stage_ms;    /* admitted -> group launched (LLR staging copy and launch calls) */
    double worst_device_ms;   /* launched -> completion seen by the scheduler (device time, including
                                 any wait behind other groups on the device) */
    double worst_copyout_ms;  /* completion seen -> results copied out, request done */
    double max_step_ms;       /* longest scheduler step (completions reaped + groups admitted), and within
                                 steps the longest: */
    double max_copy_ms;       /* host copy of one group's LLRs in, or of its results out */
    double max_launch_ms;     /* sequence of launch calls of one group */
    double max_query_ms;      /* completion query of one group */
} ldpc_server_stats;

/* Create a server on the current device (Section III-C, as above).  Before
 * returning it decodes one
 * frame of every code on every launch stream (synchronously), so that stream
 * set-up and kernel loading, which happen on first use, are not charged to
 * the first requests.  EINVAL for bad sizes or NULL arguments, EUNSUPPORTED
 * if a code does not fit the fused kernel, ENOMEM if the arena cannot be
 * allocated, EDEVICE (or the failing call's status) if the warm-up fails. */
ldpc_status ldpc_server_create(const ldpc_server_cfg *cfg, ldpc_server *out);

/*
 * Queue a request (Section III-C: a host thread handing its frames to the
 * GPU): `frames` frames of codes[code_id], LLRs llr[frames][n]
 * (host memory, float), decoded with max_iter / flags as in ldpc_decode
 * (flags 0 or LDPC_EARLY_STOP: the server runs the flooding schedule only).
 * Outputs go to host memory bits[frames][n], iters[frames] and, if non-NULL,
 * posterior[frames][n]; every buffer must stay valid and untouched until the
 * request is done.  arrival_ns: the request's arrival time on the
 * CLOCK_MONOTONIC scale for latency accounting (0 = now).  *ticket receives
 * an id for poll/wait/cancel.  EINVAL for bad arguments or a request larger
 * than the arena / group cap; EBUSY when max_queue requests are waiting.
 * If the device launch of a request's group fails, the request still
 * completes, with every iteration count set to -1 (counted in stats.failed).
 * If the scheduler itself runs out of host memory, every admitted group is
 * let finish on the device, every request not yet done completes that way,
 * and later submits return LDPC_ENOMEM.
 * Tickets stay valid until the server is destroyed.
 */
ldpc_status ldpc_server_submit(ldpc_server server, int32_t code_id, int32_t frames, int32_t max_iter, uint32_t flags,
                               const float *llr, uint8_t *bits, int32_t *iters, float *posterior, int64_t arrival_ns,
                               uint64_t *ticket);

/* *done = 1 when the request's outputs are complete (0 otherwise).  EINVAL for
 * an unknown ticket.  (Section III-C: a worker learning that its frames are
 * decoded.) */
ldpc_status ldpc_server_poll(ldpc_server server, uint64_t ticket, int32_t *done);

/* Block until the request is done or timeout_ms elapses (LDPC_EBUSY on
 * timeout); the blocking wait of Section III-C's workers. */
ldpc_status ldpc_server_wait(ldpc_server server, uint64_t ticket, double timeout_ms);

/* Remove a request that is still queued (LDPC_OK); LDPC_EBUSY if it is
 * already on the device or done.  (Serving bookkeeping; no paper passage.) */
ldpc_status ldpc_server_cancel(ldpc_server server, uint64_t ticket);

/* Counters and latency percentiles since creation or the last reset
 * (throughput and latency, the quantities of Section IV's measurements). */
ldpc_status ldpc_server_stats_get(ldpc_server server, ldpc_server_stats *out, int reset);

/* Finish every admitted and queued request, stop the scheduler, free
 * everything.  (Serving bookkeeping; no paper passage.) */
void ldpc_server_destroy(ldpc_server server);

/*
 * Workgroup size (a multiple of 64, at most 512) of the fused frame-resident
 * kernel used by ldpc_decode_batch (Section III-A: the threads that decode
 * one frame); default 512.  EINVAL for other values.  Process-wide default
 * for jobs whose code has no tuned size (ldpc_autotune_batch records one per
 * code; ldpc_tuning_clear forgets them); affects speed only, never results.
 */
ldpc_status ldpc_batch_set_threads(int32_t threads);

/*
 * Frames per workgroup of the fused kernel used by ldpc_decode_batch for FP32
 * flooding sum-product jobs whose code fits two frames in one workgroup's LDS:
 * 1 (default) or 2.  With 2, every thread runs its rows and columns for two
 * frames of a job at once (Section III-A: frames decoded side by side),
 * sharing the offsets and table reads of each edge slot; other jobs keep 1.
 * Process-wide default (tuned shapes override it); affects speed only, never
 * results.  EINVAL for other values.
 */
ldpc_status ldpc_batch_set_frames_per_group(int32_t frames);

/*
 * The launch configuration ldpc_decode_batch would use for these jobs: frames
 * per workgroup as tuned for this batch shape by ldpc_autotune_batch (or
 * ldpc_tuning_load), else the process-wide default; *threads the workgroup
 * size of the first job that runs in the fused kernel (jobs of other codes
 * may differ: ldpc_batch_job_threads gives each).  Any output may be NULL;
 * *tuned is 1 for a tuned batch shape.  Errors as ldpc_decode_batch's
 * argument checks.
 */
ldpc_status ldpc_batch_launch_config(const ldpc_job *jobs, int32_t njobs, ldpc_dtype dtype, int32_t *threads,
                                     int32_t *frames_per_group, int32_t *tuned);

/*
 * Workgroup size each job would run with in the fused kernel
 * (threads[njobs], caller-allocated; 0 for a job with no frames or one that
 * runs on the plain path).  Jobs of different sizes run as separate fused
 * launches on the same stream.  Errors as ldpc_decode_batch's argument
 * checks; EINVAL if threads is NULL with njobs > 0.  (Library bookkeeping of
 * the autotuner, Section III-A's mapping of frames onto the GPU.)
 */
ldpc_status ldpc_batch_job_threads(const ldpc_job *jobs, int32_t njobs, ldpc_dtype dtype, int32_t *threads);

/*
 * Autotuner of the batch path (Section III-A: the mapping of frames onto the
 * GPU).  Decodes the given jobs (their output buffers are overwritten,
 * inputs untouched) under candidate launch configurations, in two stages:
 * first, for each code (device architecture, code shape by sizes and degree
 * profiles, dtype, flags), that code's jobs alone at workgroup sizes 64, 128,
 * 192, 256, 384 and 512, recording the fastest size for the code (used by
 * every later batch with jobs of that code); then the whole batch with one
 * frame per workgroup and, where some job can use it, two
 * (ldpc_batch_set_frames_per_group), recording the faster for this batch
 * shape (the codes, frame counts rounded up to a power of two, iteration
 * caps, flags, dtype).  Every candidate's outputs must be bit-identical to
 * the first run's; each is timed with HIP events (3 runs after a warm-up).
 * Blocks until done.  *best_threads and *best_ms (may be NULL) receive the
 * first fused job's workgroup size and the batch's time
 * (ldpc_batch_launch_config and ldpc_batch_job_threads give the whole
 * choice).  The workspace must hold ldpc_batch_workspace_bytes (which covers
 * every candidate).  LDPC_EDEVICE if candidates disagree (then nothing is
 * recorded for these codes and this shape).
 */
ldpc_status ldpc_autotune_batch(const ldpc_job *jobs, int32_t njobs, ldpc_dtype dtype, void *workspace,
                                size_t workspace_bytes, void *stream, int32_t *best_threads, double *best_ms);

/*
 * The tuning table on disk (library bookkeeping of the autotuner above): save
 * writes every recorded choice, one text line each ("<arch> <key> <threads>
 * <frames per workgroup> <ms>", the key being the hash of the batch shape or,
 * for a per-code workgroup size, of the code, device architecture included;
 * per-code lines have frames per workgroup 0); load merges a saved table
 * into the process's (*entries, may be NULL, receives the number of lines
 * read), so a later process skips tuning for shapes already tuned on that
 * architecture.  EINVAL if the file cannot be opened or a line is malformed
 * (load keeps the lines read before it).  clear forgets every recorded
 * choice (the process-wide defaults apply again).
 */
ldpc_status ldpc_tuning_save(const char *path);
ldpc_status ldpc_tuning_load(const char *path, int32_t *entries);
void ldpc_tuning_clear(void);

/*
 * Whether frames of `code` in `dtype` can run in the fused frame-resident
 * kernel (Section III-A: one frame per workgroup) on the current device (row degree <= 32, n < 65536 and one frame's
 * messages within one workgroup's LDS).  LDPC_OK if so, LDPC_EUNSUPPORTED if
 * ldpc_decode_batch would route the code through the plain path; *lds_bytes
 * (may be NULL) receives the LDS one frame needs.
 */
ldpc_status ldpc_batch_fits_fused(ldpc_code code, ldpc_dtype dtype, size_t *lds_bytes);

/*
 * Per-kernel device timing, a measurement aid (not part of decoding; the
 * per-stage timing breakdown of Section IV, kernel by kernel).  While
 * enabled, every kernel the library launches outside a stream capture is
 * bracketed by a pair of HIP events on its own stream.  ldpc_profile_collect
 * waits for the recorded events, writes for each kernel kind k the summed
 * device duration ms[k] (milliseconds) and launch count counts[k] (arrays of
 * LDPC_KERNEL_KINDS entries, either may be NULL), and clears the records.
 * Enabling adds two event records per launch; it is off by default.
 */
typedef enum {
    LDPC_KERNEL_INGEST = 0,    /* caller layout -> frame-interleaved layout */
    LDPC_KERNEL_CHECK = 1,     /* check-node update: one iteration (flooding) or one layer (layered) */
    LDPC_KERNEL_VARIABLE = 2,  /* variable-node update + hard decision, one iteration */
    LDPC_KERNEL_OUTPUT = 3,    /* frame-interleaved -> caller layout */
    LDPC_KERNEL_FUSED = 4,     /* persistent frame-resident decoder (all iterations) */
    LDPC_KERNEL_OTHER = 5,     /* small bookkeeping kernels */
    LDPC_KERNEL_KINDS = 6
} ldpc_kernel_kind;

ldpc_status ldpc_profile_enable(int enable);
ldpc_status ldpc_profile_collect(double *ms, int64_t *counts);

/*
 * The paper's multi-stream structure (Section III-C), as a measured baseline:
 * `workers` host threads, each with its own stream, pinned staging and
 * device buffers for `frames_per_batch` frames, take batches of frames in
 * turn; a worker copies its batch's LLRs (host memory, float, [batches *
 * frames_per_batch][n], read only) into pinned staging and to the device,
 * decodes them with ldpc_decode (flags as there; FP32), copies bits and
 * iteration counts back, waits for its stream (spinning, or blocking on the
 * event when blocking_sync != 0) and copies the results into bits
 * ([batches * frames_per_batch][n]) and iters.  Blocks until every batch is
 * done.  *stats (may be NULL) receives wall time, throughput and the
 * process's CPU time over the run (getrusage: user + system, all threads).
 * EINVAL for bad sizes or flags, ENOMEM if buffers cannot be allocated,
 * EDEVICE (or a decode error) if a worker's call fails.
 */
typedef struct {
    double wall_ms;        /* first batch taken to last result copied */
    double frames_per_s;
    double mbps;           /* coded bits: frames * n per second, 1e6 */
    double cpu_ms;         /* process CPU time (user + system) during the run */
    double cpu_cores_busy; /* cpu_ms / wall_ms: host cores kept busy on average */
    double cpu_load;       /* cpu_cores_busy / online_cores */
    int32_t online_cores;
} ldpc_mstream_stats;

ldpc_status ldpc_mstream_run(ldpc_code code, int32_t workers, int32_t frames_per_batch, int32_t batches,
                             int32_t max_iter, uint32_t flags, int32_t blocking_sync, const float *llr, uint8_t *bits,
                             int32_t *iters, ldpc_mstream_stats *stats);

/*
 * Streaming copy of `bytes` (a multiple of 16; both pointers 16-byte aligned,
 * device memory) on `stream`: a yardstick for achievable HBM bandwidth and
 * for scaling hardware byte counters (Section III: the decoder is bound by
 * its memory accesses, so their achievable rate is the reference).  Not part
 * of decoding.
 */
ldpc_status ldpc_copy_probe(void *dst, const void *src, size_t bytes, void *stream);

#if defined(__GNUC__)
#pragma GCC visibility pop
#endif

#ifdef __cplusplus
}
#endif

#endif /* LDPC_H */
