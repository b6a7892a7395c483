// Batched decoding of jobs of different codes, lengths and rates.
//
// Jobs whose code fits the fused frame-resident kernel (row degree <= 32 and
// one frame's messages within the LDS of one workgroup) are packed into as
// few persistent launches as the kernel-argument table allows (<= 24 jobs and
// <= 16 distinct codes per launch); the others run through the plain
// per-iteration path on the same stream.  The batch table of each launch is
// written on the device by a tiny kernel that receives it by value.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "fused_kernels.h"

namespace ldpc {
namespace {

// Launch configuration of the fused kernel: workgroup size and frames per
// workgroup (1, or 2 for FP32 flooding sum-product jobs).
struct LaunchCfg {
    int threads = 512;
    int fpw = 1;
};

std::mutex g_mu;
LaunchCfg g_cfg;                        // default (ldpc_batch_set_threads / ldpc_batch_set_frames_per_group)
struct Tuned {
    LaunchCfg cfg;
    double ms = 0.0;
};
std::map<uint64_t, Tuned> g_tuned;      // batch shape key -> configuration chosen by ldpc_autotune_batch
std::map<uint64_t, Tuned> g_code_tuned; // code key -> workgroup size chosen for its jobs (fpw unused: 0)

constexpr int kMaxArchDevices = 64;
uint64_t g_arch_hash[kMaxArchDevices];  // per device: hash of its architecture name, 0 until looked up
char g_arch_name[kMaxArchDevices][64];

uint64_t fnv(uint64_t x, uint64_t v)
{
    for (int b = 0; b < 8; ++b) {
        x ^= (v >> (8 * b)) & 0xffu;
        x *= 1099511628211ull;
    }
    return x;
}

// The current device's architecture name (e.g. "gfx950:sramecc+:xnack-")
// and its hash, looked up once per device.  Caller holds g_mu.
const char *arch_of_current(uint64_t *hash)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxArchDevices) {
        *hash = 1;
        return "";
    }
    if (g_arch_hash[dev] == 0) {
        hipDeviceProp_t prop;
        uint64_t x = 1469598103934665603ull;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
            std::snprintf(g_arch_name[dev], sizeof(g_arch_name[dev]), "%s", prop.gcnArchName);
            for (const char *c = g_arch_name[dev]; *c; ++c)
                x = fnv(x, static_cast<unsigned char>(*c));
        }
        g_arch_hash[dev] = x | 1;
    }
    *hash = g_arch_hash[dev];
    return g_arch_name[dev];
}

// Shape of a batch for the tuning table: a hash of the device architecture,
// the dtype and, per job, the code's shape (sizes and degree histograms, not
// its address), frames rounded up to a power of two, the iteration cap and
// the flags.  Computed without allocating.  Caller holds g_mu.
uint64_t shape_key(const ldpc_job *jobs, int32_t njobs, ldpc_dtype dt)
{
    uint64_t arch = 0;
    arch_of_current(&arch);
    uint64_t x = fnv(1469598103934665603ull, arch);
    x = fnv(x, static_cast<uint64_t>(dt));
    x = fnv(x, static_cast<uint64_t>(njobs));
    for (int32_t i = 0; i < njobs; ++i) {
        uint64_t f = 1;
        while (f < static_cast<uint64_t>(jobs[i].frames))
            f <<= 1;
        x = fnv(x, jobs[i].code->shape_hash);
        x = fnv(x, f);
        x = fnv(x, static_cast<uint64_t>(jobs[i].max_iter));
        x = fnv(x, jobs[i].flags);
    }
    return x;
}

// Key of one job's code for the per-code workgroup size: device
// architecture, dtype, the code's shape and the job's flags (the decoding
// mode selects the kernel body).  Caller holds g_mu.
uint64_t code_key(const ldpc_job &j, ldpc_dtype dt)
{
    uint64_t arch = 0;
    arch_of_current(&arch);
    uint64_t x = fnv(fnv(1099511628211ull, arch), 0xc0de);
    x = fnv(x, static_cast<uint64_t>(dt));
    x = fnv(x, j.code->shape_hash);
    return fnv(x, j.flags);
}

// Workgroup size of one job's fused launch: its code's tuned size, else the
// batch's.
int job_threads(const ldpc_job &j, ldpc_dtype dt, int batch_threads)
{
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_code_tuned.empty())
        return batch_threads;
    auto it = g_code_tuned.find(code_key(j, dt));
    return it != g_code_tuned.end() ? it->second.cfg.threads : batch_threads;
}

LaunchCfg cfg_for(const ldpc_job *jobs, int32_t njobs, ldpc_dtype dt)
{
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_tuned.empty()) {
        auto it = g_tuned.find(shape_key(jobs, njobs, dt));
        if (it != g_tuned.end())
            return it->second.cfg;
    }
    return g_cfg;
}

size_t lds_limit()
{
    int dev = 0, bytes = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&bytes, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return 0;
    return static_cast<size_t>(bytes);
}

// Whether the fused kernel uses the circulant view of a QC code in a dtype
// of tsize bytes: its row tables pack tsize * j * Z and tsize * s into 16-bit
// fields, and it divides row and column indices by Z with a multiply-high,
// exact while index * Z < 2^32 (Z >= 2).  Other codes use the CSR view.
bool fused_qc_view(const ldpc_code_s *c, size_t tsize)
{
    return c->is_qc && c->Z >= 2 && tsize * static_cast<size_t>(c->n) <= 65535 &&
           tsize * static_cast<size_t>(c->Z) <= 65535 &&
           static_cast<uint64_t>(std::max(c->m, c->n)) * static_cast<uint64_t>(c->Z) < (1ull << 32);
}

struct FusedFit {
    bool ok = false;
    int bucket = 0;
    size_t lds = 0;
};

FusedFit fused_fit(const ldpc_code_s *c, ldpc_dtype dt, size_t limit)
{
    FusedFit r;
    const int d = c->max_row_deg;
    if (dt == LDPC_F32)
        r.bucket = d <= 8 ? 8 : d <= 16 ? 16 : d <= 24 ? 24 : d <= 32 ? 32 : 0;
    else
        r.bucket = d <= 8 ? 8 : d <= 16 ? 16 : d <= 32 ? 32 : 0;
    const size_t tsize = dt == LDPC_F64 ? sizeof(double) : sizeof(float);
    const bool qc = fused_qc_view(c, tsize);
    // A QC code's fused slot tables list its rows by block-row degree, which
    // only the circulant view follows: without it the code takes the plain path.
    if (r.bucket == 0 || c->n >= 65536 || (c->is_qc && !qc))
        return r;
    r.lds = fused::frame_lds_bytes(c->E, c->n, qc ? c->qc_words : 0, qc ? c->nblocks : 0, qc ? c->mb : 0, tsize);
    r.ok = r.lds <= limit;
    return r;
}

// One fused launch: up to kMaxJobs jobs over up to kMaxCodes codes (fixed
// storage, so planning needs no heap).
struct Group {
    int fpw = 1;        // frames per workgroup of this launch
    int threads = 512;  // workgroup size of this launch
    int32_t njobs = 0, ncodes = 0;
    int32_t jobs[fused::kMaxJobs];
    const ldpc_code_s *codes[fused::kMaxCodes];
    int bucket = 0;
    // maxima over the group's codes: the LDS layout is sized by them
    int64_t emax = 0;
    int32_t nmax = 0, words = 0, nblocks = 0, mb = 0;
    size_t tsize = 4;
    size_t lds() const { return fused::frame_lds_bytes(emax, nmax, words, nblocks, mb, tsize, fpw); }
    int code_index(const ldpc_code_s *c) const
    {
        for (int32_t k = 0; k < ncodes; ++k)
            if (codes[k] == c)
                return k;
        return -1;
    }
    void add_code(const ldpc_code_s *c)
    {
        const bool qc = fused_qc_view(c, tsize);
        codes[ncodes++] = c;
        emax = std::max<int64_t>(emax, c->E);
        nmax = std::max(nmax, c->n);
        words = std::max(words, qc ? c->qc_words : 0);
        nblocks = std::max(nblocks, qc ? c->nblocks : 0);
        mb = std::max(mb, qc ? c->mb : 0);
    }
};

constexpr int kPlanNotFused = -1;  // a job's code does not fit the fused kernel and no plain list was given
constexpr int kPlanTooMany = -2;   // more than max_groups launch groups would be needed

// Frames per workgroup a job runs with when fpw_pref frames are preferred:
// 2 only for FP32 flooding sum-product jobs whose code fits two frames in
// one workgroup's LDS.
int job_fpw(const ldpc_job &j, ldpc_dtype dt, int fpw_pref, size_t limit)
{
    if (fpw_pref != 2 || dt != LDPC_F32 || (j.flags & (LDPC_LAYERED | LDPC_MIN_SUM)) != 0)
        return 1;
    const ldpc_code_s *c = j.code;
    const bool qc = fused_qc_view(c, sizeof(float));
    const size_t two = fused::frame_lds_bytes(c->E, c->n, qc ? c->qc_words : 0, qc ? c->nblocks : 0,
                                              qc ? c->mb : 0, sizeof(float), 2);
    return two <= limit ? 2 : 1;
}

// Packing of the fusable jobs into launch groups (at most max_groups): jobs
// that run with the same frames per workgroup (job_fpw of cfg.fpw) and the
// same workgroup size (job_threads) form a class; classes are packed in the
// order of their first job, the jobs of a class in job order, and a group
// closes at kMaxJobs jobs, at kMaxCodes codes, or when one more code would
// not fit its LDS.  Jobs whose code does not fit go to plain[] (*nplain of
// them), or, with plain == nullptr, make the plan fail.  Returns the group
// count or kPlanNotFused / kPlanTooMany.  Allocates nothing.
int plan(const ldpc_job *jobs, int32_t njobs, ldpc_dtype dt, const LaunchCfg &cfg, Group *groups, int max_groups,
         int32_t *plain, int32_t *nplain)
{
    const size_t limit = lds_limit();
    const size_t tsize = dt == LDPC_F64 ? sizeof(double) : sizeof(float);
    constexpr int kMaxClasses = 2 * 8;  // frames per workgroup 1, 2 x workgroup sizes 64 .. 512
    int cls_fpw[kMaxClasses], cls_threads[kMaxClasses], ncls = 0;
    if (nplain)
        *nplain = 0;
    for (int32_t i = 0; i < njobs; ++i) {
        if (jobs[i].frames == 0)
            continue;
        if (!fused_fit(jobs[i].code, dt, limit).ok) {
            if (!plain)
                return kPlanNotFused;
            plain[(*nplain)++] = i;
            continue;
        }
        const int fpw = job_fpw(jobs[i], dt, cfg.fpw, limit), threads = job_threads(jobs[i], dt, cfg.threads);
        int c = 0;
        while (c < ncls && (cls_fpw[c] != fpw || cls_threads[c] != threads))
            ++c;
        if (c == ncls) {
            cls_fpw[ncls] = fpw;
            cls_threads[ncls++] = threads;
        }
    }
    int ng = 0;
    for (int c = 0; c < ncls; ++c) {
        const int first = ng;  // a job joins only the last group of its own class
        for (int32_t i = 0; i < njobs; ++i) {
            if (jobs[i].frames == 0)
                continue;
            const FusedFit fit = fused_fit(jobs[i].code, dt, limit);
            if (!fit.ok || job_fpw(jobs[i], dt, cfg.fpw, limit) != cls_fpw[c] ||
                job_threads(jobs[i], dt, cfg.threads) != cls_threads[c])
                continue;
            bool need_new = ng == first || groups[ng - 1].njobs == fused::kMaxJobs;
            if (!need_new && groups[ng - 1].code_index(jobs[i].code) < 0) {
                Group trial = groups[ng - 1];
                trial.add_code(jobs[i].code);
                need_new = groups[ng - 1].ncodes == fused::kMaxCodes || trial.lds() > limit;
            }
            if (need_new) {
                if (ng == max_groups)
                    return kPlanTooMany;
                groups[ng++] = Group{};
                groups[ng - 1].tsize = tsize;
                groups[ng - 1].fpw = cls_fpw[c];
                groups[ng - 1].threads = cls_threads[c];
            }
            Group &g = groups[ng - 1];
            g.jobs[g.njobs++] = i;
            if (g.code_index(jobs[i].code) < 0)
                g.add_code(jobs[i].code);
            g.bucket = std::max(g.bucket, fit.bucket);
        }
    }
    return ng;
}

constexpr size_t kGroupBytes = (sizeof(fused::Batch) + 255) / 256 * 256 + 256;

// Writes a launch's batch table (passed by value as the kernel argument, so
// nothing on the host must outlive the call, and the launch sequence can be
// captured in a graph) and resets the launch's work counter.
__global__ __launch_bounds__(256) void k_store_batch(fused::Batch b, fused::Batch *__restrict__ dst,
                                                     unsigned long long *counter)
{
    const int32_t *src = reinterpret_cast<const int32_t *>(&b);
    int32_t *out = reinterpret_cast<int32_t *>(dst);
    for (int w = threadIdx.x; w < static_cast<int>(sizeof(fused::Batch) / sizeof(int32_t)); w += blockDim.x)
        out[w] = src[w];
    if (threadIdx.x == 0)
        *counter = 0ull;
}

ldpc_status validate_jobs(const ldpc_job *jobs, int32_t njobs, ldpc_dtype dtype)
{
    if (njobs < 0 || (njobs > 0 && !jobs) || (dtype != LDPC_F32 && dtype != LDPC_F64))
        return LDPC_EINVAL;
    for (int32_t i = 0; i < njobs; ++i) {
        const ldpc_job &j = jobs[i];
        if (!j.code || j.frames < 0 || j.frames > LDPC_MAX_FRAMES || j.max_iter < 0 ||
            (j.flags & ~(LDPC_EARLY_STOP | LDPC_LAYERED | LDPC_MIN_SUM)) != 0)
            return LDPC_EINVAL;
        if ((j.flags & LDPC_MIN_SUM) && !ldpc::minsum_params_ok(j.ms_scale, j.ms_offset))
            return LDPC_EINVAL;
        if (j.frames > 0 && (!j.llr || !j.bits || !j.iters))
            return LDPC_EINVAL;
        if (j.frames > 0 && !ldpc::code_on_current_device(j.code))
            return LDPC_EINVAL;
    }
    return LDPC_OK;
}

size_t batch_bytes(const ldpc_job *jobs, int ngroups, const int32_t *plain, int32_t nplain, ldpc_dtype dtype)
{
    size_t stream = 0;
    for (int32_t k = 0; k < nplain; ++k) {
        const ldpc_job &j = jobs[plain[k]];
        stream = std::max(stream, stream_workspace_bytes(j.code, dtype, j.frames, j.max_iter));
    }
    return static_cast<size_t>(ngroups) * kGroupBytes + stream;
}

fused::Code code_entry(const ldpc_code_s *c, size_t tsize)
{
    const bool qc = fused_qc_view(c, tsize);
    fused::Code e{};
    e.m = c->m;
    e.n = c->n;
    e.E = static_cast<int32_t>(c->E);
    e.Z = qc ? c->Z : 1;
    e.nblocks = qc ? c->nblocks : 0;
    e.mb = qc ? c->mb : 0;
    e.nb = qc ? c->nb : 0;
    e.qc = qc ? 1 : 0;
    e.words = qc ? c->qc_words : 0;
    e.zmagic = qc ? static_cast<uint32_t>(((1ull << 32) + static_cast<uint64_t>(c->Z) - 1) / static_cast<uint64_t>(c->Z))
                  : 0u;
    e.tab = c->qc_tab;
    e.row_ptr = c->row_ptr;
    e.col_idx = c->col_idx;
    e.col_ptr = c->col_ptr;
    e.col_edge = c->col_edge;
    e.brow_order = c->brow_order;
    e.row_gmax = c->row_gmax;
    e.col_gmax = c->col_gmax;
    e.layer_ptr = c->d_layer_ptr;
    e.nlayers = static_cast<int32_t>(c->layer_dmax.size());
    e.half_rows = qc ? c->half_rows : nullptr;
    return e;
}

// Writes group g's batch table into ws (kGroupBytes: the table, then the
// work counter in its last 256 bytes) with a kernel, and launches the fused
// kernel on it.  profile: as launch_fused_bucket.
template <class A>
ldpc_status launch_group(const ldpc_job *jobs, const Group &g, char *ws, int threads, hipStream_t s, bool profile)
{
    fused::Batch b{};
    b.njobs = g.njobs;
    b.ncodes = g.ncodes;
    int32_t nblocks_max = 0;
    for (int32_t k = 0; k < g.ncodes; ++k) {
        const ldpc_code_s *c = g.codes[k];
        b.codes[k] = code_entry(c, sizeof(typename A::T));
        b.emax = std::max<int32_t>(b.emax, static_cast<int32_t>(c->E));
        b.nmax = std::max(b.nmax, c->n);
        b.words_max = std::max(b.words_max, b.codes[k].words);
        b.mb_max = std::max(b.mb_max, b.codes[k].mb);
        nblocks_max = std::max(nblocks_max, b.codes[k].nblocks);
    }
    int64_t items = 0;
    const int fpw = g.fpw;
    for (int32_t k = 0; k < g.njobs; ++k) {
        const ldpc_job &j = jobs[g.jobs[k]];
        fused::Job &e = b.jobs[k];
        e.code = g.code_index(j.code);
        e.frames = j.frames;
        e.max_iter = j.max_iter;
        e.flags = j.flags;
        e.ms_scale = j.ms_scale;
        e.ms_offset = j.ms_offset;
        e.item_begin = items;
        e.llr = j.llr;
        e.bits = j.bits;
        e.iters = j.iters;
        e.post = j.posterior;
        items += (j.frames + fpw - 1) / fpw;  // one item per frame, or per pair of frames
    }
    b.nitems = items;
    const size_t lds = fused::frame_lds_bytes(b.emax, b.nmax, b.words_max, nblocks_max, b.mb_max,
                                              sizeof(typename A::T), fpw);
    auto *d_batch = reinterpret_cast<fused::Batch *>(ws);
    auto *counter = reinterpret_cast<unsigned long long *>(ws + kGroupBytes - 256);
    {
        ProfScope ps(LDPC_KERNEL_OTHER, s, profile);
        LDPC_LAUNCH(ps, k_store_batch, dim3(1), dim3(256), 0, s, b, d_batch, counter);
    }
    switch (g.bucket) {
    case 8: return launch_fused_bucket<A, 8>(b, d_batch, counter, lds, threads, fpw, s, profile);
    case 16: return launch_fused_bucket<A, 16>(b, d_batch, counter, lds, threads, fpw, s, profile);
    case 24:
        if constexpr (std::is_same<A, ArithF32>::value)
            return launch_fused_bucket<A, 24>(b, d_batch, counter, lds, threads, fpw, s, profile);
        return launch_fused_bucket<A, 32>(b, d_batch, counter, lds, threads, fpw, s, profile);
    default: return launch_fused_bucket<A, 32>(b, d_batch, counter, lds, threads, fpw, s, profile);
    }
}

}  // namespace

size_t fused_group_bytes() { return kGroupBytes; }

}  // namespace ldpc

// Scratch memory of ldpc_decode_batch_noalloc: the batch tables and work
// counters of up to LDPC_NOALLOC_MAX_GROUPS launch groups, one kGroupBytes
// slice each, as ldpc_decode_batch lays them out in its workspace.  Every
// device holds its own copy for the life of the process.  Host code never
// uses this name as an address: it uses the per-device address that
// hipGetSymbolAddress returns (noalloc_scratch).
constexpr size_t kNoallocScratchBytes = static_cast<size_t>(LDPC_NOALLOC_MAX_GROUPS) * ldpc::kGroupBytes;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

namespace ldpc {
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];  // device address of `scratch`, per device, once looked up

// The current device's address of `scratch`, looked up on the first call
// on each device (with that device current) and kept.
ldpc_status noalloc_scratch(char **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0)
        return LDPC_EDEVICE;
    if (dev >= kMaxDevices)
        return LDPC_EUNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p)
            return LDPC_EDEVICE;
        g_scratch_ptr[dev] = p;
    }
    *out = static_cast<char *>(g_scratch_ptr[dev]);
    return LDPC_OK;
}

}  // namespace
}  // namespace ldpc

using namespace ldpc;

namespace {

// The full plan of a batch: launch groups and the jobs for the plain path.
struct FullPlan {
    std::vector<Group> groups;
    std::vector<int32_t> plain;
    int ngroups = 0;
    int32_t nplain = 0;
    void make(const ldpc_job *jobs, int32_t njobs, ldpc_dtype dtype, const LaunchCfg &cfg)
    {
        groups.resize(std::max(njobs, 1));
        plain.resize(std::max(njobs, 1));
        ngroups = plan(jobs, njobs, dtype, cfg, groups.data(), static_cast<int>(groups.size()), plain.data(),
                       &nplain);
    }
};

// Workspace of a batch under any launch configuration (the autotuner tries
// them in the caller's workspace, and tuning may split a batch into more
// launches later): one group table per fused job at most, and the plain
// path's largest workspace.
size_t batch_bytes_any(const ldpc_job *jobs, int32_t njobs, ldpc_dtype dtype)
{
    FullPlan p;
    p.make(jobs, njobs, dtype, LaunchCfg{});
    int32_t fused_jobs = 0;
    for (int32_t i = 0; i < njobs; ++i)
        fused_jobs += jobs[i].frames > 0 ? 1 : 0;
    fused_jobs -= p.nplain;
    return static_cast<size_t>(fused_jobs) * kGroupBytes + batch_bytes(jobs, 0, p.plain.data(), p.nplain, dtype);
}

}  // namespace

extern "C" ldpc_status ldpc_batch_workspace_bytes(const ldpc_job *jobs, int32_t njobs, ldpc_dtype dtype,
                                                  size_t *bytes)
try {
    if (!bytes)
        return LDPC_EINVAL;
    const ldpc_status st = validate_jobs(jobs, njobs, dtype);
    if (st != LDPC_OK)
        return st;
    *bytes = batch_bytes_any(jobs, njobs, dtype);
    return LDPC_OK;
} catch (...) {
    return ldpc::status_of_exception();
}

extern "C" ldpc_status ldpc_decode_batch(const ldpc_job *jobs, int32_t njobs, ldpc_dtype dtype, void *workspace,
                                         size_t workspace_bytes, void *stream)
try {
    const ldpc_status st = validate_jobs(jobs, njobs, dtype);
    if (st != LDPC_OK)
        return st;
    const LaunchCfg cfg = cfg_for(jobs, njobs, dtype);
    FullPlan p;
    p.make(jobs, njobs, dtype, cfg);
    const size_t need = batch_bytes(jobs, p.ngroups, p.plain.data(), p.nplain, dtype);
    if (need == 0)
        return LDPC_OK;
    if (!workspace || workspace_bytes < need || (reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
        return LDPC_EINVAL;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    char *ws = static_cast<char *>(workspace);
    for (int gi = 0; gi < p.ngroups; ++gi) {
        const Group &g = p.groups[gi];
        const ldpc_status r = dtype == LDPC_F64 ? launch_group<ArithF64>(jobs, g, ws, g.threads, s, true)
                                                : launch_group<ArithF32>(jobs, g, ws, g.threads, s, true);
        if (r != LDPC_OK)
            return r;
        ws += kGroupBytes;
    }
    for (int32_t k = 0; k < p.nplain; ++k) {
        const ldpc_job &j = jobs[p.plain[k]];
        const ldpc_status r = stream_decode(j.code, dtype, j.frames, j.max_iter, j.flags, j.llr, j.bits, j.iters,
                                            j.posterior, ws, s, j.ms_scale, j.ms_offset);
        if (r != LDPC_OK)
            return r;
    }
    return LDPC_OK;
} catch (...) {
    return ldpc::status_of_exception();
}

extern "C" ldpc_status ldpc_decode_batch_noalloc(const ldpc_job *jobs, int32_t njobs, ldpc_dtype dtype,
                                                 void *stream)
try {
    const ldpc_status st = validate_jobs(jobs, njobs, dtype);
    if (st != LDPC_OK)
        return st;
    const LaunchCfg cfg = cfg_for(jobs, njobs, dtype);
    Group groups[LDPC_NOALLOC_MAX_GROUPS];
    const int ng = plan(jobs, njobs, dtype, cfg, groups, LDPC_NOALLOC_MAX_GROUPS, nullptr, nullptr);
    if (ng < 0)
        return LDPC_EUNSUPPORTED;  // a code too large for the fused kernel, or more groups than the scratch holds
    if (ng == 0)
        return LDPC_OK;
    char *ws = nullptr;
    const ldpc_status sc = noalloc_scratch(&ws);
    if (sc != LDPC_OK)
        return sc;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    for (int gi = 0; gi < ng; ++gi) {
        const ldpc_status r = dtype == LDPC_F64
                                  ? launch_group<ArithF64>(jobs, groups[gi], ws, groups[gi].threads, s, false)
                                  : launch_group<ArithF32>(jobs, groups[gi], ws, groups[gi].threads, s, false);
        if (r != LDPC_OK)
            return r;
        ws += kGroupBytes;
    }
    return LDPC_OK;
} catch (...) {
    return ldpc::status_of_exception();
}

extern "C" ldpc_status ldpc_batch_set_threads(int32_t threads)
try {
    if (threads < 64 || threads > 512 || threads % 64 != 0)
        return LDPC_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    g_cfg.threads = threads;
    return LDPC_OK;
} catch (...) {
    return ldpc::status_of_exception();
}

extern "C" ldpc_status ldpc_batch_set_frames_per_group(int32_t frames)
try {
    if (frames != 1 && frames != 2)
        return LDPC_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    g_cfg.fpw = frames;
    return LDPC_OK;
} catch (...) {
    return ldpc::status_of_exception();
}

extern "C" ldpc_status ldpc_batch_launch_config(const ldpc_job *jobs, int32_t njobs, ldpc_dtype dtype,
                                                int32_t *threads, int32_t *frames_per_group, int32_t *tuned)
try {
    const ldpc_status st = validate_jobs(jobs, njobs, dtype);
    if (st != LDPC_OK)
        return st;
    LaunchCfg cfg;
    bool found = false;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        cfg = g_cfg;
        auto it = g_tuned.find(shape_key(jobs, njobs, dtype));
        found = it != g_tuned.end();
        if (found)
            cfg = it->second.cfg;
    }
    int t = cfg.threads;
    const size_t limit = lds_limit();
    for (int32_t i = 0; i < njobs; ++i)
        if (jobs[i].frames > 0 && fused_fit(jobs[i].code, dtype, limit).ok) {
            t = job_threads(jobs[i], dtype, cfg.threads);
            break;
        }
    if (threads)
        *threads = t;
    if (frames_per_group)
        *frames_per_group = cfg.fpw;
    if (tuned)
        *tuned = found;
    return LDPC_OK;
} catch (...) {
    return ldpc::status_of_exception();
}

extern "C" ldpc_status ldpc_batch_job_threads(const ldpc_job *jobs, int32_t njobs, ldpc_dtype dtype, int32_t *threads)
try {
    const ldpc_status st = validate_jobs(jobs, njobs, dtype);
    if (st != LDPC_OK)
        return st;
    if (njobs > 0 && !threads)
        return LDPC_EINVAL;
    const LaunchCfg cfg = cfg_for(jobs, njobs, dtype);
    const size_t limit = lds_limit();
    for (int32_t i = 0; i < njobs; ++i)
        threads[i] = jobs[i].frames > 0 && fused_fit(jobs[i].code, dtype, limit).ok
                         ? job_threads(jobs[i], dtype, cfg.threads)
                         : 0;
    return LDPC_OK;
} catch (...) {
    return ldpc::status_of_exception();
}

extern "C" void ldpc_tuning_clear(void)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_tuned.clear();
    g_code_tuned.clear();
}

// Tuning file: one line per entry, "<arch> <key> <threads> <frames per
// workgroup> <ms>", key in hex; a per-code entry (workgroup size of one
// code's jobs) has frames per workgroup 0.  Entries of another architecture
// keep their line but, their key including the architecture, never match
// here.
extern "C" ldpc_status ldpc_tuning_save(const char *path)
try {
    if (!path)
        return LDPC_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    uint64_t arch = 0;
    const char *name = arch_of_current(&arch);
    FILE *f = std::fopen(path, "w");
    if (!f)
        return LDPC_EINVAL;
    for (const auto *table : {&g_tuned, &g_code_tuned})
        for (const auto &e : *table)
            std::fprintf(f, "%s %016llx %d %d %.6f\n", name[0] ? name : "unknown",
                         static_cast<unsigned long long>(e.first), e.second.cfg.threads, e.second.cfg.fpw,
                         e.second.ms);
    return std::fclose(f) == 0 ? LDPC_OK : LDPC_EINVAL;
} catch (...) {
    return ldpc::status_of_exception();
}

extern "C" ldpc_status ldpc_tuning_load(const char *path, int32_t *entries)
try {
    if (!path)
        return LDPC_EINVAL;
    FILE *f = std::fopen(path, "r");
    if (!f)
        return LDPC_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    char arch[128];
    unsigned long long key = 0;
    int threads = 0, fpw = 0;
    double ms = 0.0;
    int32_t count = 0;
    ldpc_status rc = LDPC_OK;
    for (;;) {
        const int got = std::fscanf(f, "%127s %llx %d %d %lf", arch, &key, &threads, &fpw, &ms);
        if (got == EOF)
            break;
        if (got != 5 || threads < 64 || threads > 512 || threads % 64 != 0 || fpw < 0 || fpw > 2) {
            rc = LDPC_EINVAL;  // malformed: the entries read so far are kept
            break;
        }
        Tuned t;
        t.cfg.threads = threads;
        t.cfg.fpw = fpw;
        t.ms = ms;
        (fpw == 0 ? g_code_tuned : g_tuned)[static_cast<uint64_t>(key)] = t;
        ++count;
    }
    std::fclose(f);
    if (entries)
        *entries = count;
    return rc;
} catch (...) {
    return ldpc::status_of_exception();
}

extern "C" ldpc_status ldpc_batch_fits_fused(ldpc_code code, ldpc_dtype dtype, size_t *lds_bytes)
try {
    if (!code || (dtype != LDPC_F32 && dtype != LDPC_F64))
        return LDPC_EINVAL;
    if (!code_on_current_device(code))
        return LDPC_EINVAL;
    const FusedFit f = fused_fit(code, dtype, lds_limit());
    if (lds_bytes)
        *lds_bytes = f.lds;
    return f.ok ? LDPC_OK : LDPC_EUNSUPPORTED;
} catch (...) {
    return ldpc::status_of_exception();
}

namespace {

// Outputs of every job copied to the host (for the candidates' bitwise check).
ldpc_status snapshot(const ldpc_job *jobs, int32_t njobs, ldpc_dtype dt, hipStream_t s, std::vector<char> &out)
{
    out.clear();
    const size_t ts = dt == LDPC_F64 ? 8 : 4;
    for (int32_t i = 0; i < njobs; ++i) {
        const ldpc_job &j = jobs[i];
        const size_t fn = static_cast<size_t>(j.frames) * static_cast<size_t>(j.code->n);
        const size_t at = out.size();
        out.resize(at + fn + 4 * static_cast<size_t>(j.frames) + (j.posterior ? fn * ts : 0));
        if (hipMemcpyAsync(out.data() + at, j.bits, fn, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpyAsync(out.data() + at + fn, j.iters, 4 * static_cast<size_t>(j.frames), hipMemcpyDeviceToHost,
                           s) != hipSuccess)
            return LDPC_EDEVICE;
        if (j.posterior && hipMemcpyAsync(out.data() + at + fn + 4 * static_cast<size_t>(j.frames), j.posterior,
                                          fn * ts, hipMemcpyDeviceToHost, s) != hipSuccess)
            return LDPC_EDEVICE;
    }
    return hipStreamSynchronize(s) == hipSuccess ? LDPC_OK : LDPC_EDEVICE;
}

}  // namespace

namespace {

// Times `reps` decodes of a batch after one warm-up whose outputs are
// checked against `ref` (taken from this warm-up when ref is empty).
ldpc_status time_candidate(const ldpc_job *jobs, int32_t njobs, ldpc_dtype dtype, void *workspace,
                           size_t workspace_bytes, hipStream_t s, hipEvent_t e0, hipEvent_t e1,
                           std::vector<char> &ref, std::vector<char> &cur, double &ms_out)
{
    constexpr int kReps = 3;
    ldpc_status rc = ldpc_decode_batch(jobs, njobs, dtype, workspace, workspace_bytes, s);
    if (rc == LDPC_OK)
        rc = snapshot(jobs, njobs, dtype, s, cur);
    if (rc != LDPC_OK)
        return rc;
    if (ref.empty())
        ref = cur;
    else if (ref.size() != cur.size() || std::memcmp(ref.data(), cur.data(), ref.size()) != 0)
        return LDPC_EDEVICE;  // a launch shape changed the results: never expected, refuse to tune
    (void)hipEventRecord(e0, s);
    for (int r = 0; r < kReps && rc == LDPC_OK; ++r)
        rc = ldpc_decode_batch(jobs, njobs, dtype, workspace, workspace_bytes, s);
    (void)hipEventRecord(e1, s);
    float ms = 0.f;
    if (rc != LDPC_OK)
        return rc;
    if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
        return LDPC_EDEVICE;
    ms_out = ms / kReps;
    return LDPC_OK;
}

}  // namespace

// Two stages.  Per code (device architecture, shape, dtype, flags): the jobs
// of that code alone, at each workgroup size; the fastest is recorded for
// the code and used by every later batch (small codes keep more frames per
// CU in flight with smaller workgroups, large ones decode each frame faster
// with larger ones; jobs of different sizes run as separate launches).  Per
// batch shape: frames per workgroup 1, and 2 where some job can use it, with
// the per-code sizes.  Every candidate's outputs must equal the first run's.
extern "C" ldpc_status ldpc_autotune_batch(const ldpc_job *jobs, int32_t njobs, ldpc_dtype dtype, void *workspace,
                                           size_t workspace_bytes, void *stream, int32_t *best_threads,
                                           double *best_ms)
try {
    const ldpc_status st = validate_jobs(jobs, njobs, dtype);
    if (st != LDPC_OK)
        return st;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    static const int kThreads[] = {64, 128, 192, 256, 384, 512};
    const size_t limit = lds_limit();
    uint64_t key = 0;
    int default_threads = 512;
    std::vector<uint64_t> ckeys;
    std::vector<std::vector<ldpc_job>> subs;
    int fpw_max = 1;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        key = shape_key(jobs, njobs, dtype);
        default_threads = g_cfg.threads;
        for (int32_t i = 0; i < njobs; ++i) {
            if (jobs[i].frames == 0 || !fused_fit(jobs[i].code, dtype, limit).ok)
                continue;
            if (job_fpw(jobs[i], dtype, 2, limit) == 2)
                fpw_max = 2;
            const uint64_t ck = code_key(jobs[i], dtype);
            size_t c = 0;
            while (c < ckeys.size() && ckeys[c] != ck)
                ++c;
            if (c == ckeys.size()) {
                ckeys.push_back(ck);
                subs.emplace_back();
            }
            subs[c].push_back(jobs[i]);
        }
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0)
            (void)hipEventDestroy(e0);
        return LDPC_EDEVICE;
    }
    std::vector<char> ref, cur;
    ldpc_status rc = LDPC_OK;
    // stage 1: workgroup size per code
    for (size_t c = 0; c < ckeys.size() && rc == LDPC_OK; ++c) {
        std::vector<char> cref;
        int best_t = 0;
        double best = 0.0;
        for (int threads : kThreads) {
            {
                std::lock_guard<std::mutex> lk(g_mu);
                g_code_tuned[ckeys[c]] = Tuned{LaunchCfg{threads, 0}, 0.0};
            }
            double ms = 0.0;
            rc = time_candidate(subs[c].data(), static_cast<int32_t>(subs[c].size()), dtype, workspace,
                                workspace_bytes, s, e0, e1, cref, cur, ms);
            if (rc != LDPC_OK)
                break;
            if (best_t == 0 || ms < best) {
                best_t = threads;
                best = ms;
            }
        }
        if (rc == LDPC_OK) {
            std::lock_guard<std::mutex> lk(g_mu);
            g_code_tuned[ckeys[c]] = Tuned{LaunchCfg{best_t, 0}, best};
        }
    }
    // stage 2: frames per workgroup for the whole batch
    LaunchCfg best_cfg{default_threads, 1};
    double best_t = 0.0;
    bool have = false;
    for (int fpw = 1; fpw <= fpw_max && rc == LDPC_OK; ++fpw) {
        const LaunchCfg cand{default_threads, fpw};
        {
            std::lock_guard<std::mutex> lk(g_mu);
            g_tuned[key] = Tuned{cand, 0.0};
        }
        double ms = 0.0;
        rc = time_candidate(jobs, njobs, dtype, workspace, workspace_bytes, s, e0, e1, ref, cur, ms);
        if (rc == LDPC_OK && (!have || ms < best_t)) {
            best_cfg = cand;
            best_t = ms;
            have = true;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != LDPC_OK || !have) {
        std::lock_guard<std::mutex> lk(g_mu);
        g_tuned.erase(key);
        for (const uint64_t ck : ckeys)
            g_code_tuned.erase(ck);
        return rc != LDPC_OK ? rc : LDPC_EDEVICE;
    }
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_tuned[key] = Tuned{best_cfg, best_t};
    }
    if (best_threads) {
        *best_threads = best_cfg.threads;
        for (int32_t i = 0; i < njobs; ++i)
            if (jobs[i].frames > 0 && fused_fit(jobs[i].code, dtype, limit).ok) {
                *best_threads = job_threads(jobs[i], dtype, best_cfg.threads);
                break;
            }
    }
    if (best_ms)
        *best_ms = best_t;
    return LDPC_OK;
} catch (...) {
    return ldpc::status_of_exception();
}
