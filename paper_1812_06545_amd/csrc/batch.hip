// Batched decoding of jobs of different codes.
#include <algorithm>

#include "ldpc_internal.h"

namespace {

ldpc_status validate_jobs(const ldpc_job *jobs, int32_t njobs, ldpc_dtype dtype)
{
    if (njobs < 0 || (njobs > 0 && !jobs) || (dtype != LDPC_F32 && dtype != LDPC_F64))
        return LDPC_EINVAL;
    for (int32_t i = 0; i < njobs; ++i) {
        const ldpc_job &j = jobs[i];
        if (!j.code || j.frames < 0 || j.frames > LDPC_MAX_FRAMES || j.max_iter < 0 ||
            (j.flags & ~LDPC_EARLY_STOP) != 0)
            return LDPC_EINVAL;
        if (j.frames > 0 && (!j.llr || !j.bits || !j.iters))
            return LDPC_EINVAL;
        if (j.frames > 0 && !ldpc::code_on_current_device(j.code))
            return LDPC_EINVAL;
    }
    return LDPC_OK;
}

size_t batch_bytes(const ldpc_job *jobs, int32_t njobs, ldpc_dtype dtype)
{
    size_t b = 0;
    for (int32_t i = 0; i < njobs; ++i)
        if (jobs[i].frames > 0)
            b = std::max(b, ldpc::stream_workspace_bytes(jobs[i].code, dtype, jobs[i].frames, jobs[i].max_iter));
    return b;
}

}  // namespace

extern "C" ldpc_status ldpc_batch_workspace_bytes(const ldpc_job *jobs, int32_t njobs, ldpc_dtype dtype,
                                                  size_t *bytes)
{
    if (!bytes)
        return LDPC_EINVAL;
    const ldpc_status st = validate_jobs(jobs, njobs, dtype);
    if (st != LDPC_OK)
        return st;
    *bytes = batch_bytes(jobs, njobs, dtype);
    return LDPC_OK;
}

extern "C" ldpc_status ldpc_decode_batch(const ldpc_job *jobs, int32_t njobs, ldpc_dtype dtype, void *workspace,
                                         size_t workspace_bytes, void *stream)
{
    const ldpc_status st = validate_jobs(jobs, njobs, dtype);
    if (st != LDPC_OK)
        return st;
    const size_t need = batch_bytes(jobs, njobs, dtype);
    if (need == 0)
        return LDPC_OK;
    if (!workspace || workspace_bytes < need || (reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
        return LDPC_EINVAL;
    for (int32_t i = 0; i < njobs; ++i) {
        const ldpc_job &j = jobs[i];
        if (j.frames == 0)
            continue;
        const ldpc_status s = ldpc::stream_decode(j.code, dtype, j.frames, j.max_iter, j.flags, j.llr, j.bits,
                                                  j.iters, j.posterior, workspace, static_cast<hipStream_t>(stream));
        if (s != LDPC_OK)
            return s;
    }
    return LDPC_OK;
}
