// Plans: the launch sequence of one ldpc_decode_batch call, captured once in
// a HIP graph and replayed.  Everything the sequence needs is in kernels
// (the batch tables travel as kernel arguments, counters are reset by a
// kernel), so the graph holds kernel nodes only.
#include "ldpc_internal.h"

struct ldpc_plan_s {
    int device = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

extern "C" ldpc_status ldpc_plan_create(const ldpc_job *jobs, int32_t njobs, ldpc_dtype dtype, void *workspace,
                                        size_t workspace_bytes, ldpc_plan *out)
try {
    if (!out)
        return LDPC_EINVAL;
    size_t need = 0;
    ldpc_status st = ldpc_batch_workspace_bytes(jobs, njobs, dtype, &need);
    if (st != LDPC_OK)
        return st;
    if (need > 0 && (!workspace || workspace_bytes < need))
        return LDPC_EINVAL;
    auto *p = new (std::nothrow) ldpc_plan_s();
    if (!p)
        return LDPC_ENOMEM;
    hipStream_t s = nullptr;
    if (hipGetDevice(&p->device) != hipSuccess || hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
        delete p;
        return LDPC_EDEVICE;
    }
    st = LDPC_EDEVICE;
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) == hipSuccess) {
        const ldpc_status dec = ldpc_decode_batch(jobs, njobs, dtype, workspace, workspace_bytes, s);
        const hipError_t e = hipStreamEndCapture(s, &p->graph);
        if (dec != LDPC_OK)
            st = dec;
        else if (e == hipSuccess && hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0) == hipSuccess)
            st = LDPC_OK;
    }
    (void)hipStreamDestroy(s);
    if (st != LDPC_OK) {
        if (p->graph)
            (void)hipGraphDestroy(p->graph);
        delete p;
        return st;
    }
    *out = p;
    return LDPC_OK;
} catch (...) {
    return ldpc::status_of_exception();
}

extern "C" ldpc_status ldpc_plan_launch(ldpc_plan plan, void *stream)
try {
    if (!plan)
        return LDPC_EINVAL;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != plan->device)
        return LDPC_EINVAL;
    return hipGraphLaunch(plan->exec, static_cast<hipStream_t>(stream)) == hipSuccess ? LDPC_OK : LDPC_EDEVICE;
} catch (...) {
    return ldpc::status_of_exception();
}

extern "C" void ldpc_plan_destroy(ldpc_plan plan)
try {
    if (!plan)
        return;
    if (plan->exec)
        (void)hipGraphExecDestroy(plan->exec);
    if (plan->graph)
        (void)hipGraphDestroy(plan->graph);
    delete plan;
} catch (...) {
}
