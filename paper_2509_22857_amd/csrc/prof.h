// Opt-in launch timing: HIP events around launches of named kernel classes,
// with the algorithmic bytes each launch moves.  Off by default; when on, the
// events are recorded on the stream the kernel runs on.
#pragma once
#include <hip/hip_runtime.h>

enum ProfKernel {
    PK_NTT_FWD = 0,
    PK_NTT_INV,
    PK_BCONV,
    PK_KIP,
    PK_MODDOWN,
    PK_CONV_CONTRACT,
    PK_ACT_TENSOR,
    PK_RESCALE,
    PK_DENSE_MAC,
    PK_EW,
    PK_MAC,
    PK_TENSOR,
    PK_COPY,
    PK_COUNT
};

extern bool g_prof_on;

struct ProfScope {
    int kid;
    double bytes;
    double work;
    hipStream_t s;
    hipEvent_t a = nullptr, b = nullptr;
    ProfScope(int kid_, hipStream_t s_, double bytes_, double work_ = 0.0);
    ~ProfScope();
};

#define CKC_PROF(kid, stream, bytes, work) ProfScope _prof_scope_##__LINE__((kid), (stream), (bytes), (work))
