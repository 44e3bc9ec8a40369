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

// Opt-in count of launches per kernel instantiation (name plus template
// arguments), so that tests can check which variant a call ran.  Off by
// default; ckc_variant_enable turns it on and clears the counts.
extern bool g_variant_on;
void count_variant_slow(const char *base, int a, int b, const char *suffix);
inline void count_variant(const char *base, int a = -1, int b = -1, const char *suffix = "") {
    if (g_variant_on) count_variant_slow(base, a, b, suffix);
}
