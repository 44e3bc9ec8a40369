// Launch timing registry behind ckc_prof_enable / ckc_prof_query.
#include <string.h>

#include <mutex>
#include <vector>

#include "ckc_internal.h"
#include "prof.h"

bool g_prof_on = false;

namespace {
struct Rec {
    int kid;
    double bytes, work;
    hipEvent_t a, b;
};
std::mutex g_mu;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;

hipEvent_t get_event() {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

const char *kNames[PK_COUNT] = {"ntt_fwd", "ntt_inv", "bconv", "kip", "moddown", "conv_contract",
                                "act_tensor", "rescale", "dense_mac", "ew", "mac_plain", "tensor", "copy"};
}  // namespace

ProfScope::ProfScope(int kid_, hipStream_t s_, double bytes_, double work_) : kid(kid_), bytes(bytes_), work(work_), s(s_) {
    if (!g_prof_on) return;
    a = get_event();
    b = get_event();
    if (a) (void)hipEventRecord(a, s);
}

ProfScope::~ProfScope() {
    if (!g_prof_on || !a || !b) return;
    (void)hipEventRecord(b, s);
    std::lock_guard<std::mutex> lk(g_mu);
    g_recs.push_back(Rec{kid, bytes, work, a, b});
}

extern "C" int ckc_prof_enable(int on) {
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto &r : g_recs) {
        g_pool.push_back(r.a);
        g_pool.push_back(r.b);
    }
    g_recs.clear();
    g_prof_on = on != 0;
    return CKC_OK;
}

extern "C" int ckc_prof_query(const char *name, int64_t *launches, double *total_ms, double *bytes, double *work) {
    CKC_REQUIRE(name && launches && total_ms && bytes && work, CKC_EINVAL, "null argument");
    int kid = -1;
    for (int i = 0; i < PK_COUNT; ++i)
        if (strcmp(name, kNames[i]) == 0) kid = i;
    CKC_REQUIRE(kid >= 0, CKC_EINVAL, std::string("unknown kernel class ") + name);
    std::lock_guard<std::mutex> lk(g_mu);
    int64_t n = 0;
    double ms = 0, by = 0, wk = 0;
    for (auto &r : g_recs) {
        if (r.kid != kid) continue;
        CKC_HIP(hipEventSynchronize(r.b));
        float t = 0;
        CKC_HIP(hipEventElapsedTime(&t, r.a, r.b));
        ++n;
        ms += t;
        by += r.bytes;
        wk += r.work;
    }
    *launches = n;
    *total_ms = ms;
    *bytes = by;
    *work = wk;
    return CKC_OK;
}
