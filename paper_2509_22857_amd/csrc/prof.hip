// Launch timing registry behind ckc_prof_enable / ckc_prof_query.
#include <stdio.h>
#include <string.h>

#include <map>
#include <mutex>
#include <string>
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

bool g_variant_on = false;

namespace {
std::mutex g_vmu;
std::map<std::string, int64_t> g_variants;
}  // namespace

void count_variant_slow(const char *base, int a, int b, const char *suffix) {
    char name[96];
    if (a < 0) snprintf(name, sizeof name, "%s%s", base, suffix);
    else if (b < 0) snprintf(name, sizeof name, "%s<%d>%s", base, a, suffix);
    else snprintf(name, sizeof name, "%s<%d,%d>%s", base, a, b, suffix);
    std::lock_guard<std::mutex> lk(g_vmu);
    ++g_variants[name];
}

extern "C" int ckc_variant_enable(int on) {
    std::lock_guard<std::mutex> lk(g_vmu);
    g_variants.clear();
    g_variant_on = on != 0;
    return CKC_OK;
}

extern "C" int ckc_variant_count(const char *name, int64_t *launches) {
    CKC_REQUIRE(name && launches, CKC_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(g_vmu);
    auto it = g_variants.find(name);
    *launches = it == g_variants.end() ? 0 : it->second;
    return CKC_OK;
}

extern "C" int ckc_variant_list(char *buf, size_t cap) {
    CKC_REQUIRE(buf && cap > 0, CKC_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(g_vmu);
    std::string s;
    for (auto &kv : g_variants) s += kv.first + "=" + std::to_string(kv.second) + "\n";
    CKC_REQUIRE(s.size() < cap, CKC_EINVAL, "variant list does not fit the buffer");
    snprintf(buf, cap, "%s", s.c_str());
    return CKC_OK;
}
