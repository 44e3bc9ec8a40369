// Tunable launch choices: names, allowed values and the process-wide setting.
#include <atomic>
#include <string.h>
#include <string>

#include "ckc_internal.h"
#include "tune.h"

namespace {
struct KnobDef {
    const char *name;
    int def;
    int lo, hi;
};
constexpr KnobDef kDefs[TK_COUNT] = {
    {"conv_outs", 8, 8, 16},
    {"conv_imgs", 4, 1, 4},
    {"ks_batch", 64, 8, 64},
    {"conv_fuse", 1, 0, 1},
    {"conv_rows", 1, 1, 2},
};
std::atomic<int> g_val[TK_COUNT] = {{8}, {4}, {64}, {1}, {1}};

bool allowed(int k, int v) {
    if (v < kDefs[k].lo || v > kDefs[k].hi) return false;
    if (k == TK_CONV_OUTS) return v == 8 || v == 16;
    if (k == TK_CONV_IMGS) return v == 1 || v == 2 || v == 4;
    return true;
}
int find(const char *name) {
    for (int k = 0; k < TK_COUNT; ++k)
        if (strcmp(name, kDefs[k].name) == 0) return k;
    return -1;
}
}  // namespace

int tune_value(TuneKnob k) { return g_val[k].load(std::memory_order_relaxed); }

extern "C" int ckc_tune_set(const char *knob, int value) {
    CKC_REQUIRE(knob, CKC_EINVAL, "null knob name");
    const int k = find(knob);
    CKC_REQUIRE(k >= 0, CKC_EINVAL, std::string("unknown tuning knob ") + knob);
    CKC_REQUIRE(allowed(k, value), CKC_EINVAL, std::string("value not allowed for knob ") + knob);
    g_val[k].store(value, std::memory_order_relaxed);
    return CKC_OK;
}

extern "C" int ckc_tune_get(const char *knob, int *value) {
    CKC_REQUIRE(knob && value, CKC_EINVAL, "null argument");
    const int k = find(knob);
    CKC_REQUIRE(k >= 0, CKC_EINVAL, std::string("unknown tuning knob ") + knob);
    *value = g_val[k].load(std::memory_order_relaxed);
    return CKC_OK;
}
