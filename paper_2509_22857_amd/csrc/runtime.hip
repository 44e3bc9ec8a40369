// Native network runner: a plan (the layer program of one network, parsed
// once from JSON) executed for a batch of encrypted images through the
// library's own entry points.  Intermediate ciphertexts are allocated on the
// caller's stream and freed after their last use.
#include <stdlib.h>
#include <string.h>

#include <map>
#include <memory>
#include <string>
#include <vector>

#include "ckc_internal.h"

namespace {

// ---------------------------------------------------------------- JSON
// A small reader for the plan format: objects, arrays, numbers, strings
// (escapes \" and \\ only), true, false, null.
struct JVal {
    enum Kind { NUL, BOOL, NUM, STR, ARR, OBJ } kind = NUL;
    double num = 0;
    bool b = false;
    std::string str;
    std::vector<JVal> arr;
    std::vector<std::pair<std::string, JVal>> obj;
    const JVal *get(const char *key) const {
        for (const auto &kv : obj)
            if (kv.first == key) return &kv.second;
        return nullptr;
    }
};

struct JParser {
    const char *p;
    std::string err;
    void ws() {
        while (*p == ' ' || *p == '\n' || *p == '\t' || *p == '\r') ++p;
    }
    bool lit(const char *w) {
        const size_t n = strlen(w);
        if (strncmp(p, w, n) != 0) return false;
        p += n;
        return true;
    }
    bool str(std::string &out) {
        if (*p != '"') return false;
        ++p;
        while (*p && *p != '"') {
            if (*p == '\\') {
                ++p;
                if (*p != '"' && *p != '\\') return false;
            }
            out.push_back(*p++);
        }
        if (*p != '"') return false;
        ++p;
        return true;
    }
    bool value(JVal &v, int depth) {
        if (depth > 32) return false;
        ws();
        if (*p == '{') {
            v.kind = JVal::OBJ;
            ++p;
            ws();
            if (*p == '}') return ++p, true;
            for (;;) {
                ws();
                std::string k;
                if (!str(k)) return false;
                ws();
                if (*p++ != ':') return false;
                JVal x;
                if (!value(x, depth + 1)) return false;
                v.obj.emplace_back(std::move(k), std::move(x));
                ws();
                if (*p == ',') {
                    ++p;
                    continue;
                }
                if (*p == '}') return ++p, true;
                return false;
            }
        }
        if (*p == '[') {
            v.kind = JVal::ARR;
            ++p;
            ws();
            if (*p == ']') return ++p, true;
            for (;;) {
                JVal x;
                if (!value(x, depth + 1)) return false;
                v.arr.push_back(std::move(x));
                ws();
                if (*p == ',') {
                    ++p;
                    continue;
                }
                if (*p == ']') return ++p, true;
                return false;
            }
        }
        if (*p == '"') {
            v.kind = JVal::STR;
            return str(v.str);
        }
        if (lit("true")) return v.kind = JVal::BOOL, v.b = true, true;
        if (lit("false")) return v.kind = JVal::BOOL, v.b = false, true;
        if (lit("null")) return v.kind = JVal::NUL, true;
        char *end = nullptr;
        v.num = strtod(p, &end);
        if (end == p) return false;
        v.kind = JVal::NUM;
        p = end;
        return true;
    }
};

// ---------------------------------------------------------------- plan
enum StepOp { OP_CONV, OP_ACT, OP_DENSE, OP_POOL };

struct Step {
    StepOp op;
    int layer = -1;                 // index into the plan's layers (not for pool)
    int in = -1, out = -1;          // tensor ids
    int count = 0;                  // output ciphertexts per image
    int level = 0;                  // level the layer runs at
    bool rescale = false;           // one rescale after the layer
    int short_layer = -1, short_in = -1, short_level = 0;  // residual shortcut conv
    ckc_layout layout{};            // pool: the input's layout
    std::vector<int> free_after;    // tensors whose last use is this step
};

}  // namespace

struct ckc_plan {
    ckc_ctx *ctx = nullptr;
    std::vector<const ckc_layer *> layers;
    std::vector<Step> steps;
    int n_tensors = 0;
    int input = -1, input_count = 0, input_level = 0;
    int output = -1, output_count = 0, output_level = 0;
};

namespace {

int int_field(const JVal &o, const char *k, int *v, bool required = true) {
    const JVal *f = o.get(k);
    if (!f) {
        if (required) {
            ckc_set_error(std::string("plan: missing field ") + k);
            return CKC_EINVAL;
        }
        return CKC_OK;
    }
    CKC_REQUIRE(f->kind == JVal::NUM && f->num == double(int(f->num)), CKC_EINVAL,
                std::string("plan: field ") + k + " must be an integer");
    *v = int(f->num);
    return CKC_OK;
}

int tensor_id(std::map<std::string, int> &ids, const JVal &o, const char *k, bool create, int *id) {
    const JVal *f = o.get(k);
    CKC_REQUIRE(f && f->kind == JVal::STR, CKC_EINVAL, std::string("plan: field ") + k + " must be a tensor name");
    auto it = ids.find(f->str);
    if (it == ids.end()) {
        CKC_REQUIRE(create, CKC_EINVAL, "plan: tensor " + f->str + " is read before it is written");
        const int n = int(ids.size());
        ids[f->str] = n;
        *id = n;
    } else {
        CKC_REQUIRE(!create, CKC_EINVAL, "plan: tensor " + f->str + " is written twice");
        *id = it->second;
    }
    return CKC_OK;
}

struct DevCts {
    // one tensor of a pass: n ciphertexts in one device allocation
    uint64_t *base = nullptr;
    std::vector<ckc_ct> ct;
};

}  // namespace

extern "C" int ckc_batch_plan(ckc_ctx *c, const char *json, ckc_layer *const *layers, int n_layers,
                              ckc_plan **out) {
    CKC_REQUIRE(c && json && out && n_layers >= 0 && (n_layers == 0 || layers), CKC_EINVAL, "null argument");
    *out = nullptr;
    JParser jp{json, ""};
    JVal root;
    CKC_REQUIRE(jp.value(root, 0) && root.kind == JVal::OBJ, CKC_EINVAL, "plan: not a JSON object");
    auto P = std::make_unique<ckc_plan>();
    P->ctx = c;
    for (int i = 0; i < n_layers; ++i) {
        CKC_REQUIRE(layers[i], CKC_EINVAL, "plan: null layer handle");
        P->layers.push_back(layers[i]);
    }
    std::map<std::string, int> ids;
    const JVal *inp = root.get("input");
    CKC_REQUIRE(inp && inp->kind == JVal::OBJ, CKC_EINVAL, "plan: missing input");
    CKC_TRY(tensor_id(ids, *inp, "name", true, &P->input));
    CKC_TRY(int_field(*inp, "count", &P->input_count));
    CKC_TRY(int_field(*inp, "level", &P->input_level));
    CKC_REQUIRE(P->input_count > 0 && P->input_level >= 0 && P->input_level < c->nq, CKC_EINVAL,
                "plan: bad input shape");
    std::vector<int> count_of{P->input_count}, level_of{P->input_level};
    const JVal *steps = root.get("steps");
    CKC_REQUIRE(steps && steps->kind == JVal::ARR && !steps->arr.empty(), CKC_EINVAL, "plan: missing steps");
    for (const JVal &sj : steps->arr) {
        CKC_REQUIRE(sj.kind == JVal::OBJ, CKC_EINVAL, "plan: a step is not an object");
        const JVal *op = sj.get("op");
        CKC_REQUIRE(op && op->kind == JVal::STR, CKC_EINVAL, "plan: step without op");
        Step st;
        if (op->str == "conv") st.op = OP_CONV;
        else if (op->str == "act") st.op = OP_ACT;
        else if (op->str == "dense") st.op = OP_DENSE;
        else if (op->str == "pool") st.op = OP_POOL;
        else {
            ckc_set_error("plan: unknown op " + op->str);
            return CKC_EINVAL;
        }
        CKC_TRY(tensor_id(ids, sj, "in", false, &st.in));
        CKC_TRY(tensor_id(ids, sj, "out", true, &st.out));
        CKC_TRY(int_field(sj, "count", &st.count));
        CKC_TRY(int_field(sj, "level", &st.level));
        int rs = 0;
        CKC_TRY(int_field(sj, "rescale", &rs, false));
        st.rescale = rs != 0;
        CKC_REQUIRE(st.count > 0 && st.level >= (st.rescale ? 1 : 0) && st.level < c->nq, CKC_EINVAL,
                    "plan: bad step shape");
        CKC_REQUIRE(level_of[st.in] == st.level, CKC_ELEVEL, "plan: a step's input is not at its level");
        if (st.op == OP_POOL) {
            const JVal *lj = sj.get("layout");
            CKC_REQUIRE(lj && lj->kind == JVal::OBJ, CKC_EINVAL, "plan: pool without layout");
            CKC_TRY(int_field(*lj, "block", &st.layout.block));
            CKC_TRY(int_field(*lj, "row_stride", &st.layout.row_stride));
            CKC_TRY(int_field(*lj, "gap", &st.layout.gap));
            CKC_TRY(int_field(*lj, "height", &st.layout.height));
            CKC_TRY(int_field(*lj, "width", &st.layout.width));
            CKC_TRY(int_field(*lj, "members", &st.layout.members));
            CKC_TRY(int_field(*lj, "flags", &st.layout.flags, false));
            CKC_REQUIRE(st.count == count_of[st.in], CKC_EINVAL, "plan: pooling keeps the channel count");
        } else {
            CKC_TRY(int_field(sj, "layer", &st.layer));
            CKC_REQUIRE(st.layer >= 0 && st.layer < n_layers, CKC_EINVAL, "plan: layer index out of range");
        }
        if (st.op == OP_ACT) CKC_REQUIRE(st.count == count_of[st.in], CKC_EINVAL, "plan: activation keeps the count");
        if (const JVal *sh = sj.get("short")) {
            CKC_REQUIRE(st.op == OP_CONV && sh->kind == JVal::OBJ, CKC_EINVAL, "plan: shortcut only on a conv");
            CKC_TRY(int_field(*sh, "layer", &st.short_layer));
            CKC_TRY(int_field(*sh, "level", &st.short_level));
            CKC_TRY(tensor_id(ids, *sh, "in", false, &st.short_in));
            CKC_REQUIRE(st.short_layer >= 0 && st.short_layer < n_layers, CKC_EINVAL,
                        "plan: shortcut layer index out of range");
            CKC_REQUIRE(st.short_level <= level_of[st.short_in] && st.short_level >= 0, CKC_ELEVEL,
                        "plan: shortcut level above its input's");
        }
        count_of.push_back(st.count);
        level_of.push_back(st.rescale ? st.level - 1 : st.level);
        P->steps.push_back(st);
    }
    P->n_tensors = int(ids.size());
    const JVal *outn = root.get("output");
    CKC_REQUIRE(outn && outn->kind == JVal::STR && ids.count(outn->str), CKC_EINVAL, "plan: unknown output");
    P->output = ids[outn->str];
    P->output_count = count_of[P->output];
    P->output_level = level_of[P->output];
    // liveness: free every intermediate after the step that reads it last
    std::vector<int> last(P->n_tensors, -1);
    for (int i = 0; i < int(P->steps.size()); ++i) {
        last[P->steps[i].in] = i;
        if (P->steps[i].short_in >= 0) last[P->steps[i].short_in] = i;
    }
    for (int t = 0; t < P->n_tensors; ++t)
        if (t != P->input && t != P->output && last[t] >= 0) P->steps[last[t]].free_after.push_back(t);
    *out = P.release();
    return CKC_OK;
}

extern "C" int ckc_batch_plan_info(const ckc_plan *P, int *in_count, int *in_level, int *out_count,
                                   int *out_level) {
    CKC_REQUIRE(P, CKC_EINVAL, "null plan");
    if (in_count) *in_count = P->input_count;
    if (in_level) *in_level = P->input_level;
    if (out_count) *out_count = P->output_count;
    if (out_level) *out_level = P->output_level;
    return CKC_OK;
}

extern "C" int ckc_batch_plan_destroy(ckc_plan *P) {
    delete P;
    return CKC_OK;
}

namespace {

// one pass of the plan over n images that share one key set
int run_pass(ckc_plan *P, const ckc_evk *evk, ckc_ct *const *inputs, ckc_ct *const *outputs, int n,
             hipStream_t s) {
    ckc_ctx *c = P->ctx;
    std::vector<DevCts> T(P->n_tensors);
    auto release = [&](int t) {
        if (T[t].base) (void)hipFreeAsync(T[t].base, s);
        T[t] = DevCts{};
    };
    auto alloc = [&](int t, int count, int level) -> int {
        const size_t w = ckc_ct_words(c, level, 2);
        const size_t total = size_t(count) * n;
        hipError_t e = hipMallocAsync((void **)&T[t].base, 8 * w * total, s);
        if (e != hipSuccess) {
            T[t].base = nullptr;
            (void)hipGetLastError();
            ckc_set_error(std::string("batch run hipMallocAsync: ") + hipGetErrorString(e));
            return CKC_ENOMEM;
        }
        T[t].ct.resize(total);
        for (size_t i = 0; i < total; ++i) T[t].ct[i] = ckc_ct{T[t].base + i * w, level, 2, 1.0};
        return CKC_OK;
    };
    auto fail = [&](int rc) {
        for (int t = 0; t < P->n_tensors; ++t)
            if (t != P->input) release(t);
        return rc;
    };
    // the input tensor: the requests' ciphertexts, image-major
    T[P->input].ct.resize(size_t(P->input_count) * n);
    for (int r = 0; r < n; ++r)
        for (int i = 0; i < P->input_count; ++i) T[P->input].ct[size_t(r) * P->input_count + i] = inputs[r][i];
    for (const Step &st : P->steps) {
        const int cnt = st.count;
        int rc = alloc(st.out, cnt, st.level);
        if (rc != CKC_OK) return fail(rc);
        ckc_ct *in = T[st.in].ct.data(), *o = T[st.out].ct.data();
        const ckc_layer *L = st.layer >= 0 ? P->layers[st.layer] : nullptr;
        switch (st.op) {
            case OP_CONV: rc = ckc_eval_conv(c, evk, L, in, n, o, s); break;
            case OP_ACT: rc = ckc_eval_quad_act(c, evk, L, in, n, o, s); break;
            case OP_DENSE: rc = ckc_eval_dense(c, evk, L, in, n, o, s); break;
            case OP_POOL: rc = ckc_eval_avgpool2(c, evk, &st.layout, in, int(T[st.in].ct.size()), o, s); break;
        }
        if (rc != CKC_OK) return fail(rc);
        if (st.short_layer >= 0) {
            // residual: the shortcut input mod-dropped to the shortcut's
            // level, its 1x1 convolution, then added to the main branch
            std::vector<ckc_ct> xs = T[st.short_in].ct;
            DevCts dropped;
            if (!xs.empty() && xs[0].level != st.short_level) {
                const size_t w = ckc_ct_words(c, st.short_level, 2);
                hipError_t e = hipMallocAsync((void **)&dropped.base, 8 * w * xs.size(), s);
                if (e != hipSuccess) {
                    (void)hipGetLastError();
                    ckc_set_error(std::string("batch run hipMallocAsync: ") + hipGetErrorString(e));
                    return fail(CKC_ENOMEM);
                }
                for (size_t i = 0; i < xs.size() && rc == CKC_OK; ++i) {
                    ckc_ct d{dropped.base + i * w, st.short_level, 2, 1.0};
                    rc = ckc_mod_drop(c, &xs[i], st.short_level, &d, s);
                    xs[i] = d;
                }
            }
            DevCts sc;
            const size_t w = ckc_ct_words(c, st.short_level, 2);
            if (rc == CKC_OK) {
                hipError_t e = hipMallocAsync((void **)&sc.base, 8 * w * size_t(cnt) * n, s);
                if (e != hipSuccess) {
                    (void)hipGetLastError();
                    ckc_set_error(std::string("batch run hipMallocAsync: ") + hipGetErrorString(e));
                    rc = CKC_ENOMEM;
                }
            }
            if (rc == CKC_OK) {
                sc.ct.resize(size_t(cnt) * n);
                for (size_t i = 0; i < sc.ct.size(); ++i) sc.ct[i] = ckc_ct{sc.base + i * w, st.short_level, 2, 1.0};
                rc = ckc_eval_conv(c, evk, P->layers[st.short_layer], xs.data(), n, sc.ct.data(), s);
                if (rc == CKC_OK) rc = ckc_add_many(c, o, sc.ct.data(), int(sc.ct.size()), o, s);
            }
            if (dropped.base) (void)hipFreeAsync(dropped.base, s);
            if (sc.base) (void)hipFreeAsync(sc.base, s);
            if (rc != CKC_OK) return fail(rc);
        }
        if (st.rescale) {
            DevCts r;
            const size_t w = ckc_ct_words(c, st.level - 1, 2);
            hipError_t e = hipMallocAsync((void **)&r.base, 8 * w * T[st.out].ct.size(), s);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                ckc_set_error(std::string("batch run hipMallocAsync: ") + hipGetErrorString(e));
                return fail(CKC_ENOMEM);
            }
            r.ct.resize(T[st.out].ct.size());
            for (size_t i = 0; i < r.ct.size(); ++i) r.ct[i] = ckc_ct{r.base + i * w, st.level - 1, 2, 1.0};
            rc = ckc_rescale_many(c, o, int(r.ct.size()), r.ct.data(), s);
            release(st.out);
            T[st.out] = std::move(r);
            if (rc != CKC_OK) return fail(rc);
        }
        for (int t : st.free_after) release(t);
    }
    // results into the caller's buffers
    const DevCts &res = T[P->output];
    const size_t w = ckc_ct_words(c, P->output_level, 2);
    int rc = CKC_OK;
    for (int r = 0; r < n && rc == CKC_OK; ++r)
        for (int k = 0; k < P->output_count; ++k) {
            const ckc_ct &src = res.ct[size_t(r) * P->output_count + k];
            ckc_ct &dst = outputs[r][k];
            hipError_t e = hipMemcpyAsync(dst.d, src.d, 8 * w, hipMemcpyDeviceToDevice, s);
            if (e != hipSuccess) {
                ckc_set_error(std::string("batch run copy: ") + hipGetErrorString(e));
                rc = CKC_EDEVICE;
                break;
            }
            dst.level = src.level;
            dst.npoly = 2;
            dst.scale = src.scale;
        }
    return fail(rc);
}

}  // namespace

extern "C" int ckc_batch_run(ckc_plan *P, const ckc_evk *const *evks, ckc_ct *const *inputs, int n_requests,
                             ckc_ct *const *outputs, void *stream) {
    CKC_REQUIRE(P && evks && inputs && outputs && n_requests >= 0, CKC_EINVAL, "null argument");
    for (int r = 0; r < n_requests; ++r) {
        CKC_REQUIRE(evks[r] && inputs[r] && outputs[r], CKC_EINVAL, "null request entry");
        for (int i = 0; i < P->input_count; ++i)
            CKC_REQUIRE(inputs[r][i].d && inputs[r][i].level == P->input_level && inputs[r][i].npoly == 2,
                        CKC_ELEVEL, "batch run: an input is not a 2-poly ciphertext at the plan's input level");
        for (int k = 0; k < P->output_count; ++k)
            CKC_REQUIRE(outputs[r][k].d, CKC_EINVAL, "batch run: null output buffer");
    }
    const hipStream_t s = (hipStream_t)stream;
    // consecutive requests under one key set run as one pass (their images
    // share every key-switching and contraction launch)
    for (int r0 = 0; r0 < n_requests;) {
        int r1 = r0 + 1;
        while (r1 < n_requests && evks[r1] == evks[r0]) ++r1;
        CKC_TRY(run_pass(P, evks[r0], inputs + r0, outputs + r0, r1 - r0, s));
        r0 = r1;
    }
    return CKC_OK;
}
