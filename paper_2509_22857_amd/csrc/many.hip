// Batched evaluator operations (the Section 2.2 operations applied to whole
// batches of ciphertexts): hoisted rotations, multiplication with
// relinearisation, and plaintext multiply-accumulate.  Each launch covers up to
// kMaxBatch ciphertexts, so an evaluation key or a plaintext is read from HBM
// once per launch instead of once per ciphertext.
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "batch.h"
#include "prof.h"

uint64_t galois_element(const ckc_ctx *c, int64_t step);

namespace {

hipStream_t S(void *s) { return (hipStream_t)s; }
unsigned tiles(size_t N) { return unsigned(std::min<size_t>(N / 256, 64)); }

// every ciphertext non-null, at one level in range, with `npoly` polynomials
// and (if same_scale) scales within 2^-30 of the first
int check_batch(const ckc_ctx *c, const ckc_ct *in, int n, int npoly, const char *what, bool same_scale = true) {
    const int level = in[0].level;
    CKC_REQUIRE(level >= 0 && level < c->nq, CKC_ELEVEL, std::string(what) + ": level out of range");
    for (int i = 0; i < n; ++i) {
        CKC_REQUIRE(in[i].d, CKC_EINVAL, std::string(what) + ": null ciphertext");
        CKC_REQUIRE(in[i].level == level, CKC_ELEVEL, std::string(what) + ": ciphertext levels differ");
        CKC_REQUIRE(in[i].npoly == npoly, CKC_ESHAPE,
                    std::string(what) + ": expected " + std::to_string(npoly) + "-polynomial ciphertexts");
        CKC_REQUIRE(!same_scale || std::fabs(in[i].scale / in[0].scale - 1.0) <= std::ldexp(1.0, -30), CKC_ESCALE,
                    std::string(what) + ": ciphertext scales differ");
    }
    return CKC_OK;
}

// D[b] = (a0 b0, a0 b1 + a1 b0, a1 b1) in NTT form; grid (tiles, limbs, batch)
__global__ __launch_bounds__(256) void k_tensor_b(Ptrs a, Ptrs b, uint64_t *__restrict__ D, int nl,
                                                  const Prime *__restrict__ primes, int logN) {
    const int t = blockIdx.y, bi = blockIdx.z;
    const size_t N = size_t(1) << logN, pw = size_t(nl) * N;
    const Prime P = primes[t];
    const uint64_t *a0 = a.p[bi] + size_t(t) * N, *a1 = a0 + pw;
    const uint64_t *b0 = b.p[bi] + size_t(t) * N, *b1 = b0 + pw;
    uint64_t *d = D + bi * 3 * pw + size_t(t) * N;
    for (size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x; k < N; k += size_t(gridDim.x) * blockDim.x) {
        const uint64_t x0 = a0[k], x1 = a1[k], y0 = b0[k], y1 = b1[k];
        d[k] = mul_mod(x0, y0, P);
        d[pw + k] = reduce128(add128(mul64x64(x0, y1), mul64x64(x1, y0)), P);
        d[2 * pw + k] = mul_mod(x1, y1, P);
    }
}

// out[o] = sum_{t < T} in[o T + t] * pt[t] for the no outputs of one launch
// (no T <= kMaxBatch); grid (N / 256, limbs), one coefficient per thread.
// Each thread reads its T plaintext words once and reuses them for both
// polynomials of every output, so a launch reads each plaintext from HBM once
// (with a grid dimension per output and polynomial every block re-read them:
// 1.8x the algorithmic bytes).  Up to kMacRegTerms terms sit in registers;
// more are re-read per output, from cache.
constexpr int kMacRegTerms = 16;
__global__ __launch_bounds__(256) void k_mac_plain_b(Ptrs in, int T, Ptrs pt, Ptrs out, int no, int nl,
                                                     const Prime *__restrict__ primes, int logN) {
    const int limb = blockIdx.y;
    const size_t N = size_t(1) << logN;
    const size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const Prime P = primes[limb];
    const int pcap = fold_cap(P.k);
    const uint64_t r64 = P.r2;  // 2^64 mod q
    const size_t lo = size_t(limb) * N + k;
    uint64_t pv[kMacRegTerms];
#pragma unroll
    for (int t = 0; t < kMacRegTerms; ++t) pv[t] = t < T ? pt.p[t][lo] : 0;
    for (int o = 0; o < no; ++o) {
        for (int poly = 0; poly < 2; ++poly) {
            const size_t off = size_t(poly) * nl * N + lo;
            accc acc{0, 0, 0, 0, 0};
            int cnt = 0;
            auto step = [&](uint64_t x, uint64_t w) {
                macc(acc, x, w);
                if (++cnt == pcap) {
                    acc = macc_folded(acc, r64);
                    cnt = 0;
                }
            };
#pragma unroll
            for (int t = 0; t < kMacRegTerms; ++t)
                if (t < T) step(in.p[o * T + t][off], pv[t]);
            for (int t = kMacRegTerms; t < T; ++t) step(in.p[o * T + t][off], pt.p[t][lo]);
            out.p[o][off] = reduce128(accc_value(acc), P);
        }
    }
}

}  // namespace

extern "C" int ckc_rotate_many(ckc_ctx *c, const ckc_evk *evk, const ckc_ct *in, int n, const int32_t *steps,
                               int n_steps, ckc_ct *out, void *stream) {
    CKC_REQUIRE(c && evk && in && out && n >= 0 && n_steps >= 0 && (n_steps == 0 || steps), CKC_EINVAL,
                "null argument");
    CKC_REQUIRE(!evk->is_group(), CKC_EINVAL, "rotate_many: a key group serves layer calls only");
    if (n == 0 || n_steps == 0) return CKC_OK;
    CKC_TRY(check_batch(c, in, n, 2, "rotate_many"));
    const int level = in[0].level;
    for (int j = 0; j < n_steps; ++j) {
        const uint64_t g = galois_element(c, steps[j]);
        CKC_REQUIRE(g == 1 || evk->galois.count(g), CKC_ENOKEY,
                    "rotate_many: missing Galois key for step " + std::to_string(steps[j]));
    }
    for (int i = 0; i < n * n_steps; ++i) {
        CKC_REQUIRE(out[i].d, CKC_EINVAL, "rotate_many: null output");
        for (int b = 0; b < n; ++b)
            CKC_REQUIRE(out[i].d != in[b].d, CKC_EINVAL, "rotate_many: output aliases an input");
    }
    hipStream_t s = S(stream);
    const std::vector<int32_t> st(steps, steps + n_steps);
    for (int b0 = 0; b0 < n; b0 += kMaxBatch) {
        const int nb = std::min(kMaxBatch, n - b0);
        Ptrs ip{};
        std::vector<Ptrs> dst(n_steps);
        for (int b = 0; b < nb; ++b) {
            ip.p[b] = in[b0 + b].d;
            for (int j = 0; j < n_steps; ++j) dst[j].p[b] = out[size_t(b0 + b) * n_steps + j].d;
        }
        CKC_TRY(hoisted_group(c, evk, ip, nb, level, st, dst, s));
    }
    for (int i = 0; i < n * n_steps; ++i) {
        out[i].level = level;
        out[i].npoly = 2;
        out[i].scale = in[i / n_steps].scale;
    }
    return CKC_OK;
}

extern "C" int ckc_mul_relin_many(ckc_ctx *c, const ckc_evk *evk, const ckc_ct *a, const ckc_ct *b, int n,
                                  ckc_ct *out, void *stream) {
    CKC_REQUIRE(c && evk && a && b && out && n >= 0, CKC_EINVAL, "null argument");
    CKC_REQUIRE(!evk->is_group(), CKC_EINVAL, "mul_relin_many: a key group serves layer calls only");
    if (n == 0) return CKC_OK;
    CKC_REQUIRE(evk->relin, CKC_ENOKEY, "mul_relin_many: no relinearisation key");
    CKC_TRY(check_batch(c, a, n, 2, "mul_relin_many", false));
    CKC_TRY(check_batch(c, b, n, 2, "mul_relin_many", false));
    CKC_REQUIRE(a[0].level == b[0].level, CKC_ELEVEL, "mul_relin_many: operand levels differ");
    for (int i = 0; i < n; ++i) CKC_REQUIRE(out[i].d, CKC_EINVAL, "mul_relin_many: null output");
    hipStream_t s = S(stream);
    const size_t N = c->N;
    const int level = a[0].level, nl = level + 1, nt = nl + c->np, dnum = c->dnum_at(level);
    const size_t pw = size_t(nl) * N;
    const int nbmax = std::min(kMaxBatch, n);
    DevBuf D, digits;
    CKC_TRY(D.alloc(8 * 3 * pw * nbmax, s));
    CKC_TRY(digits.alloc(8 * N * nt * dnum * nbmax, s));
    for (int b0 = 0; b0 < n; b0 += kMaxBatch) {
        const int nb = std::min(kMaxBatch, n - b0);
        Ptrs ap{}, bp{}, d0{}, d1{}, o0{}, o1{};
        for (int i = 0; i < nb; ++i) {
            ap.p[i] = a[b0 + i].d;
            bp.p[i] = b[b0 + i].d;
            d0.p[i] = D.u64() + size_t(i) * 3 * pw;
            d1.p[i] = d0.p[i] + pw;
            o0.p[i] = out[b0 + i].d;
            o1.p[i] = out[b0 + i].d + pw;
        }
        {
            CKC_PROF(PK_TENSOR, s, 8.0 * N * nl * nb * 7.0, 0.0);
            hipLaunchKernelGGL(k_tensor_b, dim3(tiles(N), unsigned(nl), unsigned(nb)), dim3(256), 0, s, ap, bp,
                               D.u64(), nl, c->dprimes(), c->logN);
        }
        CKC_HIP(hipGetLastError());
        CKC_TRY(ks_modup_b(c, D.u64() + 2 * pw, 3 * pw, nb, level, digits.u64(), s));
        CKC_TRY(ks_apply_b(c, digits.u64(), nb, level, evk->relin->u64(), 1, &d0, &d1, false, o0, o1, s));
    }
    for (int i = 0; i < n; ++i) {
        out[i].level = level;
        out[i].npoly = 2;
        out[i].scale = a[i].scale * b[i].scale;
    }
    return CKC_OK;
}

extern "C" int ckc_mac_plain_many(ckc_ctx *c, const ckc_ct *in, const ckc_pt *pt, int n_terms, int n_out,
                                  ckc_ct *out, void *stream) {
    CKC_REQUIRE(c && in && pt && out && n_terms >= 1 && n_out >= 0, CKC_EINVAL, "null argument");
    CKC_REQUIRE(n_terms <= kMaxBatch, CKC_EINVAL, "mac_plain_many: more than 64 terms");
    if (n_out == 0) return CKC_OK;
    CKC_TRY(check_batch(c, in, n_out * n_terms, 2, "mac_plain_many"));
    const int level = in[0].level, nl = level + 1;
    for (int t = 0; t < n_terms; ++t) {
        CKC_REQUIRE(pt[t].d, CKC_EINVAL, "mac_plain_many: null plaintext");
        CKC_REQUIRE(pt[t].level >= level, CKC_ELEVEL, "mac_plain_many: plaintext level below the ciphertexts'");
        CKC_REQUIRE(std::fabs(pt[t].scale / pt[0].scale - 1.0) <= std::ldexp(1.0, -30), CKC_ESCALE,
                    "mac_plain_many: plaintext scales differ");
    }
    for (int o = 0; o < n_out; ++o) {
        CKC_REQUIRE(out[o].d, CKC_EINVAL, "mac_plain_many: null output");
        for (int i = 0; i < n_out * n_terms; ++i)
            CKC_REQUIRE(out[o].d != in[i].d, CKC_EINVAL, "mac_plain_many: output aliases an input");
    }
    hipStream_t s = S(stream);
    const size_t N = c->N;
    Ptrs pp{};
    for (int t = 0; t < n_terms; ++t) pp.p[t] = pt[t].d;
    const int per = kMaxBatch / n_terms;  // outputs per launch
    for (int o0 = 0; o0 < n_out; o0 += per) {
        const int no = std::min(per, n_out - o0);
        Ptrs ip{}, op{};
        for (int o = 0; o < no; ++o) {
            op.p[o] = out[o0 + o].d;
            for (int t = 0; t < n_terms; ++t) ip.p[o * n_terms + t] = in[size_t(o0 + o) * n_terms + t].d;
        }
        CKC_PROF(PK_MAC, s, 8.0 * N * nl * (2.0 * no * n_terms + n_terms + 2.0 * no), 2.0 * N * nl * no * n_terms);
        hipLaunchKernelGGL(k_mac_plain_b, dim3(unsigned(N / 256), unsigned(nl)), dim3(256), 0, s, ip, n_terms, pp,
                           op, no, nl, c->dprimes(), c->logN);
        CKC_HIP(hipGetLastError());
    }
    for (int o = 0; o < n_out; ++o) {
        out[o].level = level;
        out[o].npoly = 2;
        out[o].scale = in[size_t(o) * n_terms].scale * pt[0].scale;
    }
    return CKC_OK;
}
