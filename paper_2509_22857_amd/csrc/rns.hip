// RNS kernels shared by the C-ABI entry points: limb-wise arithmetic,
// permutations, tensor products, constants, the ModUp conversion tables and
// Galois tables, and rescale of a single ciphertext.  Key switching lives in
// batch.hip.
#include <math.h>

#include <algorithm>

#include "ckc_internal.h"
#include "prof.h"

namespace {

constexpr int kEwThreads = 256;

__global__ __launch_bounds__(kEwThreads) void k_ew(int op, uint64_t *__restrict__ out,
                                                   const uint64_t *__restrict__ a,
                                                   const uint64_t *__restrict__ b, int nlimbs,
                                                   size_t a_ps, size_t b_ps, size_t o_ps, LimbMap map,
                                                   const Prime *__restrict__ primes, int logN) {
    const int limb = blockIdx.y, poly = blockIdx.z;
    const Prime P = primes[map.prime(limb)];
    const size_t N = size_t(1) << logN;
    const uint64_t *al = a + poly * a_ps + size_t(limb) * N;
    const uint64_t *bl = b ? b + poly * b_ps + size_t(limb) * N : nullptr;
    uint64_t *ol = out + poly * o_ps + size_t(limb) * N;
    for (size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x; k < N; k += size_t(gridDim.x) * blockDim.x) {
        const uint64_t x = al[k];
        uint64_t r;
        switch (op) {
            case EW_ADD: r = add_mod(x, bl[k], P.q); break;
            case EW_SUB: r = sub_mod(x, bl[k], P.q); break;
            case EW_MUL: r = mul_mod(x, bl[k], P); break;
            case EW_NEG: r = neg_mod(x, P.q); break;
            default: r = x; break;
        }
        ol[k] = r;
    }
}

// Rescale: centred top limb t (coefficient form) -> t mod q_i for i < l.
__global__ __launch_bounds__(256) void k_rescale_lift(const uint64_t *__restrict__ top, int npoly,
                                                      size_t top_ps, uint64_t *__restrict__ dst, int level,
                                                      const Prime *__restrict__ primes, int logN) {
    const int i = blockIdx.y, p = blockIdx.z;
    const size_t N = size_t(1) << logN;
    const uint64_t ql = primes[level].q, half = ql >> 1;
    const Prime P = primes[i];
    const uint64_t qlm = reduce64(ql, P);
    const uint64_t *t = top + p * top_ps;
    uint64_t *o = dst + (size_t(p) * level + i) * N;
    for (size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x; k < N; k += size_t(gridDim.x) * blockDim.x) {
        const uint64_t v = t[k];
        const uint64_t vm = reduce64(v, P);
        o[k] = v > half ? sub_mod(vm, qlm, P.q) : vm;
    }
}

// out[p][i] = (in[p][i] - lift[p][i]) * q_l^-1 mod q_i
__global__ __launch_bounds__(256) void k_rescale_combine(const uint64_t *__restrict__ in, size_t in_ps,
                                                         const uint64_t *__restrict__ lift,
                                                         uint64_t *__restrict__ out, size_t out_ps, int level,
                                                         const uint64_t *__restrict__ rinv,
                                                         const Prime *__restrict__ primes, int logN, int nq) {
    const int i = blockIdx.y, p = blockIdx.z;
    const size_t N = size_t(1) << logN;
    const uint64_t q = primes[i].q;
    const uint64_t iv = rinv[(size_t(level) * nq + i) * 2], ivp = rinv[(size_t(level) * nq + i) * 2 + 1];
    const uint64_t *x = in + p * in_ps + size_t(i) * N;
    const uint64_t *t = lift + (size_t(p) * level + i) * N;
    uint64_t *o = out + p * out_ps + size_t(i) * N;
    for (size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x; k < N; k += size_t(gridDim.x) * blockDim.x)
        o[k] = mul_shoup(sub_mod(x[k], t[k], q), iv, ivp, q);
}

__global__ void k_copy_limbs(const uint64_t *__restrict__ src, size_t src_ps, uint64_t *__restrict__ dst,
                             size_t dst_ps, size_t words) {
    const int p = blockIdx.y;
    const uint64_t *s = src + p * src_ps;
    uint64_t *d = dst + p * dst_ps;
    for (size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x; k < words; k += size_t(gridDim.x) * blockDim.x)
        d[k] = s[k];
}

// out[t][k] = in[t][perm[k]]
__global__ void k_permute(const uint64_t *__restrict__ in, uint64_t *__restrict__ out,
                          const uint32_t *__restrict__ perm, int logN) {
    const int t = blockIdx.y;
    const size_t N = size_t(1) << logN;
    for (size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x; k < N; k += size_t(gridDim.x) * blockDim.x)
        out[size_t(t) * N + k] = in[size_t(t) * N + perm[k]];
}

// d0 = a0 b0, d1 = a0 b1 + a1 b0, d2 = a1 b1 (NTT form)
__global__ void k_tensor(const uint64_t *__restrict__ a, const uint64_t *__restrict__ b, uint64_t *__restrict__ o,
                         int nl, const Prime *__restrict__ primes, int logN) {
    const int t = blockIdx.y;
    const size_t N = size_t(1) << logN, ps = size_t(nl) * N;
    const Prime P = primes[t];
    for (size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x; k < N; k += size_t(gridDim.x) * blockDim.x) {
        const size_t i = size_t(t) * N + k;
        const uint64_t a0 = a[i], a1 = a[ps + i], b0 = b[i], b1 = b[ps + i];
        o[i] = mul_mod(a0, b0, P);
        o[ps + i] = reduce128(add128(mul64x64(a0, b1), mul64x64(a1, b0)), P);
        o[2 * ps + i] = mul_mod(a1, b1, P);
    }
}

// c0 += v (the same residue at every NTT point: a constant polynomial)
__global__ void k_add_const(const uint64_t *__restrict__ a, uint64_t *__restrict__ o,
                            const uint64_t *__restrict__ v, const Prime *__restrict__ primes, int logN) {
    const int t = blockIdx.y;
    const size_t N = size_t(1) << logN;
    const uint64_t q = primes[t].q, c = v[t];
    for (size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x; k < N; k += size_t(gridDim.x) * blockDim.x)
        o[size_t(t) * N + k] = add_mod(a[size_t(t) * N + k], c, q);
}

unsigned tiles_for(size_t N) { return unsigned(std::min<size_t>(N / 256, 64)); }

// host helpers ------------------------------------------------------------
uint64_t h_mulmod(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)(((unsigned __int128)a * b) % q); }
uint64_t h_powmod(uint64_t a, uint64_t e, uint64_t q) {
    uint64_t r = 1 % q;
    a %= q;
    while (e) {
        if (e & 1) r = h_mulmod(r, a, q);
        a = h_mulmod(a, a, q);
        e >>= 1;
    }
    return r;
}
uint64_t h_inv(uint64_t a, uint64_t q) { return h_powmod(a, q - 2, q); }
uint64_t h_shoup(uint64_t w, uint64_t q) { return (uint64_t)(((unsigned __int128)w << 64) / q); }

}  // namespace

int copy_limbs(const uint64_t *src, size_t src_ps, uint64_t *dst, size_t dst_ps, size_t words, int npoly,
               hipStream_t s) {
    if (words == 0 || npoly == 0) return CKC_OK;
    CKC_PROF(PK_COPY, s, 16.0 * double(words) * npoly, 0.0);
    hipLaunchKernelGGL(k_copy_limbs, dim3(unsigned(std::min<size_t>((words + 255) / 256, 2048)), unsigned(npoly)),
                       dim3(256), 0, s, src, src_ps, dst, dst_ps, words);
    CKC_HIP(hipGetLastError());
    return CKC_OK;
}

size_t words_ct(const ckc_ctx *c, int level, int npoly) { return size_t(npoly) * size_t(level + 1) * c->N; }

int ew_binary(const ckc_ctx *c, EwOp op, uint64_t *out, const uint64_t *a, const uint64_t *b, int npoly,
              int nlimbs, size_t a_ps, size_t b_ps, size_t o_ps, LimbMap map, hipStream_t s) {
    if (npoly <= 0 || nlimbs <= 0) return CKC_OK;
    hipLaunchKernelGGL(k_ew, dim3(tiles_for(c->N), unsigned(nlimbs), unsigned(npoly)), dim3(kEwThreads), 0, s,
                       int(op), out, a, b, nlimbs, a_ps, b_ps, o_ps, map, c->dprimes(), c->logN);
    CKC_HIP(hipGetLastError());
    return CKC_OK;
}

// Constants for ModUp of digit `digit` at `level`: source = the digit's
// primes, targets = every limb of the extended basis (l+1 Q limbs, then P).
const BconvTable *modup_table(ckc_ctx *c, int level, int digit, int *rc) {
    std::lock_guard<std::mutex> g(c->mu);
    auto key = std::make_pair(level, digit);
    auto it = c->modup_tabs.find(key);
    if (it != c->modup_tabs.end()) return it->second.get();
    auto t = std::make_unique<BconvTable>();
    const int lo = digit * c->alpha, hi = std::min(lo + c->alpha - 1, level);
    const int ns = hi - lo + 1, nt = level + 1 + c->np;
    std::vector<uint64_t> inv(ns), invp(ns), hat(size_t(nt) * ns);
    for (int i = 0; i < ns; ++i) {
        const uint64_t qi = c->mods[lo + i];
        uint64_t prod = 1 % qi;
        for (int j = 0; j < ns; ++j)
            if (j != i) prod = h_mulmod(prod, c->mods[lo + j] % qi, qi);
        inv[i] = h_inv(prod, qi);
        invp[i] = h_shoup(inv[i], qi);
    }
    LimbMap m{level + 1, c->nq};
    std::vector<uint64_t> neg_s(nt), s_half(ns);
    for (int i = 0; i < ns; ++i) s_half[i] = c->mods[lo + i] >> 1;
    for (int tt = 0; tt < nt; ++tt) {
        const uint64_t qt = c->mods[m.prime(tt)];
        const uint64_t r64 = uint64_t(((unsigned __int128)1 << 64) % qt);
        uint64_t S = 1 % qt;
        for (int i = 0; i < ns; ++i) {
            uint64_t prod = 1 % qt;
            for (int j = 0; j < ns; ++j)
                if (j != i) prod = h_mulmod(prod, c->mods[lo + j] % qt, qt);
            // times 2^64 mod q_t: the conversion ends in a Montgomery reduction
            hat[size_t(tt) * ns + i] = h_mulmod(prod, r64, qt);
            S = h_mulmod(S, c->mods[lo + i] % qt, qt);
        }
        neg_s[tt] = h_mulmod((qt - S) % qt, r64, qt);
    }
    t->ns = ns;
    t->nt = nt;
    t->iscale_h.resize(2 * size_t(ns));
    for (int i = 0; i < ns; ++i) {
        const uint64_t qi = c->mods[lo + i];
        t->iscale_h[2 * i] = h_mulmod(h_inv(c->N % qi, qi), inv[i], qi);
        t->iscale_h[2 * i + 1] = h_shoup(t->iscale_h[2 * i], qi);
    }
    if ((*rc = t->iscale.upload(t->iscale_h.data(), 8 * t->iscale_h.size())) != CKC_OK) return nullptr;
    if ((*rc = t->inv.upload(inv.data(), 8 * ns)) != CKC_OK) return nullptr;
    if ((*rc = t->invp.upload(invp.data(), 8 * ns)) != CKC_OK) return nullptr;
    if ((*rc = t->hat.upload(hat.data(), 8 * hat.size())) != CKC_OK) return nullptr;
    if ((*rc = t->neg_s.upload(neg_s.data(), 8 * neg_s.size())) != CKC_OK) return nullptr;
    if ((*rc = t->s_half.upload(s_half.data(), 8 * s_half.size())) != CKC_OK) return nullptr;
    const BconvTable *r = t.get();
    c->modup_tabs[key] = std::move(t);
    *rc = CKC_OK;
    return r;
}

const uint64_t *modup_scale(ckc_ctx *c, int level, int *rc) {
    {
        std::lock_guard<std::mutex> g(c->mu);
        auto it = c->modup_scale.find(level);
        if (it != c->modup_scale.end()) return it->second->u64();
    }
    std::vector<uint64_t> v;
    for (int j = 0; j < c->dnum_at(level); ++j) {
        const BconvTable *t = modup_table(c, level, j, rc);
        if (!t) return nullptr;
        v.insert(v.end(), t->iscale_h.begin(), t->iscale_h.end());
    }
    auto m = std::make_unique<DevMem>();
    if ((*rc = m->upload(v.data(), 8 * v.size())) != CKC_OK) return nullptr;
    std::lock_guard<std::mutex> g(c->mu);
    auto &slot = c->modup_scale[level];
    if (!slot) slot = std::move(m);
    *rc = CKC_OK;
    return slot->u64();
}

uint64_t galois_element(const ckc_ctx *c, int64_t step) {
    const int64_t n = int64_t(c->N / 2);
    const int64_t r = ((step % n) + n) % n;
    const uint64_t M = 2 * c->N;
    uint64_t g = 1;
    for (int64_t i = 0; i < r; ++i) g = (g * 5) % M;
    return g;
}

// g^-1 mod 2N: the odd residues mod 2N form a group of order N, so g^(N-1)
uint64_t galois_inverse(const ckc_ctx *c, uint64_t g) {
    const uint64_t M = 2 * c->N;
    uint64_t r = 1, b = g % M, e = c->N - 1;
    while (e) {
        if (e & 1) r = (r * b) % M;
        b = (b * b) % M;
        e >>= 1;
    }
    return r;
}

// NTT-domain permutation of sigma_g: index k holds a(psi^(2 brev(k) + 1)),
// so sigma_g(a) at k is a at the index whose exponent is g (2 brev(k) + 1).
const uint64_t *galois_table(ckc_ctx *c, uint64_t g, int *rc) {
    std::lock_guard<std::mutex> lk(c->mu);
    auto it = c->galois_perm.find(g);
    if (it != c->galois_perm.end()) return it->second->u64();
    const size_t N = c->N;
    const int logN = c->logN;
    auto brev = [logN](uint64_t x) {
        uint64_t r = 0;
        for (int i = 0; i < logN; ++i) r = (r << 1) | ((x >> i) & 1);
        return r;
    };
    std::vector<uint32_t> perm(N);
    const uint64_t mask = 2 * N - 1;
    for (size_t k = 0; k < N; ++k) {
        const uint64_t e = ((2 * brev(k) + 1) * g) & mask;
        perm[k] = uint32_t(brev((e - 1) / 2));
    }
    auto m = std::make_unique<DevMem>();
    if ((*rc = m->upload(perm.data(), 4 * N)) != CKC_OK) return nullptr;
    const uint64_t *r = m->u64();
    c->galois_perm[g] = std::move(m);
    *rc = CKC_OK;
    return r;
}

int rescale_impl(ckc_ctx *c, const uint64_t *in, int npoly, int level, uint64_t *out, hipStream_t s) {
    const size_t N = c->N;
    const int nl = level + 1;
    DevBuf top, lift;
    CKC_TRY(top.alloc(8 * N * npoly, s));
    CKC_TRY(lift.alloc(8 * N * npoly * level, s));
    CKC_TRY(copy_limbs(in + size_t(level) * N, size_t(nl) * N, top.u64(), N, N, npoly, s));
    const LimbMap one{0, level};  // every limb of `top` is prime q_level
    CKC_TRY(ntt_inverse(c, top.u64(), 1, one, npoly, N, s));
    hipLaunchKernelGGL(k_rescale_lift, dim3(tiles_for(N), unsigned(level), unsigned(npoly)), dim3(256), 0, s,
                       top.u64(), npoly, N, lift.u64(), level, c->dprimes(), c->logN);
    CKC_HIP(hipGetLastError());
    CKC_TRY(ntt_forward(c, lift.u64(), level, qmap(), npoly, size_t(level) * N, s));
    hipLaunchKernelGGL(k_rescale_combine, dim3(tiles_for(N), unsigned(level), unsigned(npoly)), dim3(256), 0, s,
                       in, size_t(nl) * N, lift.u64(), out, size_t(level) * N, level, c->rescale_inv.u64(),
                       c->dprimes(), c->logN, c->nq);
    CKC_HIP(hipGetLastError());
    return CKC_OK;
}

int permute_limbs(const ckc_ctx *c, const uint64_t *src, uint64_t *dst, int nlimbs, const uint32_t *perm,
                  hipStream_t s) {
    hipLaunchKernelGGL(k_permute, dim3(tiles_for(c->N), unsigned(nlimbs)), dim3(256), 0, s, src, dst, perm, c->logN);
    CKC_HIP(hipGetLastError());
    return CKC_OK;
}

int tensor_impl(ckc_ctx *c, const uint64_t *a, const uint64_t *b, uint64_t *out, int level, hipStream_t s) {
    hipLaunchKernelGGL(k_tensor, dim3(tiles_for(c->N), unsigned(level + 1)), dim3(256), 0, s, a, b, out, level + 1,
                       c->dprimes(), c->logN);
    CKC_HIP(hipGetLastError());
    return CKC_OK;
}

// exact residues of round(value * scale) (an integer-valued double) per Q prime
static uint64_t h_dint_mod(double v, uint64_t q) {
    const double av = fabs(v);
    uint64_t r;
    if (av < 9.2e18) {
        r = uint64_t(av) % q;
    } else {
        int e;
        const double mant = frexp(av, &e);
        const uint64_t M = uint64_t(ldexp(mant, 53));
        r = h_mulmod(M % q, h_powmod(2, uint64_t(e - 53), q), q);
    }
    return (v < 0 && r) ? q - r : r;
}

int add_const_impl(ckc_ctx *c, const ckc_ct *a, double value, ckc_ct *out, hipStream_t s) {
    const int nl = a->level + 1;
    const size_t ps = size_t(nl) * c->N;
    const double v = round(value * a->scale);
    std::vector<uint64_t> res(nl);
    for (int t = 0; t < nl; ++t) res[t] = h_dint_mod(v, c->mods[t]);
    DevBuf rb;
    CKC_TRY(rb.alloc(8 * nl, s));
    CKC_HIP(hipMemcpyAsync(rb.p, res.data(), 8 * nl, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_add_const, dim3(tiles_for(c->N), unsigned(nl)), dim3(256), 0, s, a->d, out->d, rb.u64(),
                       c->dprimes(), c->logN);
    CKC_HIP(hipGetLastError());
    if (out->d != a->d) CKC_TRY(copy_limbs(a->d + ps, 0, out->d + ps, 0, ps * (a->npoly - 1), 1, s));
    // the host residues must outlive the async copy
    CKC_HIP(hipStreamSynchronize(s));
    out->level = a->level;
    out->npoly = a->npoly;
    out->scale = a->scale;
    return CKC_OK;
}
