// C-ABI entry points: context set-up, keys, client operations and
// homomorphic arithmetic.  Argument checking happens here; the kernels live in
// ntt.hip, rns.hip and client.hip.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <set>

#include "batch.h"

static thread_local std::string g_err;
void ckc_set_error(const std::string &msg) { g_err = msg; }
extern "C" const char *ckc_last_error(void) { return g_err.c_str(); }

int copy_limbs(const uint64_t *src, size_t src_ps, uint64_t *dst, size_t dst_ps, size_t words, int npoly,
               hipStream_t s);
int encode_impl(ckc_ctx *c, const double *slots_h, size_t nslots, int level, double scale, uint64_t *m,
                hipStream_t s, bool ext = false);
int decode_impl(ckc_ctx *c, const uint64_t *m, double scale, double *out_h, size_t nslots, hipStream_t s);
int secret_impl(ckc_ctx *c, ckc_sk *sk, uint64_t seed, hipStream_t s);
int switch_key_impl(ckc_ctx *c, const ckc_sk *sk, uint64_t key_id, const uint64_t *sprime, uint64_t *key,
                    hipStream_t s);
int encrypt_impl(ckc_ctx *c, const ckc_sk *sk, const uint64_t *m, int level, uint64_t stream_id, uint64_t *ct,
                 hipStream_t s);
int decrypt_impl(ckc_ctx *c, const ckc_sk *sk, const uint64_t *ct, int level, int npoly, uint64_t *m,
                 hipStream_t s);
int permute_limbs(const ckc_ctx *c, const uint64_t *src, uint64_t *dst, int nlimbs, const uint32_t *perm,
                  hipStream_t s);
uint64_t galois_inverse(const ckc_ctx *c, uint64_t g);

namespace {

using u128 = unsigned __int128;
uint64_t hmul(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)(((u128)a * b) % q); }
uint64_t hpow(uint64_t a, uint64_t e, uint64_t q) {
    uint64_t r = 1 % q;
    a %= q;
    while (e) {
        if (e & 1) r = hmul(r, a, q);
        a = hmul(a, a, q);
        e >>= 1;
    }
    return r;
}
uint64_t hinv(uint64_t a, uint64_t q) { return hpow(a, q - 2, q); }
uint64_t hshoup(uint64_t w, uint64_t q) { return (uint64_t)(((u128)w << 64) / q); }

bool is_prime_u64(uint64_t n) {
    if (n < 2) return false;
    static const uint64_t bases[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    for (uint64_t p : bases)
        if (n % p == 0) return n == p;
    uint64_t d = n - 1;
    int r = 0;
    while ((d & 1) == 0) {
        d >>= 1;
        ++r;
    }
    for (uint64_t a : bases) {
        uint64_t x = hpow(a, d, n);
        if (x == 1 || x == n - 1) continue;
        bool comp = true;
        for (int i = 1; i < r; ++i) {
            x = hmul(x, x, n);
            if (x == n - 1) {
                comp = false;
                break;
            }
        }
        if (comp) return false;
    }
    return true;
}

Prime make_prime(uint64_t q) {
    Prime P{};
    P.q = q;
    int k = 64 - __builtin_clzll(q);
    P.k = k;
    P.mu = (uint64_t)(((u128)1 << (2 * k)) / q);
    P.r2 = (uint64_t)(((u128)1 << 64) % q);
    P.r2p = hshoup(P.r2, q);
    P.onep = (uint64_t)(((u128)1 << 64) / q);
    // q^-1 mod 2^64 by Newton's iteration (each step doubles the correct
    // low bits; q odd, so q is its own inverse mod 8)
    uint64_t inv = q;
    for (int i = 0; i < 5; ++i) inv *= 2 - q * inv;
    P.qinv = 0 - inv;
    return P;
}

uint64_t brev_bits(uint64_t x, int bits) {
    uint64_t r = 0;
    for (int i = 0; i < bits; ++i) r = (r << 1) | ((x >> i) & 1);
    return r;
}

// (cos, sin)(2 pi j / M), 0 <= j < M/2, M a power of two: folded into
// [0, pi/4] by octant symmetry, then 12-term Taylor series by Horner's rule,
// using IEEE +, -, *, / only, in one fixed order (the encoding's rounding
// depends on every bit of these tables, and libm's cos/sin differ across
// compilers in the last bit).
void series_cs(double x, double &c, double &s) {
    double cf[12], sf[12];
    double fc = 1.0, fs = 1.0;
    for (int i = 0; i < 12; ++i) {
        if (i > 0) {
            fc = fc / double((2 * i - 1) * (2 * i));
            fs = fs / double((2 * i) * (2 * i + 1));
        }
        cf[i] = (i & 1) ? -fc : fc;
        sf[i] = (i & 1) ? -fs : fs;
    }
    const double y = x * x;
    double pc = cf[11], ps = sf[11];
    for (int i = 10; i >= 0; --i) {
        pc = pc * y;
        pc = pc + cf[i];
        ps = ps * y;
        ps = ps + sf[i];
    }
    c = pc;
    s = x * ps;
}

void twiddle(uint64_t j, uint64_t M, double &c, double &s) {
    const double step = (2.0 * M_PI) / double(M);
    const uint64_t e8 = M / 8, e4 = M / 4, e38 = 3 * (M / 8), e2 = M / 2;
    double a, b;
    if (j <= e8) {
        series_cs(double(j) * step, a, b);
        c = a;
        s = b;
    } else if (j <= e4) {
        series_cs(double(e4 - j) * step, a, b);
        c = b;
        s = a;
    } else if (j <= e38) {
        series_cs(double(j - e4) * step, a, b);
        c = -b;
        s = a;
    } else {
        series_cs(double(e2 - j) * step, a, b);
        c = -a;
        s = b;
    }
}

hipStream_t S(void *s) { return (hipStream_t)s; }

int check_ct(const ckc_ctx *c, const ckc_ct *a, const char *what) {
    CKC_REQUIRE(a && a->d, CKC_EINVAL, std::string(what) + ": null ciphertext");
    CKC_REQUIRE(a->level >= 0 && a->level < c->nq, CKC_ELEVEL, std::string(what) + ": level out of range");
    CKC_REQUIRE(a->npoly >= 2 && a->npoly <= 3, CKC_ESHAPE, std::string(what) + ": npoly must be 2 or 3");
    return CKC_OK;
}
int check_scales(double a, double b) {
    CKC_REQUIRE(fabs(a / b - 1.0) <= ldexp(1.0, -30), CKC_ESCALE, "operand scales differ");
    return CKC_OK;
}

}  // namespace

// ======================================================================= ctx
extern "C" int ckc_ctx_create(int log_n, const uint64_t *q, int n_q, const uint64_t *p, int n_p, int alpha,
                              ckc_ctx **out) {
    CKC_REQUIRE(out && q && p, CKC_EINVAL, "null argument");
    CKC_REQUIRE(log_n >= 12 && log_n <= 16, CKC_EUNSUPPORTED, "log_n must be in [12, 16]");
    CKC_REQUIRE(n_q >= 1 && n_p >= 1 && n_q + n_p <= 96, CKC_EINVAL, "bad prime counts");
    CKC_REQUIRE(alpha >= 1 && alpha <= n_q, CKC_EINVAL, "bad alpha");
    CKC_REQUIRE(alpha <= kMaxBconv && n_p <= kMaxBconv, CKC_EUNSUPPORTED,
                "at most 8 primes per key-switching digit and 8 special primes");
    const size_t N = size_t(1) << log_n;
    std::set<uint64_t> seen;
    for (int i = 0; i < n_q + n_p; ++i) {
        const uint64_t m = i < n_q ? q[i] : p[i - n_q];
        CKC_REQUIRE(m < (uint64_t(1) << 62) && m > (1u << 20), CKC_EUNSUPPORTED, "moduli must lie in (2^20, 2^62)");
        CKC_REQUIRE((m - 1) % (2 * N) == 0, CKC_EINVAL, "modulus not 1 mod 2N");
        CKC_REQUIRE(is_prime_u64(m), CKC_EINVAL, "modulus not prime");
        CKC_REQUIRE(seen.insert(m).second, CKC_EINVAL, "duplicate modulus");
    }
    // sums of up to dnum + 1 (key inner product, with the P c0 term of the
    // extended form) or alpha / n_p (basis conversion) products of residues
    // are accumulated in 128 bits without reduction; their Montgomery
    // reduction reduces the high word before adding mulhi(m, q), so it holds
    // for every count within the accumulator's cap, up to q < 2^62
    {
        uint64_t qmax = 0;
        for (int i = 0; i < n_q; ++i) qmax = std::max(qmax, q[i]);
        for (int i = 0; i < n_p; ++i) qmax = std::max(qmax, p[i]);
        const int dnum = (n_q + alpha - 1) / alpha;
        const long double bound =
            (long double)qmax * (long double)qmax * (long double)std::max(dnum + 1, std::max(alpha, n_p));
        CKC_REQUIRE(bound < 0x1p127L * 2.0L, CKC_EUNSUPPORTED, "moduli too large for 128-bit accumulation of the digits");
        CKC_REQUIRE(dnum <= 16, CKC_EUNSUPPORTED, "at most 16 key-switching digits");
        const int kmax = 64 - __builtin_clzll(qmax);
        CKC_REQUIRE(std::max(dnum + 1, std::max(alpha, n_p)) <= prod_cap(kmax), CKC_EUNSUPPORTED,
                    "too many digits for the carry-free accumulator at this modulus size");
    }
    auto c = std::make_unique<ckc_ctx>();
    c->logN = log_n;
    c->N = N;
    c->nq = n_q;
    c->np = n_p;
    c->alpha = alpha;
    for (int i = 0; i < n_q; ++i) c->mods.push_back(q[i]);
    for (int i = 0; i < n_p; ++i) c->mods.push_back(p[i]);
    const int np = c->nprimes();
    for (int t = 0; t < np; ++t) c->primes_h.push_back(make_prime(c->mods[t]));
    CKC_TRY(c->primes_d.upload(c->primes_h.data(), sizeof(Prime) * np));

    // NTT tables
    std::vector<uint64_t> tw(N * np), twp(N * np), itw(N * np), itwp(N * np), ninv(2 * np);
    for (int t = 0; t < np; ++t) {
        const uint64_t m = c->mods[t];
        uint64_t psi = 0;
        for (uint64_t x = 2;; ++x) {
            const uint64_t g = hpow(x, (m - 1) / (2 * N), m);
            if (hpow(g, N, m) == m - 1) {
                psi = g;
                break;
            }
        }
        c->psi_h.push_back(psi);
        const uint64_t ipsi = hinv(psi, m);
        std::vector<uint64_t> pw(N), ipw(N);
        uint64_t x = 1, y = 1;
        for (size_t i = 0; i < N; ++i) {
            pw[i] = x;
            ipw[i] = y;
            x = hmul(x, psi, m);
            y = hmul(y, ipsi, m);
        }
        for (size_t k = 0; k < N; ++k) {
            const uint64_t r = brev_bits(k, log_n);
            tw[t * N + k] = pw[r];
            twp[t * N + k] = hshoup(pw[r], m);
            itw[t * N + k] = ipw[r];
            itwp[t * N + k] = hshoup(ipw[r], m);
        }
        ninv[2 * t] = hinv(N % m, m);
        ninv[2 * t + 1] = hshoup(ninv[2 * t], m);
    }
    CKC_TRY(c->tw.upload(tw.data(), 8 * tw.size()));
    CKC_TRY(c->twp.upload(twp.data(), 8 * twp.size()));
    CKC_TRY(c->itw.upload(itw.data(), 8 * itw.size()));
    CKC_TRY(c->itwp.upload(itwp.data(), 8 * itwp.size()));
    CKC_TRY(c->ninv.upload(ninv.data(), 8 * ninv.size()));

    // FFT tables: twiddles of the length-n DFT and the zeta^k twist
    const size_t n = N / 2;
    std::vector<double> fw(2 * (n / 2)), tws(2 * n);
    for (size_t e = 0; e < n / 2; ++e) twiddle(e, n, fw[2 * e], fw[2 * e + 1]);
    for (size_t k = 0; k < n; ++k) twiddle(k, 2 * N, tws[2 * k], tws[2 * k + 1]);
    std::vector<uint32_t> sidx(n);
    uint64_t g = 1;
    for (size_t j = 0; j < n; ++j) {
        sidx[j] = uint32_t((g - 1) / 4);
        g = (g * 5) % (2 * N);
    }
    CKC_TRY(c->fft_w.upload(fw.data(), 8 * fw.size()));
    CKC_TRY(c->twist.upload(tws.data(), 8 * tws.size()));
    CKC_TRY(c->slot_idx.upload(sidx.data(), 4 * sidx.size()));

    // rescale constants q_l^-1 mod q_i
    std::vector<uint64_t> rinv(size_t(n_q) * n_q * 2, 0);
    for (int l = 1; l < n_q; ++l)
        for (int i = 0; i < l; ++i) {
            const uint64_t qi = c->mods[i];
            const uint64_t v = hinv(c->mods[l] % qi, qi);
            rinv[(size_t(l) * n_q + i) * 2] = v;
            rinv[(size_t(l) * n_q + i) * 2 + 1] = hshoup(v, qi);
        }
    CKC_TRY(c->rescale_inv.upload(rinv.data(), 8 * rinv.size()));

    // ModDown: P^-1 mod q_i, and P -> q_i conversion constants
    std::vector<uint64_t> pinv(2 * n_q), pmod(2 * n_q), inv(n_p), invp(n_p), hat(size_t(n_q) * n_p);
    for (int i = 0; i < n_q; ++i) {
        const uint64_t qi = c->mods[i];
        uint64_t P = 1 % qi;
        for (int k = 0; k < n_p; ++k) P = hmul(P, p[k] % qi, qi);
        pinv[2 * i] = hinv(P, qi);
        pinv[2 * i + 1] = hshoup(pinv[2 * i], qi);
        pmod[2 * i] = P;
        pmod[2 * i + 1] = hshoup(P, qi);
        for (int a = 0; a < n_p; ++a) {
            uint64_t h = 1 % qi;
            for (int b = 0; b < n_p; ++b)
                if (b != a) h = hmul(h, p[b] % qi, qi);
            hat[size_t(i) * n_p + a] = hmul(h, (uint64_t)(((u128)1 << 64) % qi), qi);  // times 2^64 mod q_i
        }
    }
    c->p_to_q.iscale_h.resize(2 * size_t(n_p));
    for (int a = 0; a < n_p; ++a) {
        const uint64_t pa = p[a];
        uint64_t h = 1 % pa;
        for (int b = 0; b < n_p; ++b)
            if (b != a) h = hmul(h, p[b] % pa, pa);
        inv[a] = hinv(h, pa);
        invp[a] = hshoup(inv[a], pa);
        c->p_to_q.iscale_h[2 * a] = hmul(hinv(N % pa, pa), inv[a], pa);
        c->p_to_q.iscale_h[2 * a + 1] = hshoup(c->p_to_q.iscale_h[2 * a], pa);
    }
    CKC_TRY(c->p_to_q.iscale.upload(c->p_to_q.iscale_h.data(), 8 * c->p_to_q.iscale_h.size()));
    CKC_TRY(c->pinv.upload(pinv.data(), 8 * pinv.size()));
    CKC_TRY(c->pmod.upload(pmod.data(), 8 * pmod.size()));
    c->p_to_q.ns = n_p;
    c->p_to_q.nt = n_q;
    CKC_TRY(c->p_to_q.inv.upload(inv.data(), 8 * n_p));
    CKC_TRY(c->p_to_q.invp.upload(invp.data(), 8 * n_p));
    CKC_TRY(c->p_to_q.hat.upload(hat.data(), 8 * hat.size()));
    // centring of the P -> Q conversion: (-P) 2^64 mod q_i, and p_k >> 1
    std::vector<uint64_t> neg_p(n_q), p_half(n_p);
    for (int i = 0; i < n_q; ++i) {
        const uint64_t qi = c->mods[i];
        neg_p[i] = hmul((qi - pmod[2 * i]) % qi, (uint64_t)(((u128)1 << 64) % qi), qi);
    }
    for (int a = 0; a < n_p; ++a) p_half[a] = p[a] >> 1;
    CKC_TRY(c->p_to_q.neg_s.upload(neg_p.data(), 8 * neg_p.size()));
    CKC_TRY(c->p_to_q.s_half.upload(p_half.data(), 8 * p_half.size()));
    // ModUp tables of every level, so that no key switch builds one later
    for (int l = 0; l < n_q; ++l) {
        int rc = CKC_OK;
        if (!modup_scale(c.get(), l, &rc)) return rc;
    }
    *out = c.release();
    return CKC_OK;
}

extern "C" int ckc_ctx_destroy(ckc_ctx *c) {
    delete c;
    arena_trim();
    return CKC_OK;
}
extern "C" size_t ckc_ct_words(const ckc_ctx *c, int level, int npoly) { return words_ct(c, level, npoly); }
extern "C" size_t ckc_pt_words(const ckc_ctx *c, int level) { return size_t(level + 1) * c->N; }
extern "C" size_t ckc_ct_bytes(const ckc_ctx *c, int level, int npoly) { return 8 * words_ct(c, level, npoly); }

namespace {
std::atomic<int> g_fault_after{0}, g_fault_code{0};
}
int test_fault_take() {
    if (g_fault_after.load(std::memory_order_relaxed) <= 0) return 0;
    if (g_fault_after.fetch_sub(1) != 1) return 0;
    return g_fault_code.load();
}
extern "C" int ckc_set_test_fault(int call_index, int code) {
    CKC_REQUIRE(call_index >= 0 && (call_index == 0 || code < 0), CKC_EINVAL, "fault needs a negative error code");
    g_fault_code.store(code);
    g_fault_after.store(call_index);
    return CKC_OK;
}
extern "C" uint64_t ckc_ctx_root(const ckc_ctx *c, int t) {
    return (t >= 0 && t < c->nprimes()) ? c->psi_h[t] : 0;
}

extern "C" int ckc_ntt(const ckc_ctx *c, uint64_t *d, int n_blocks, int n_limbs, int inverse, void *stream) {
    CKC_REQUIRE(c && d, CKC_EINVAL, "null argument");
    CKC_REQUIRE(n_limbs >= 1 && n_limbs <= c->nq && n_blocks >= 0, CKC_EINVAL, "bad limb count");
    const size_t stride = size_t(n_limbs) * c->N;
    // grid.z is limited to 65535 blocks per launch
    for (int b0 = 0; b0 < n_blocks; b0 += 65535) {
        const int nb = std::min(65535, n_blocks - b0);
        uint64_t *p = d + size_t(b0) * stride;
        if (inverse)
            CKC_TRY(ntt_inverse(c, p, n_limbs, qmap(), nb, stride, S(stream)));
        else
            CKC_TRY(ntt_forward(c, p, n_limbs, qmap(), nb, stride, S(stream)));
    }
    return CKC_OK;
}

// ======================================================================= keys
static int add_galois(ckc_ctx *c, const ckc_sk *sk, ckc_evk *evk, const int32_t *steps, int n, hipStream_t s) {
    const size_t N = c->N;
    const int np = c->nprimes();
    for (int i = 0; i < n; ++i) {
        const uint64_t g = galois_element(c, steps[i]);
        if (g == 1 || evk->galois.count(g)) continue;
        int rc;
        const uint32_t *perm = (const uint32_t *)galois_table(c, g, &rc);
        if (!perm) return rc;
        DevBuf sp;
        CKC_TRY(sp.alloc(8 * N * np, s));
        // sigma_g(s) in the NTT domain: a gather through the permutation, every prime
        CKC_TRY(permute_limbs(c, sk->s_ntt.u64(), sp.u64(), np, perm, s));
        // generate, then store permuted by sigma_g^-1 (the key inner product
        // reads digits in order and scatters its outputs through pi_g^-1)
        DevBuf raw;
        CKC_TRY(raw.alloc(8 * evk->key_words, s));
        CKC_TRY(switch_key_impl(c, sk, g, sp.u64(), raw.u64(), s));
        const uint32_t *iperm = (const uint32_t *)galois_table(c, galois_inverse(c, g), &rc);
        if (!iperm) return rc;
        auto key = std::make_unique<DevMem>();
        CKC_TRY(key->alloc(8 * evk->key_words));
        CKC_TRY(permute_limbs(c, raw.u64(), key->u64(), int(evk->key_words / N), iperm, s));
        CKC_HIP(hipStreamSynchronize(s));
        evk->galois[g] = std::move(key);
    }
    return CKC_OK;
}

extern "C" int ckc_keygen(ckc_ctx *c, uint64_t seed, const int32_t *steps, int n_steps, ckc_sk **sk_out,
                          ckc_evk **evk_out, void *stream) {
    CKC_REQUIRE(c && sk_out && evk_out, CKC_EINVAL, "null argument");
    CKC_REQUIRE(n_steps >= 0 && (n_steps == 0 || steps), CKC_EINVAL, "bad steps");
    hipStream_t s = S(stream);
    auto sk = std::make_unique<ckc_sk>();
    CKC_TRY(secret_impl(c, sk.get(), seed, s));
    auto evk = std::make_unique<ckc_evk>();
    const size_t N = c->N;
    const int np = c->nprimes();
    evk->dnum = c->dnum_at(c->nq - 1);
    evk->key_words = size_t(evk->dnum) * 2 * np * N;
    // relinearisation key: s' = s^2 (pointwise in the NTT domain)
    DevBuf s2;
    CKC_TRY(s2.alloc(8 * N * np, s));
    CKC_TRY(ew_binary(c, EW_MUL, s2.u64(), sk->s_ntt.u64(), sk->s_ntt.u64(), 1, np, 0, 0, 0, qmap(), s));
    evk->relin = std::make_unique<DevMem>();
    CKC_TRY(evk->relin->alloc(8 * evk->key_words));
    CKC_TRY(switch_key_impl(c, sk.get(), 0, s2.u64(), evk->relin->u64(), s));
    CKC_TRY(add_galois(c, sk.get(), evk.get(), steps, n_steps, s));
    CKC_HIP(hipStreamSynchronize(s));
    *sk_out = sk.release();
    *evk_out = evk.release();
    return CKC_OK;
}

extern "C" int ckc_evk_add_rotations(ckc_ctx *c, const ckc_sk *sk, ckc_evk *evk, const int32_t *steps, int n_steps,
                                     void *stream) {
    CKC_REQUIRE(c && sk && evk, CKC_EINVAL, "null argument");
    CKC_TRY(add_galois(c, sk, evk, steps, n_steps, S(stream)));
    CKC_HIP(hipStreamSynchronize(S(stream)));
    return CKC_OK;
}

extern "C" int ckc_sk_destroy(ckc_sk *sk) {
    delete sk;
    return CKC_OK;
}
extern "C" int ckc_evk_destroy(ckc_evk *e) {
    delete e;
    return CKC_OK;
}
extern "C" size_t ckc_evk_bytes(const ckc_evk *e) {
    if (!e) return 0;
    size_t n = e->galois.size() + (e->relin ? 1 : 0);
    return n * e->key_words * 8;
}

extern "C" int ckc_evk_group_create(const ckc_evk *const *keys, int n_keys, const int32_t *key_of_img, int n_img,
                                    ckc_evk **group) {
    CKC_REQUIRE(keys && key_of_img && group && n_keys >= 1 && n_img >= 1, CKC_EINVAL, "null or empty argument");
    auto g = std::make_unique<ckc_evk>();
    for (int k = 0; k < n_keys; ++k) {
        CKC_REQUIRE(keys[k] && !keys[k]->is_group(), CKC_EINVAL, "a key group's members are key sets");
        CKC_REQUIRE(keys[k]->dnum == keys[0]->dnum && keys[k]->key_words == keys[0]->key_words, CKC_EINVAL,
                    "key sets of one group come from one context");
        g->members.push_back(keys[k]);
    }
    for (int i = 0; i < n_img; ++i) {
        CKC_REQUIRE(key_of_img[i] >= 0 && key_of_img[i] < n_keys, CKC_EINVAL, "key index out of range");
        g->key_of_img.push_back(key_of_img[i]);
    }
    g->dnum = keys[0]->dnum;
    g->key_words = keys[0]->key_words;
    *group = g.release();
    return CKC_OK;
}

int check_evk_images(const ckc_evk *e, int n_img, const char *what) {
    CKC_REQUIRE(!e->is_group() || int(e->key_of_img.size()) == n_img, CKC_EINVAL,
                std::string(what) + ": the key group covers " + std::to_string(e->key_of_img.size()) +
                    " images, the call " + std::to_string(n_img));
    return CKC_OK;
}

// ======================================================================= client
extern "C" int ckc_encode(ckc_ctx *c, const double *slots, size_t n, int level, double scale, ckc_pt *out,
                          void *stream) {
    CKC_REQUIRE(c && out && out->d && (n == 0 || slots), CKC_EINVAL, "null argument");
    CKC_REQUIRE(n <= c->N / 2, CKC_EINVAL, "too many slots");
    CKC_REQUIRE(level >= 0 && level < c->nq, CKC_ELEVEL, "level out of range");
    CKC_REQUIRE(scale > 0 && isfinite(scale), CKC_EINVAL, "bad scale");
    CKC_TRY(encode_impl(c, slots, n, level, scale, out->d, S(stream)));
    out->level = level;
    out->scale = scale;
    return CKC_OK;
}

extern "C" int ckc_encrypt(ckc_ctx *c, const ckc_sk *sk, const ckc_pt *pt, uint64_t stream_id, ckc_ct *out,
                           void *stream) {
    CKC_REQUIRE(c && sk && pt && pt->d && out && out->d, CKC_EINVAL, "null argument");
    CKC_REQUIRE(pt->level >= 0 && pt->level < c->nq, CKC_ELEVEL, "level out of range");
    CKC_TRY(encrypt_impl(c, sk, pt->d, pt->level, stream_id, out->d, S(stream)));
    out->level = pt->level;
    out->npoly = 2;
    out->scale = pt->scale;
    return CKC_OK;
}

extern "C" int ckc_encode_encrypt_image(ckc_ctx *c, const ckc_sk *sk, const double *chw, int C, int H, int W,
                                        int members, int block, int row_stride, int level, double scale,
                                        uint64_t stream_id, ckc_ct *out, void *stream) {
    CKC_REQUIRE(c && sk && chw && out, CKC_EINVAL, "null argument");
    CKC_REQUIRE(C > 0 && H > 0 && W > 0 && members > 0 && block > 0 && row_stride >= W, CKC_EINVAL, "bad image shape");
    CKC_REQUIRE(size_t(H - 1) * row_stride + W <= size_t(block) && size_t(members) * block <= c->N / 2, CKC_EINVAL,
                "image does not fit the slot layout");
    CKC_REQUIRE(level >= 0 && level < c->nq, CKC_ELEVEL, "level out of range");
    CKC_REQUIRE(scale > 0 && isfinite(scale), CKC_EINVAL, "bad scale");
    for (int ch = 0; ch < C; ++ch) CKC_REQUIRE(out[ch].d, CKC_EINVAL, "null output buffer");
    const hipStream_t s = S(stream);
    DevBuf m;
    CKC_TRY(m.alloc(8 * size_t(level + 1) * c->N, s));
    std::vector<double> v(size_t(members) * block);
    for (int ch = 0; ch < C; ++ch) {
        // member mm's copy of channel ch: pixel (r, x) at slot mm block + r row_stride + x
        std::fill(v.begin(), v.end(), 0.0);
        for (int mm = 0; mm < members; ++mm)
            for (int r = 0; r < H; ++r)
                std::copy(chw + (size_t(ch) * H + r) * W, chw + (size_t(ch) * H + r) * W + W,
                          v.begin() + size_t(mm) * block + size_t(r) * row_stride);
        CKC_TRY(encode_impl(c, v.data(), v.size(), level, scale, m.u64(), s, false));
        CKC_TRY(encrypt_impl(c, sk, m.u64(), level, stream_id + uint64_t(ch), out[ch].d, s));
        out[ch].level = level;
        out[ch].npoly = 2;
        out[ch].scale = scale;
    }
    return CKC_OK;
}

extern "C" int ckc_decrypt(ckc_ctx *c, const ckc_sk *sk, const ckc_ct *ct, ckc_pt *out, void *stream) {
    CKC_REQUIRE(c && sk && out && out->d, CKC_EINVAL, "null argument");
    CKC_TRY(check_ct(c, ct, "decrypt"));
    CKC_TRY(decrypt_impl(c, sk, ct->d, ct->level, ct->npoly, out->d, S(stream)));
    out->level = ct->level;
    out->scale = ct->scale;
    return CKC_OK;
}

extern "C" int ckc_decode(ckc_ctx *c, const ckc_pt *pt, double *slots, size_t n, void *stream) {
    CKC_REQUIRE(c && pt && pt->d && (n == 0 || slots), CKC_EINVAL, "null argument");
    CKC_REQUIRE(n <= c->N / 2, CKC_EINVAL, "too many slots");
    return decode_impl(c, pt->d, pt->scale, slots, n, S(stream));
}

// ======================================================================= arithmetic
static int addsub(ckc_ctx *c, const ckc_ct *a, const ckc_ct *b, ckc_ct *out, EwOp op, void *stream) {
    CKC_TRY(check_ct(c, a, "add"));
    CKC_TRY(check_ct(c, b, "add"));
    CKC_REQUIRE(out && out->d, CKC_EINVAL, "null output");
    CKC_REQUIRE(a->level == b->level, CKC_ELEVEL, "levels differ");
    CKC_TRY(check_scales(a->scale, b->scale));
    const size_t N = c->N, ps = size_t(a->level + 1) * N;
    const int nl = a->level + 1, common = std::min(a->npoly, b->npoly);
    hipStream_t s = S(stream);
    CKC_TRY(ew_binary(c, op, out->d, a->d, b->d, common, nl, ps, ps, ps, qmap(), s));
    if (a->npoly > common)
        CKC_TRY(copy_limbs(a->d + common * ps, 0, out->d + common * ps, 0, ps, 1, s));
    if (b->npoly > common) {
        if (op == EW_ADD)
            CKC_TRY(copy_limbs(b->d + common * ps, 0, out->d + common * ps, 0, ps, 1, s));
        else
            CKC_TRY(ew_binary(c, EW_NEG, out->d + common * ps, b->d + common * ps, nullptr, 1, nl, 0, 0, 0, qmap(), s));
    }
    out->level = a->level;
    out->npoly = std::max(a->npoly, b->npoly);
    out->scale = a->scale;
    return CKC_OK;
}

extern "C" int ckc_add(ckc_ctx *c, const ckc_ct *a, const ckc_ct *b, ckc_ct *out, void *stream) {
    return addsub(c, a, b, out, EW_ADD, stream);
}
extern "C" int ckc_sub(ckc_ctx *c, const ckc_ct *a, const ckc_ct *b, ckc_ct *out, void *stream) {
    return addsub(c, a, b, out, EW_SUB, stream);
}

extern "C" int ckc_add_plain(ckc_ctx *c, const ckc_ct *a, const ckc_pt *p, ckc_ct *out, void *stream) {
    CKC_TRY(check_ct(c, a, "add_plain"));
    CKC_REQUIRE(p && p->d && out && out->d, CKC_EINVAL, "null argument");
    CKC_REQUIRE(p->level >= a->level, CKC_ELEVEL, "plaintext level too low");
    CKC_TRY(check_scales(a->scale, p->scale));
    const size_t ps = size_t(a->level + 1) * c->N;
    hipStream_t s = S(stream);
    CKC_TRY(ew_binary(c, EW_ADD, out->d, a->d, p->d, 1, a->level + 1, 0, 0, 0, qmap(), s));
    if (out->d != a->d) CKC_TRY(copy_limbs(a->d + ps, 0, out->d + ps, 0, ps * (a->npoly - 1), 1, s));
    out->level = a->level;
    out->npoly = a->npoly;
    out->scale = a->scale;
    return CKC_OK;
}

int add_const_impl(ckc_ctx *c, const ckc_ct *a, double value, ckc_ct *out, hipStream_t s);

extern "C" int ckc_add_const(ckc_ctx *c, const ckc_ct *a, double value, ckc_ct *out, void *stream) {
    CKC_TRY(check_ct(c, a, "add_const"));
    CKC_REQUIRE(out && out->d, CKC_EINVAL, "null output");
    CKC_REQUIRE(isfinite(value), CKC_EINVAL, "non-finite constant");
    return add_const_impl(c, a, value, out, S(stream));
}

extern "C" int ckc_mul_plain(ckc_ctx *c, const ckc_ct *a, const ckc_pt *p, ckc_ct *out, void *stream) {
    CKC_TRY(check_ct(c, a, "mul_plain"));
    CKC_REQUIRE(p && p->d && out && out->d, CKC_EINVAL, "null argument");
    CKC_REQUIRE(p->level >= a->level, CKC_ELEVEL, "plaintext level too low");
    const size_t ps = size_t(a->level + 1) * c->N;
    CKC_TRY(ew_binary(c, EW_MUL, out->d, a->d, p->d, a->npoly, a->level + 1, ps, 0, ps, qmap(), S(stream)));
    out->level = a->level;
    out->npoly = a->npoly;
    out->scale = a->scale * p->scale;
    return CKC_OK;
}

int tensor_impl(ckc_ctx *c, const uint64_t *a, const uint64_t *b, uint64_t *out, int level, hipStream_t s);

extern "C" int ckc_tensor(ckc_ctx *c, const ckc_ct *a, const ckc_ct *b, ckc_ct *out, void *stream) {
    CKC_TRY(check_ct(c, a, "tensor"));
    CKC_TRY(check_ct(c, b, "tensor"));
    CKC_REQUIRE(out && out->d && out->d != a->d && out->d != b->d, CKC_EINVAL, "output must not alias");
    CKC_REQUIRE(a->npoly == 2 && b->npoly == 2, CKC_ESHAPE, "tensor needs 2-poly inputs");
    CKC_REQUIRE(a->level == b->level, CKC_ELEVEL, "levels differ");
    CKC_TRY(tensor_impl(c, a->d, b->d, out->d, a->level, S(stream)));
    out->level = a->level;
    out->npoly = 3;
    out->scale = a->scale * b->scale;
    return CKC_OK;
}

int relin_impl(ckc_ctx *c, const ckc_evk *evk, const ckc_ct *in, ckc_ct *out, void *stream) {
    CKC_REQUIRE(!evk || !evk->is_group(), CKC_EINVAL, "relin: a key group serves layer calls only");
    CKC_TRY(check_ct(c, in, "relin"));
    CKC_REQUIRE(evk && out && out->d, CKC_EINVAL, "null argument");
    CKC_REQUIRE(in->npoly == 3, CKC_ESHAPE, "relin needs a 3-poly ciphertext");
    CKC_REQUIRE(evk->relin, CKC_ENOKEY, "no relinearisation key");
    hipStream_t s = S(stream);
    const size_t N = c->N;
    const int nl = in->level + 1, nt = nl + c->np;
    DevBuf digits;
    CKC_TRY(digits.alloc(8 * N * nt * size_t(c->dnum_at(in->level)), s));
    const size_t ps = size_t(nl) * N;
    CKC_TRY(ks_modup_b(c, in->d + 2 * ps, 0, 1, in->level, digits.u64(), s));
    Ptrs a0{}, a1{}, o0{}, o1{};
    a0.p[0] = in->d;
    a1.p[0] = in->d + ps;
    o0.p[0] = out->d;
    o1.p[0] = out->d + ps;
    CKC_TRY(ks_apply_b(c, digits.u64(), 1, in->level, evk->relin->u64(), 1, &a0, &a1, false, o0, o1, s));
    out->level = in->level;
    out->npoly = 2;
    out->scale = in->scale;
    return CKC_OK;
}

extern "C" int ckc_relin(ckc_ctx *c, const ckc_evk *evk, const ckc_ct *in, ckc_ct *out, void *stream) {
    return relin_impl(c, evk, in, out, stream);
}

size_t relin_scratch_bytes(const ckc_ctx *c, int level) {
    // digits [dnum][l+1+n_P][N], held throughout; then ModUp's coefficient
    // copy [l+1][N] (released before) the key inner product's outputs
    // [2][l+1] + [2][n_P] and ModDown's conversion [2][l+1] limbs
    const size_t limb = 8 * c->N;
    auto up = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t nl = size_t(level) + 1, nt = nl + c->np;
    const size_t digits = up(limb * nt * size_t(c->dnum_at(level)));
    const size_t modup = up(limb * nl);
    const size_t apply = up(limb * nl * 2) + up(limb * c->np * 2) + up(limb * nl * 2);
    return digits + std::max(modup, apply);
}

extern "C" int ckc_rotate(ckc_ctx *c, const ckc_evk *evk, const ckc_ct *in, const int32_t *steps, int n_steps,
                          ckc_ct *out, void *stream) {
    CKC_REQUIRE(!evk || !evk->is_group(), CKC_EINVAL, "rotate: a key group serves layer calls only");
    CKC_TRY(check_ct(c, in, "rotate"));
    CKC_REQUIRE(evk && out && (n_steps == 0 || steps), CKC_EINVAL, "null argument");
    CKC_REQUIRE(in->npoly == 2, CKC_ESHAPE, "rotation needs a 2-poly ciphertext");
    hipStream_t s = S(stream);
    const size_t N = c->N;
    const int nl = in->level + 1, nt = nl + c->np;
    const size_t ps = size_t(nl) * N;
    bool need_ks = false;
    for (int i = 0; i < n_steps; ++i) {
        CKC_REQUIRE(out[i].d && out[i].d != in->d, CKC_EINVAL, "rotation output missing or aliasing the input");
        const uint64_t g = galois_element(c, steps[i]);
        if (g != 1) {
            need_ks = true;
            CKC_REQUIRE(evk->galois.count(g), CKC_ENOKEY, "missing Galois key for step " + std::to_string(steps[i]));
        }
    }
    DevBuf digits;
    if (need_ks) {
        CKC_TRY(digits.alloc(8 * N * nt * size_t(c->dnum_at(in->level)), s));
        CKC_TRY(ks_modup_b(c, in->d + ps, 0, 1, in->level, digits.u64(), s));
    }
    for (int i = 0; i < n_steps; ++i) {
        const uint64_t g = galois_element(c, steps[i]);
        if (g == 1) {
            CKC_TRY(copy_limbs(in->d, 0, out[i].d, 0, 2 * ps, 1, s));
        } else {
            Ptrs a0{}, o0{}, o1{};
            a0.p[0] = in->d;
            o0.p[0] = out[i].d;
            o1.p[0] = out[i].d + ps;
            CKC_TRY(ks_apply_b(c, digits.u64(), 1, in->level, evk->galois.at(g)->u64(), g, &a0, nullptr, true, o0, o1, s));
        }
        out[i].level = in->level;
        out[i].npoly = 2;
        out[i].scale = in->scale;
    }
    return CKC_OK;
}

extern "C" int ckc_rescale(ckc_ctx *c, const ckc_ct *in, ckc_ct *out, void *stream) {
    CKC_TRY(check_ct(c, in, "rescale"));
    CKC_REQUIRE(in->level >= 1, CKC_ELEVEL, "cannot rescale at level 0");
    CKC_REQUIRE(out && out->d && out->d != in->d, CKC_EINVAL, "output missing or aliasing the input");
    CKC_TRY(rescale_impl(c, in->d, in->npoly, in->level, out->d, S(stream)));
    out->scale = in->scale / double(c->mods[in->level]);
    out->level = in->level - 1;
    out->npoly = in->npoly;
    return CKC_OK;
}

extern "C" int ckc_mod_drop(ckc_ctx *c, const ckc_ct *in, int to_level, ckc_ct *out, void *stream) {
    CKC_TRY(check_ct(c, in, "mod_drop"));
    CKC_REQUIRE(out && out->d, CKC_EINVAL, "null output");
    CKC_REQUIRE(to_level >= 0 && to_level <= in->level, CKC_ELEVEL, "bad target level");
    const size_t N = c->N;
    const size_t in_ps = size_t(in->level + 1) * N, out_ps = size_t(to_level + 1) * N;
    hipStream_t s = S(stream);
    if (out->d == in->d) {
        // compact in place, poly by poly (poly 0 needs no move)
        for (int p = 1; p < in->npoly; ++p) {
            DevBuf tmp;
            CKC_TRY(tmp.alloc(8 * out_ps, s));
            CKC_TRY(copy_limbs(in->d + p * in_ps, 0, tmp.u64(), 0, out_ps, 1, s));
            CKC_TRY(copy_limbs(tmp.u64(), 0, out->d + p * out_ps, 0, out_ps, 1, s));
        }
    } else {
        CKC_TRY(copy_limbs(in->d, in_ps, out->d, out_ps, out_ps, in->npoly, s));
    }
    out->level = to_level;
    out->npoly = in->npoly;
    out->scale = in->scale;
    return CKC_OK;
}
