/*
 * CPU oracle for the leveled RNS-CKKS evaluator -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, exact C.  Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg load this library; the product path never does.  It shares
 * no code with the GPU library: every definition here is written from the
 * mathematics of RNS-CKKS (paper Section 2.2, "Leveled Fully Homomorphic
 * Encryption") and the canonical readings listed in the design notes.
 *
 * Representation: every polynomial is held in COEFFICIENT form, one limb per
 * prime, limb-major ([limb][N] uint64, values in [0, q)).  Products are taken
 * through a textbook negacyclic NTT (evaluation at psi^(2k+1), natural order),
 * which is an internal detail: results are always returned in coefficient
 * form, so nothing here depends on how the GPU orders its NTT domain.
 *
 * Functions follow the RNS-CKKS operations the paper relies on (Section 2.2):
 * encoding with scale Delta, RLWE encryption, addition, multiplication,
 * rotation by a slot step, rescaling that drops one modulus, and hybrid key
 * switching with a special modulus P.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

/* pi as the nearest double (0x400921FB54442D18) */
static const double OC_PI = 3.14159265358979323846;

typedef unsigned __int128 u128;

#define OC_MAXP 96

/* ------------------------------------------------------------------------ */
/* scalar modular arithmetic (q < 2^63)                                      */
/* ------------------------------------------------------------------------ */
static inline uint64_t mulmod(uint64_t a, uint64_t b, uint64_t q) {
    return (uint64_t)(((u128)a * b) % q);
}
static inline uint64_t addmod(uint64_t a, uint64_t b, uint64_t q) {
    uint64_t s = a + b;
    return s >= q ? s - q : s;
}
static inline uint64_t submod(uint64_t a, uint64_t b, uint64_t q) {
    return a >= b ? a - b : a + (q - b);
}
static uint64_t powmod(uint64_t a, uint64_t e, uint64_t q) {
    uint64_t r = 1 % q;
    a %= q;
    while (e) {
        if (e & 1) r = mulmod(r, a, q);
        a = mulmod(a, a, q);
        e >>= 1;
    }
    return r;
}
/* q prime: Fermat inverse */
static uint64_t invmod(uint64_t a, uint64_t q) { return powmod(a % q, q - 2, q); }

/* signed integer -> residue in [0, q) */
static inline uint64_t from_signed(int64_t v, uint64_t q) {
    if (v >= 0) return (uint64_t)v % q;
    uint64_t m = (uint64_t)(-(v + 1)) + 1; /* |v| without overflow */
    m %= q;
    return m ? q - m : 0;
}

/* ------------------------------------------------------------------------ */
/* SplitMix64 (Steele, Lea, Flood 2014) in counter form                      */
/* ------------------------------------------------------------------------ */
static const uint64_t GAMMA = 0x9e3779b97f4a7c15ULL;
static inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}
/* stream key for (master seed, tag, index) */
uint64_t oc_stream_key(uint64_t seed, uint64_t tag, uint64_t idx) {
    return mix64(mix64(seed + tag * GAMMA) + idx * GAMMA);
}
/* j-th output of the SplitMix64 generator whose state starts at key */
uint64_t oc_draw(uint64_t key, uint64_t j) { return mix64(key + (j + 1) * GAMMA); }

/* samplers, all counter based (no rejection) */
static inline uint64_t uniform_mod(uint64_t u, uint64_t q) { return (uint64_t)(((u128)u * q) >> 64); }
static inline int ternary(uint64_t u) {
    int t = (int)(((u128)u * 3) >> 64); /* 0, 1, 2 */
    return t == 2 ? -1 : t;
}
static inline int cbd21(uint64_t u) {
    return __builtin_popcountll(u & 0x1fffffULL) - __builtin_popcountll((u >> 21) & 0x1fffffULL);
}

enum { TAG_SECRET = 1, TAG_KEY_A = 2, TAG_KEY_E = 3, TAG_ENC_A = 4, TAG_ENC_E = 5 };

/* ------------------------------------------------------------------------ */
/* context: the prime list and per-prime NTT tables                          */
/* ------------------------------------------------------------------------ */
typedef struct {
    int logN;
    size_t N;
    int nprimes;           /* total primes: Q chain then P */
    int nq, np;
    uint64_t mod[OC_MAXP];
    uint64_t psi[OC_MAXP]; /* primitive 2N-th root of unity */
    uint64_t *psi_pow;     /* [nprimes][N]  psi^i           */
    uint64_t *ipsi_pow;    /* [nprimes][N]  psi^-i * N^-1   */
    uint64_t *w_pow;       /* [nprimes][N/2] omega^i, omega = psi^2 */
    uint64_t *iw_pow;      /* [nprimes][N/2] omega^-i */
} oc_ctx;

static uint64_t find_psi(uint64_t q, size_t N) {
    /* smallest x >= 2 whose (q-1)/2N power has order exactly 2N */
    for (uint64_t x = 2;; ++x) {
        uint64_t g = powmod(x, (q - 1) / (2 * N), q);
        if (powmod(g, N, q) == q - 1) return g;
    }
}

oc_ctx *oc_create(int logN, int nq, const uint64_t *q, int np, const uint64_t *p) {
    if (nq + np > OC_MAXP) return NULL;
    oc_ctx *c = (oc_ctx *)calloc(1, sizeof(oc_ctx));
    c->logN = logN;
    c->N = (size_t)1 << logN;
    c->nq = nq;
    c->np = np;
    c->nprimes = nq + np;
    for (int i = 0; i < nq; ++i) c->mod[i] = q[i];
    for (int i = 0; i < np; ++i) c->mod[nq + i] = p[i];
    size_t N = c->N;
    c->psi_pow = (uint64_t *)malloc(sizeof(uint64_t) * N * c->nprimes);
    c->ipsi_pow = (uint64_t *)malloc(sizeof(uint64_t) * N * c->nprimes);
    c->w_pow = (uint64_t *)malloc(sizeof(uint64_t) * (N / 2) * c->nprimes);
    c->iw_pow = (uint64_t *)malloc(sizeof(uint64_t) * (N / 2) * c->nprimes);
    for (int t = 0; t < c->nprimes; ++t) {
        uint64_t m = c->mod[t];
        uint64_t psi = find_psi(m, N);
        c->psi[t] = psi;
        uint64_t ipsi = invmod(psi, m), ninv = invmod(N % m, m);
        uint64_t *pp = c->psi_pow + (size_t)t * N, *ip = c->ipsi_pow + (size_t)t * N;
        uint64_t x = 1, y = ninv;
        for (size_t i = 0; i < N; ++i) {
            pp[i] = x;
            ip[i] = y;
            x = mulmod(x, psi, m);
            y = mulmod(y, ipsi, m);
        }
        uint64_t w = mulmod(psi, psi, m), iw = invmod(w, m);
        uint64_t *wp = c->w_pow + (size_t)t * (N / 2), *iwp = c->iw_pow + (size_t)t * (N / 2);
        x = 1;
        y = 1;
        for (size_t i = 0; i < N / 2; ++i) {
            wp[i] = x;
            iwp[i] = y;
            x = mulmod(x, w, m);
            y = mulmod(y, iw, m);
        }
    }
    return c;
}

void oc_destroy(oc_ctx *c) {
    if (!c) return;
    free(c->psi_pow);
    free(c->ipsi_pow);
    free(c->w_pow);
    free(c->iw_pow);
    free(c);
}

uint64_t oc_psi(const oc_ctx *c, int t) { return c->psi[t]; }

/* ------------------------------------------------------------------------ */
/* negacyclic NTT (textbook): A_k = a(psi^(2k+1)), k in natural order        */
/* ------------------------------------------------------------------------ */
static void bit_reverse(uint64_t *a, size_t N) {
    for (size_t i = 1, j = 0; i < N; ++i) {
        size_t bit = N >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) {
            uint64_t t = a[i];
            a[i] = a[j];
            a[j] = t;
        }
    }
}

/* cyclic DFT over Z_q with root table wp[i] = w^i (i < N/2), w of order N */
static void cyclic_ntt(uint64_t *a, size_t N, uint64_t q, const uint64_t *wp) {
    bit_reverse(a, N);
    for (size_t len = 2; len <= N; len <<= 1) {
        size_t half = len >> 1, step = N / len;
        for (size_t i = 0; i < N; i += len) {
            for (size_t j = 0; j < half; ++j) {
                uint64_t u = a[i + j];
                uint64_t v = mulmod(a[i + j + half], wp[j * step], q);
                a[i + j] = addmod(u, v, q);
                a[i + j + half] = submod(u, v, q);
            }
        }
    }
}

void oc_ntt(const oc_ctx *c, int t, uint64_t *a) {
    size_t N = c->N;
    uint64_t q = c->mod[t];
    const uint64_t *pp = c->psi_pow + (size_t)t * N;
    for (size_t i = 0; i < N; ++i) a[i] = mulmod(a[i], pp[i], q);
    cyclic_ntt(a, N, q, c->w_pow + (size_t)t * (N / 2));
}

void oc_intt(const oc_ctx *c, int t, uint64_t *a) {
    size_t N = c->N;
    uint64_t q = c->mod[t];
    cyclic_ntt(a, N, q, c->iw_pow + (size_t)t * (N / 2));
    const uint64_t *ip = c->ipsi_pow + (size_t)t * N;
    for (size_t i = 0; i < N; ++i) a[i] = mulmod(a[i], ip[i], q);
}

/* c = a * b mod (X^N + 1, q_t), all coefficient form; c may alias a or b */
void oc_polymul(const oc_ctx *c, int t, const uint64_t *a, const uint64_t *b, uint64_t *out) {
    size_t N = c->N;
    uint64_t q = c->mod[t];
    uint64_t *x = (uint64_t *)malloc(8 * N), *y = (uint64_t *)malloc(8 * N);
    memcpy(x, a, 8 * N);
    memcpy(y, b, 8 * N);
    oc_ntt(c, t, x);
    oc_ntt(c, t, y);
    for (size_t i = 0; i < N; ++i) x[i] = mulmod(x[i], y[i], q);
    oc_intt(c, t, x);
    memcpy(out, x, 8 * N);
    free(x);
    free(y);
}

/* ------------------------------------------------------------------------ */
/* automorphism sigma_g : a(X) -> a(X^g), g odd                               */
/* ------------------------------------------------------------------------ */
void oc_automorphism(const oc_ctx *c, int t, const uint64_t *a, uint64_t g, uint64_t *out) {
    size_t N = c->N;
    uint64_t q = c->mod[t], mask = 2 * N - 1;
    for (size_t i = 0; i < N; ++i) {
        uint64_t e = ((uint64_t)i * g) & mask; /* X^i -> X^(ig mod 2N) */
        if (e < N)
            out[e] = a[i];
        else
            out[e - N] = a[i] ? q - a[i] : 0; /* X^N = -1 */
    }
}

/* Galois element of a left rotation by r slots: 5^(r mod N/2) mod 2N */
uint64_t oc_galois_elt(const oc_ctx *c, int64_t r) {
    int64_t n = (int64_t)(c->N / 2);
    int64_t rr = ((r % n) + n) % n;
    uint64_t g = 1, m = 2 * c->N;
    for (int64_t i = 0; i < rr; ++i) g = (g * 5) % m;
    return g;
}

/* ------------------------------------------------------------------------ */
/* PRNG-driven sampling (canonical draw order, shared by definition only)    */
/* ------------------------------------------------------------------------ */
/* secret: s_k in {-1,0,1}, draw k of stream (seed, SECRET, 0) */
void oc_sample_secret(const oc_ctx *c, uint64_t seed, int8_t *s) {
    uint64_t key = oc_stream_key(seed, TAG_SECRET, 0);
    for (size_t k = 0; k < c->N; ++k) s[k] = (int8_t)ternary(oc_draw(key, k));
}

/* ternary vector -> limbs of the listed primes */
static void signed_small_to_limb(const int32_t *v, size_t N, uint64_t q, uint64_t *out) {
    for (size_t k = 0; k < N; ++k) out[k] = from_signed(v[k], q);
}

/* ------------------------------------------------------------------------ */
/* key generation                                                             */
/*                                                                            */
/* Hybrid key switching from s' to s with digits D_j = {q_{j*alpha} ..}:      */
/*   b_j = -a_j*s + e_j + P*Theta_j*s'   over every Q and P prime,            */
/*   a_j  uniform,  Theta_j = 1 mod primes of D_j, 0 mod the others.          */
/* Output layout: key[j][2][nprimes][N] coefficient form, poly 0 = b, 1 = a.  */
/* key_id selects the PRNG streams (0 = relinearisation, g = Galois elt g).   */
/* ------------------------------------------------------------------------ */
void oc_keygen_switch(const oc_ctx *c, uint64_t seed, uint64_t key_id, int alpha,
                      const int8_t *s, const uint64_t *sprime /* [nprimes][N] coeff */,
                      uint64_t *key /* [dnum][2][nprimes][N] */) {
    size_t N = c->N;
    int np = c->nprimes, nq = c->nq;
    int dnum = (nq + alpha - 1) / alpha;
    int32_t *sv = (int32_t *)malloc(4 * N), *ev = (int32_t *)malloc(4 * N);
    for (size_t k = 0; k < N; ++k) sv[k] = s[k];
    uint64_t *slimb = (uint64_t *)malloc(8 * N), *tmp = (uint64_t *)malloc(8 * N);
    for (int j = 0; j < dnum; ++j) {
        uint64_t ka = oc_stream_key(seed, TAG_KEY_A, key_id * 64 + (uint64_t)j);
        uint64_t ke = oc_stream_key(seed, TAG_KEY_E, key_id * 64 + (uint64_t)j);
        for (size_t k = 0; k < N; ++k) ev[k] = cbd21(oc_draw(ke, k));
        for (int t = 0; t < np; ++t) {
            uint64_t q = c->mod[t];
            uint64_t *b = key + (((size_t)j * 2 + 0) * np + t) * N;
            uint64_t *a = key + (((size_t)j * 2 + 1) * np + t) * N;
            for (size_t k = 0; k < N; ++k) a[k] = uniform_mod(oc_draw(ka, (uint64_t)t * N + k), q);
            signed_small_to_limb(sv, N, q, slimb);
            oc_polymul(c, t, a, slimb, tmp); /* a*s */
            for (size_t k = 0; k < N; ++k) b[k] = submod(from_signed(ev[k], q), tmp[k], q);
            int in_digit = (t < nq) && (t / alpha == j);
            if (in_digit) {
                uint64_t Pm = 1 % q; /* P mod q_t */
                for (int i = 0; i < c->np; ++i) Pm = mulmod(Pm, c->mod[nq + i] % q, q);
                const uint64_t *sp = sprime + (size_t)t * N;
                for (size_t k = 0; k < N; ++k) b[k] = addmod(b[k], mulmod(Pm, sp[k], q), q);
            }
        }
    }
    free(sv);
    free(ev);
    free(slimb);
    free(tmp);
}

/* ------------------------------------------------------------------------ */
/* encryption / decryption (symmetric, the client holds s)                   */
/* ct = (-a*s + m + e, a) over q_0..q_level, a uniform, e centred binomial   */
/* ------------------------------------------------------------------------ */
void oc_encrypt(const oc_ctx *c, uint64_t seed, uint64_t stream_id, const int8_t *s,
                const uint64_t *m /* [level+1][N] */, int level, uint64_t *ct /* [2][level+1][N] */) {
    size_t N = c->N;
    int nl = level + 1;
    uint64_t ka = oc_stream_key(seed, TAG_ENC_A, stream_id);
    uint64_t ke = oc_stream_key(seed, TAG_ENC_E, stream_id);
    int32_t *ev = (int32_t *)malloc(4 * N), *sv = (int32_t *)malloc(4 * N);
    for (size_t k = 0; k < N; ++k) {
        ev[k] = cbd21(oc_draw(ke, k));
        sv[k] = s[k];
    }
    uint64_t *slimb = (uint64_t *)malloc(8 * N), *tmp = (uint64_t *)malloc(8 * N);
    for (int t = 0; t < nl; ++t) {
        uint64_t q = c->mod[t];
        uint64_t *c0 = ct + (size_t)t * N, *c1 = ct + ((size_t)nl + t) * N;
        for (size_t k = 0; k < N; ++k) c1[k] = uniform_mod(oc_draw(ka, (uint64_t)t * N + k), q);
        signed_small_to_limb(sv, N, q, slimb);
        oc_polymul(c, t, c1, slimb, tmp);
        const uint64_t *mt = m + (size_t)t * N;
        for (size_t k = 0; k < N; ++k)
            c0[k] = addmod(submod(mt[k], tmp[k], q), from_signed(ev[k], q), q);
    }
    free(ev);
    free(sv);
    free(slimb);
    free(tmp);
}

/* m = c0 + c1*s (+ c2*s^2) over q_0..q_level */
void oc_decrypt(const oc_ctx *c, const int8_t *s, const uint64_t *ct, int npoly, int level, uint64_t *m) {
    size_t N = c->N;
    int nl = level + 1;
    int32_t *sv = (int32_t *)malloc(4 * N);
    for (size_t k = 0; k < N; ++k) sv[k] = s[k];
    uint64_t *slimb = (uint64_t *)malloc(8 * N), *s2 = (uint64_t *)malloc(8 * N), *tmp = (uint64_t *)malloc(8 * N);
    for (int t = 0; t < nl; ++t) {
        uint64_t q = c->mod[t];
        signed_small_to_limb(sv, N, q, slimb);
        const uint64_t *c0 = ct + (size_t)t * N, *c1 = ct + ((size_t)nl + t) * N;
        oc_polymul(c, t, c1, slimb, tmp);
        uint64_t *mt = m + (size_t)t * N;
        for (size_t k = 0; k < N; ++k) mt[k] = addmod(c0[k], tmp[k], q);
        if (npoly == 3) {
            const uint64_t *c2 = ct + ((size_t)2 * nl + t) * N;
            oc_polymul(c, t, slimb, slimb, s2);
            oc_polymul(c, t, c2, s2, tmp);
            for (size_t k = 0; k < N; ++k) mt[k] = addmod(mt[k], tmp[k], q);
        }
    }
    free(sv);
    free(slimb);
    free(s2);
    free(tmp);
}

/* ------------------------------------------------------------------------ */
/* hybrid key switching                                                       */
/* ------------------------------------------------------------------------ */
/*
 * ModUp of digit j of d (coefficient form, limbs q_0..q_level):
 * digit primes D = {q_i : i in [j*alpha, min(j*alpha+alpha-1, level)]}, Q_j
 * their product.  For every target prime t (q_0..q_level then P):
 *   t in D : the limb itself;
 *   else   : sum_{i in D} v_i * (Q_j/q_i mod t)  mod t,
 *            v_i = [d_i * (Q_j/q_i)^-1]_{q_i} taken in (-q_i/2, q_i/2]
 * (fast basis conversion, no correction term, centred: the digit is lifted
 * to its centred representative plus u Q_j with |u| < |D|/2.  The key switch
 * multiplies the digit by the key's error; a digit lifted from [0, Q_j)
 * carries a mean of about Q_j/2 in every coefficient, and that constant
 * polynomial times the error sums the error's coefficients, which in the
 * slots near 1 grows like N^1.5.)
 * out: [level+1+np][N].
 */
void oc_modup_digit(const oc_ctx *c, const uint64_t *d, int level, int alpha, int j, uint64_t *out) {
    size_t N = c->N;
    int lo = j * alpha, hi = j * alpha + alpha - 1;
    if (hi > level) hi = level;
    int nd = hi - lo + 1;
    int ntarget = level + 1 + c->np;
    /* (Q_j/q_i)^-1 mod q_i */
    uint64_t qhat_inv[OC_MAXP];
    for (int a = 0; a < nd; ++a) {
        uint64_t qi = c->mod[lo + a], prod = 1 % qi;
        for (int b = 0; b < nd; ++b)
            if (b != a) prod = mulmod(prod, c->mod[lo + b] % qi, qi);
        qhat_inv[a] = invmod(prod, qi);
    }
    uint64_t *y = (uint64_t *)malloc(8 * N * nd);
    for (int a = 0; a < nd; ++a) {
        uint64_t qi = c->mod[lo + a];
        const uint64_t *di = d + (size_t)(lo + a) * N;
        for (size_t k = 0; k < N; ++k) y[(size_t)a * N + k] = mulmod(di[k], qhat_inv[a], qi);
    }
    for (int tt = 0; tt < ntarget; ++tt) {
        int t = tt <= level ? tt : c->nq + (tt - level - 1); /* prime index */
        uint64_t *o = out + (size_t)tt * N;
        if (tt >= lo && tt <= hi) {
            memcpy(o, d + (size_t)tt * N, 8 * N);
            continue;
        }
        uint64_t m = c->mod[t];
        uint64_t qhat_t[OC_MAXP]; /* Q_j/q_i mod t */
        uint64_t Qj_t = 1 % m;    /* Q_j mod t */
        for (int a = 0; a < nd; ++a) {
            uint64_t prod = 1 % m;
            for (int b = 0; b < nd; ++b)
                if (b != a) prod = mulmod(prod, c->mod[lo + b] % m, m);
            qhat_t[a] = prod;
            Qj_t = mulmod(Qj_t, c->mod[lo + a] % m, m);
        }
        for (size_t k = 0; k < N; ++k) {
            uint64_t acc = 0;
            for (int a = 0; a < nd; ++a) {
                uint64_t qa = c->mod[lo + a], v = y[(size_t)a * N + k];
                acc = addmod(acc, mulmod(v % m, qhat_t[a], m), m);
                /* v > qa/2 stands for v - qa: subtract qa (Q_j/qa) = Q_j */
                if (v > qa / 2) acc = submod(acc, Qj_t, m);
            }
            o[k] = acc;
        }
    }
    free(y);
}

/*
 * ModDown: x over q_0..q_level then P (coefficient form) ->
 *   [x_i - FastBConv_{P -> q_i}(x_P)] * P^-1 mod q_i,  i <= level
 * with the centred fast conversion
 *   FastBConv_{P->q}(x) = sum_k v_k (P/p_k mod q),
 *   v_k = [x_k (P/p_k)^-1]_{p_k} taken in (-p_k/2, p_k/2],
 * which is x_P + u P with |u| < np/2, so the division by P rounds to the
 * nearest integer up to a symmetric error: an unbiased rounding (a biased
 * one, such as the same sum over [0, p_k), adds a constant times (c1 part) s
 * to the decryption, whose slot values grow like N^1.5 in the slots near 1).
 */
void oc_moddown(const oc_ctx *c, const uint64_t *x, int level, uint64_t *out) {
    size_t N = c->N;
    int np = c->np, nq = c->nq;
    uint64_t phat_inv[OC_MAXP];
    for (int a = 0; a < np; ++a) {
        uint64_t pa = c->mod[nq + a], prod = 1 % pa;
        for (int b = 0; b < np; ++b)
            if (b != a) prod = mulmod(prod, c->mod[nq + b] % pa, pa);
        phat_inv[a] = invmod(prod, pa);
    }
    uint64_t *y = (uint64_t *)malloc(8 * N * np);
    for (int a = 0; a < np; ++a) {
        uint64_t pa = c->mod[nq + a];
        const uint64_t *xa = x + (size_t)(level + 1 + a) * N;
        for (size_t k = 0; k < N; ++k) y[(size_t)a * N + k] = mulmod(xa[k], phat_inv[a], pa);
    }
    for (int i = 0; i <= level; ++i) {
        uint64_t q = c->mod[i];
        uint64_t phat_q[OC_MAXP], Pq = 1 % q;
        for (int a = 0; a < np; ++a) {
            uint64_t prod = 1 % q;
            for (int b = 0; b < np; ++b)
                if (b != a) prod = mulmod(prod, c->mod[nq + b] % q, q);
            phat_q[a] = prod;
            Pq = mulmod(Pq, c->mod[nq + a] % q, q);
        }
        uint64_t Pinv = invmod(Pq, q);
        const uint64_t *xi = x + (size_t)i * N;
        uint64_t *o = out + (size_t)i * N;
        for (size_t k = 0; k < N; ++k) {
            uint64_t conv = 0;
            for (int a = 0; a < np; ++a) {
                uint64_t pa = c->mod[nq + a], v = y[(size_t)a * N + k];
                conv = addmod(conv, mulmod(v % q, phat_q[a], q), q);
                /* v > pa/2 stands for v - pa: subtract pa (P/pa) = P */
                if (v > pa / 2) conv = submod(conv, Pq, q);
            }
            o[k] = mulmod(submod(xi[k], conv, q), Pinv, q);
        }
    }
    free(y);
}

/*
 * Key switch of d (coefficient form, q_0..q_level) under key (layout of
 * oc_keygen_switch, generated at the top level), with an optional Galois
 * element g applied to every ModUp output before the product (g = 1: none).
 * Returns the two polynomials (u0, u1) over q_0..q_level:
 *   u_b = ModDown( sum_j sigma_g(ModUp_j(d)) * key_j[b] ).
 */
/*
 * The key switch before its ModDown (the extended-basis product):
 *   acc_b = sum_j sigma_g(ModUp_j(d)) * key_j[b]   over q_0..q_level then P,
 * acc: [2][level+1+np][N] (coefficient form).
 */
void oc_keyswitch_ext(const oc_ctx *c, const uint64_t *d, int level, int alpha, uint64_t g,
                      const uint64_t *key, uint64_t *acc) {
    size_t N = c->N;
    int np = c->nprimes;
    int nt = level + 1 + c->np;
    int dnum_l = (level + 1 + alpha - 1) / alpha;
    uint64_t *digit = (uint64_t *)malloc(8 * N * nt);
    uint64_t *rot = (uint64_t *)malloc(8 * N);
    uint64_t *prod = (uint64_t *)malloc(8 * N);
    memset(acc, 0, (size_t)2 * nt * N * 8);
    for (int j = 0; j < dnum_l; ++j) {
        oc_modup_digit(c, d, level, alpha, j, digit);
        for (int tt = 0; tt < nt; ++tt) {
            int t = tt <= level ? tt : c->nq + (tt - level - 1);
            uint64_t q = c->mod[t];
            const uint64_t *dg = digit + (size_t)tt * N;
            if (g != 1) {
                oc_automorphism(c, t, dg, g, rot);
                dg = rot;
            }
            for (int b = 0; b < 2; ++b) {
                const uint64_t *kb = key + (((size_t)j * 2 + b) * np + t) * N;
                oc_polymul(c, t, dg, kb, prod);
                uint64_t *ab = acc + ((size_t)b * nt + tt) * N;
                for (size_t k = 0; k < N; ++k) ab[k] = addmod(ab[k], prod[k], q);
            }
        }
    }
    free(digit);
    free(rot);
    free(prod);
}

void oc_keyswitch(const oc_ctx *c, const uint64_t *d, int level, int alpha, uint64_t g,
                  const uint64_t *key, uint64_t *u /* [2][level+1][N] */) {
    size_t N = c->N;
    int nt = level + 1 + c->np;
    uint64_t *acc = (uint64_t *)malloc((size_t)2 * nt * N * 8);
    oc_keyswitch_ext(c, d, level, alpha, g, key, acc);
    for (int b = 0; b < 2; ++b) oc_moddown(c, acc + (size_t)b * nt * N, level, u + (size_t)b * (level + 1) * N);
    free(acc);
}

/* ------------------------------------------------------------------------ */
/* rescale with rounding: drop q_level                                        */
/*   t = [c]_{q_l}, centred to (-q_l/2, q_l/2];  c_i <- (c_i - t) q_l^-1     */
/* ------------------------------------------------------------------------ */
void oc_rescale(const oc_ctx *c, const uint64_t *x, int npoly, int level, uint64_t *out) {
    size_t N = c->N;
    uint64_t ql = c->mod[level], half = ql >> 1;
    for (int p = 0; p < npoly; ++p) {
        const uint64_t *top = x + ((size_t)p * (level + 1) + level) * N;
        for (int i = 0; i < level; ++i) {
            uint64_t q = c->mod[i], inv = invmod(ql % q, q);
            const uint64_t *xi = x + ((size_t)p * (level + 1) + i) * N;
            uint64_t *o = out + ((size_t)p * level + i) * N;
            for (size_t k = 0; k < N; ++k) {
                uint64_t tv = top[k];
                uint64_t tq = tv > half ? submod(tv % q, ql % q, q) : tv % q; /* centred t mod q */
                o[k] = mulmod(submod(xi[k], tq, q), inv, q);
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* encoding: canonical special FFT (fixed operation order, IEEE double)       */
/*                                                                            */
/* slots z_j (j < n = N/2) sit at the roots zeta^(5^j), zeta = e^(i pi / N).  */
/* With 5^j mod 2N = 1 + 4 t_j, the slot values are the length-n DFT of      */
/* w_k zeta^k evaluated at index t_j, where m_k = Re w_k, m_{k+n} = Im w_k.   */
/* Encoding inverts that:                                                     */
/*   y[t_j] = z_j;  Y = unnormalised inverse DFT (radix-2 DIT below);         */
/*   w_k = Y_k * (cos(pi k/N)/n, -sin(pi k/N)/n);  m = round(Delta * w).       */
/* ------------------------------------------------------------------------ */
/*
 * Canonical twiddles: (cos, sin)(2 pi j / M) for integers 0 <= j < M/2 and
 * M a power of two, computed with IEEE +, -, *, / only in one fixed order so
 * that every implementation gets the same bits (libm's cos/sin are not
 * bitwise reproducible across compilers).  The angle is folded into
 * [0, pi/4] by octant symmetry; cos and sin there are Taylor series
 * (12 terms) evaluated by Horner's rule.
 */
static void taylor_cs(double x, double *c, double *s) {
    /* signed coefficients (-1)^i / (2i)! and (-1)^i / (2i+1)!, by a chain of divisions */
    double ca[12], sa[12];
    double fc = 1.0, fs = 1.0;
    for (int i = 0; i < 12; ++i) {
        if (i > 0) {
            fc = fc / (double)((2 * i - 1) * (2 * i));
            fs = fs / (double)((2 * i) * (2 * i + 1));
        }
        ca[i] = (i & 1) ? -fc : fc;
        sa[i] = (i & 1) ? -fs : fs;
    }
    double y = x * x, pc = ca[11], ps = sa[11];
    for (int i = 10; i >= 0; --i) {
        pc = pc * y;
        pc = pc + ca[i];
        ps = ps * y;
        ps = ps + sa[i];
    }
    *c = pc;
    *s = x * ps;
}

static void canon_cs(uint64_t j, uint64_t M, double *c, double *s) {
    const double step = (2.0 * OC_PI) / (double)M;
    uint64_t o8 = M / 8, o4 = M / 4, o38 = 3 * (M / 8), o2 = M / 2;
    double a, b;
    if (j <= o8) {
        taylor_cs((double)j * step, &a, &b);
        *c = a;
        *s = b;
    } else if (j <= o4) {
        taylor_cs((double)(o4 - j) * step, &a, &b);
        *c = b;
        *s = a;
    } else if (j <= o38) {
        taylor_cs((double)(j - o4) * step, &a, &b);
        *c = -b;
        *s = a;
    } else {
        taylor_cs((double)(o2 - j) * step, &a, &b);
        *c = -a;
        *s = b;
    }
}

void oc_canon_cs(uint64_t j, uint64_t M, double *c, double *s) { canon_cs(j, M, c, s); }

static void fft_dit(double *re, double *im, size_t n, int inverse) {
    /* bit-reversal permutation */
    for (size_t i = 1, j = 0; i < n; ++i) {
        size_t bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) {
            double t = re[i];
            re[i] = re[j];
            re[j] = t;
            t = im[i];
            im[i] = im[j];
            im[j] = t;
        }
    }
    for (size_t len = 2; len <= n; len <<= 1) {
        size_t half = len >> 1, step = n / len;
        for (size_t i = 0; i < n; i += len) {
            for (size_t j = 0; j < half; ++j) {
                size_t e = j * step; /* twiddle exponent, < n/2 */
                double wr, ws;
                canon_cs(e, n, &wr, &ws);
                double wi = inverse ? -ws : ws;
                double xr = re[i + j + half], xi = im[i + j + half];
                double vr = xr * wr - xi * wi;
                double vi = xr * wi + xi * wr;
                double ur = re[i + j], ui = im[i + j];
                re[i + j] = ur + vr;
                im[i + j] = ui + vi;
                re[i + j + half] = ur - vr;
                im[i + j + half] = ui - vi;
            }
        }
    }
}

/* exact residue of the integer-valued double v modulo q */
static uint64_t double_int_mod(double v, uint64_t q) {
    if (fabs(v) < 9.2e18) return from_signed((int64_t)v, q);
    int e;
    double mant = frexp(fabs(v), &e); /* |v| = mant * 2^e, mant in [0.5,1) */
    uint64_t M = (uint64_t)ldexp(mant, 53);
    uint64_t r = mulmod(M % q, powmod(2, (uint64_t)(e - 53), q), q);
    return v < 0 ? (r ? q - r : 0) : r;
}

static void encode_limbs(const oc_ctx *c, const double *z_re, const double *z_im, size_t nslots, double delta,
                         int level, int with_p, uint64_t *m, double *w_out);

/* rounds half away from zero, then reduces into each of the first nl primes */
void oc_encode(const oc_ctx *c, const double *z_re, const double *z_im, size_t nslots, double delta,
               int level, uint64_t *m /* [level+1][N] */, double *w_out /* optional [2][n] */) {
    encode_limbs(c, z_re, z_im, nslots, delta, level, 0, m, w_out);
}

/* the same integer coefficients reduced into q_0..q_level and then every P
 * prime: m [level+1+np][N] (a plaintext of the extended basis Q_l u P) */
void oc_encode_ext(const oc_ctx *c, const double *z_re, const double *z_im, size_t nslots, double delta,
                   int level, uint64_t *m) {
    encode_limbs(c, z_re, z_im, nslots, delta, level, 1, m, NULL);
}

static void encode_limbs(const oc_ctx *c, const double *z_re, const double *z_im, size_t nslots, double delta,
                         int level, int with_p, uint64_t *m, double *w_out) {
    size_t N = c->N, n = N / 2;
    double *re = (double *)calloc(n, sizeof(double)), *im = (double *)calloc(n, sizeof(double));
    uint64_t g = 1, M2 = 2 * N;
    for (size_t j = 0; j < n; ++j) {
        size_t tj = (size_t)((g - 1) / 4);
        if (j < nslots) {
            re[tj] = z_re[j];
            im[tj] = z_im ? z_im[j] : 0.0;
        }
        g = (g * 5) % M2;
    }
    fft_dit(re, im, n, 1);
    for (size_t k = 0; k < n; ++k) {
        double cz, sz;
        canon_cs(k, 2 * N, &cz, &sz);
        double tr = cz * (1.0 / (double)n), ti = -sz * (1.0 / (double)n);
        double wr = re[k] * tr - im[k] * ti;
        double wi = re[k] * ti + im[k] * tr;
        re[k] = wr;
        im[k] = wi;
    }
    if (w_out) {
        memcpy(w_out, re, n * sizeof(double));
        memcpy(w_out + n, im, n * sizeof(double));
    }
    int nl = level + 1, nt = nl + (with_p ? c->np : 0);
    for (size_t k = 0; k < n; ++k) {
        double a = round(delta * re[k]), b = round(delta * im[k]);
        for (int t = 0; t < nt; ++t) {
            uint64_t q = c->mod[t < nl ? t : c->nq + (t - nl)];
            m[(size_t)t * N + k] = double_int_mod(a, q);
            m[(size_t)t * N + k + n] = double_int_mod(b, q);
        }
    }
    free(re);
    free(im);
}

/* decode from centred integer coefficients (already lifted, as doubles) */
void oc_decode(const oc_ctx *c, const double *mcoef /* [N] */, double scale, double *z_re, double *z_im) {
    size_t N = c->N, n = N / 2;
    double *re = (double *)malloc(n * sizeof(double)), *im = (double *)malloc(n * sizeof(double));
    for (size_t k = 0; k < n; ++k) {
        double tr, ti;
        canon_cs(k, 2 * N, &tr, &ti);
        double ar = mcoef[k], ai = mcoef[k + n];
        re[k] = ar * tr - ai * ti;
        im[k] = ar * ti + ai * tr;
    }
    fft_dit(re, im, n, 0);
    uint64_t g = 1, M2 = 2 * N;
    for (size_t j = 0; j < n; ++j) {
        size_t tj = (size_t)((g - 1) / 4);
        z_re[j] = re[tj] / scale;
        if (z_im) z_im[j] = im[tj] / scale;
        g = (g * 5) % M2;
    }
    free(re);
    free(im);
}

/* integer value of the constant c*scale (rounded), reduced mod the listed primes */
void oc_const_residues(const oc_ctx *c, double value, double scale, int nl, uint64_t *out) {
    double v = round(value * scale);
    for (int t = 0; t < nl; ++t) out[t] = double_int_mod(v, c->mod[t]);
}

/* ------------------------------------------------------------------------ */
/* limb-wise helpers used by the Python layer                                */
/* ------------------------------------------------------------------------ */
void oc_limb_add(const oc_ctx *c, int t, const uint64_t *a, const uint64_t *b, uint64_t *o) {
    uint64_t q = c->mod[t];
    for (size_t k = 0; k < c->N; ++k) o[k] = addmod(a[k], b[k], q);
}
void oc_limb_sub(const oc_ctx *c, int t, const uint64_t *a, const uint64_t *b, uint64_t *o) {
    uint64_t q = c->mod[t];
    for (size_t k = 0; k < c->N; ++k) o[k] = submod(a[k], b[k], q);
}
