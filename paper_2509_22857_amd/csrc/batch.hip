// Batched hybrid key switching and batched ciphertext kernels.
//
// One launch covers up to kMaxBatch ciphertexts.  The key inner product keeps
// each key word in registers and loops over the batch, so a Galois or
// relinearisation key is read from HBM once per launch instead of once per
// ciphertext.
#include <algorithm>

#include "batch.h"
#include "prof.h"

const BconvTable *modup_table(ckc_ctx *c, int level, int digit, int *rc);
const uint64_t *galois_table(ckc_ctx *c, uint64_t g, int *rc);
uint64_t galois_inverse(const ckc_ctx *c, uint64_t g);

namespace {

unsigned tiles(size_t N) { return unsigned(std::min<size_t>(N / 256, 64)); }

__global__ void k_gather(Ptrs src, size_t src_off, uint64_t *__restrict__ dst, size_t dst_bs, size_t words) {
    const int b = blockIdx.y;
    const uint64_t *s = src.p[b] + src_off;
    uint64_t *d = dst + b * dst_bs;
    for (size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x; k < words; k += size_t(gridDim.x) * blockDim.x)
        d[k] = s[k];
}

__global__ void k_copy_pp(Ptrs src, Ptrs dst, size_t words) {
    const int b = blockIdx.y;
    const uint64_t *sp = src.p[b];
    uint64_t *d = dst.p[b];
    for (size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x; k < words; k += size_t(gridDim.x) * blockDim.x)
        d[k] = sp[k];
}

// key inner product with key reuse across the batch.  A Galois key is stored
// permuted by sigma_g^-1 (key'[m] = key[pi_g^-1(m)]), and since sigma_g acts on
// NTT-form values as a permutation commuting with pointwise products,
//   sum_j sigma_g(D_j) * key_j = sigma_g(sum_j D_j * key'_j):
// the digits are read in order and only the two outputs are scattered,
//   u[b][p][tt][scat(m)] = sum_j digits[b][j][tt][m] * key'[j][p][prime(tt)][m]
// with scat = pi_g^-1 (none for relinearisation).  Q limbs (tt < nl) go to
// accq [b][2][nl][N], P limbs to accp [b][2][np][N].  One thread per
// coefficient keeps its 2 DNUM key words in registers for the whole batch;
// the digit loads of one ciphertext are issued together (DNUM is a template
// parameter, so the loop is straight-line code).  Keys are stored times 2^64
// mod q, so each output's sum ends in one Montgomery reduction (redc_accc),
// which removes that factor, instead of a general 128-bit reduction.
template <int DNUM>
__global__ __launch_bounds__(256) void k_kip_b(const uint64_t *__restrict__ digits, int nb, int dnum_rt, int nt,
                                               int nl, const uint64_t *__restrict__ key, int nprimes, LimbMap map,
                                               const uint32_t *__restrict__ scat, uint64_t *__restrict__ accq,
                                               uint64_t *__restrict__ accp, const Prime *__restrict__ primes,
                                               int logN) {
    const int tt = blockIdx.y;
    const size_t N = size_t(1) << logN;
    const int dnum = DNUM > 0 ? DNUM : dnum_rt;
    const int pi = map.prime(tt);
    const Prime P = primes[pi];
    const int np = nt - nl;
    const size_t dig_bs = size_t(dnum) * nt * N;
    const bool lowq = tt < nl;
    uint64_t *obase = lowq ? accq + size_t(tt) * N : accp + size_t(tt - nl) * N;
    const size_t o_bs = lowq ? size_t(2) * nl * N : size_t(2) * np * N;
    const size_t o_ps = lowq ? size_t(nl) * N : size_t(np) * N;
    constexpr int KD = DNUM > 0 ? DNUM : kMaxDnum;
    for (size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x; k < N; k += size_t(gridDim.x) * blockDim.x) {
        uint64_t kb[KD], ka[KD];
#pragma unroll
        for (int j = 0; j < KD; ++j) {
            if (DNUM > 0 || j < dnum) {
                kb[j] = key[((size_t(j) * 2 + 0) * nprimes + pi) * N + k];
                ka[j] = key[((size_t(j) * 2 + 1) * nprimes + pi) * N + k];
            }
        }
        const size_t dst = scat ? scat[k] : k;
        const uint64_t *dg = digits + size_t(tt) * N + k;
        uint64_t *ob = obase + dst;
        for (int b = 0; b < nb; ++b) {
            uint64_t d[KD];
#pragma unroll
            for (int j = 0; j < KD; ++j)
                if (DNUM > 0 || j < dnum) d[j] = dg[size_t(j) * nt * N];
            accc a0{0, 0, 0, 0, 0}, a1{0, 0, 0, 0, 0};
#pragma unroll
            for (int j = 0; j < KD; ++j) {
                if (DNUM > 0 || j < dnum) {
                    macc(a0, d[j], kb[j]);
                    macc(a1, d[j], ka[j]);
                }
            }
            ob[0] = redc_accc<KD>(a0, P);
            ob[o_ps] = redc_accc<KD>(a1, P);
            dg += dig_bs;
            ob += o_bs;
        }
    }
}

using KipFn = void (*)(const uint64_t *, int, int, int, int, const uint64_t *, int, LimbMap, const uint32_t *,
                       uint64_t *, uint64_t *, const Prime *, int);
KipFn kip_kernel(int dnum) {
    switch (dnum) {
        case 1: return k_kip_b<1>;
        case 2: return k_kip_b<2>;
        case 3: return k_kip_b<3>;
        case 4: return k_kip_b<4>;
        case 5: return k_kip_b<5>;
        case 6: return k_kip_b<6>;
        case 7: return k_kip_b<7>;
        case 8: return k_kip_b<8>;
        default: return k_kip_b<0>;
    }
}

// key inner product kept in the extended basis (double hoisting): the same
// products as k_kip_b, written to dst.p[b] = [2][nt][N] at index scat(m), with
// P * c0[b][m] added on the Q limbs of polynomial 0 (at the output index
// scat(m) the rotated c0 is c0[pi_g(scat(m))] = c0[m], so the thread reads
// its own, coalesced, word of c0).
template <int DNUM>
__global__ __launch_bounds__(256) void k_kip_ext(const uint64_t *__restrict__ digits, int nb, int dnum_rt, int nt,
                                                 int nl, const uint64_t *__restrict__ key, int nprimes, LimbMap map,
                                                 const uint32_t *__restrict__ scat, Ptrs c0, Ptrs dst,
                                                 const uint64_t *__restrict__ pmod, const Prime *__restrict__ primes,
                                                 int logN) {
    const int tt = blockIdx.y;
    const size_t N = size_t(1) << logN;
    const int dnum = DNUM > 0 ? DNUM : dnum_rt;
    const int pi = map.prime(tt);
    const Prime P = primes[pi];
    const size_t dig_bs = size_t(dnum) * nt * N;
    const bool lowq = tt < nl;
    const uint64_t pm = lowq ? mul_shoup(pmod[2 * tt], P.r2, P.r2p, P.q) : 0;  // P 2^64 mod q
    constexpr int KD = DNUM > 0 ? DNUM : kMaxDnum;
    for (size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x; k < N; k += size_t(gridDim.x) * blockDim.x) {
        uint64_t kb[KD], ka[KD];
#pragma unroll
        for (int j = 0; j < KD; ++j) {
            if (DNUM > 0 || j < dnum) {
                kb[j] = key[((size_t(j) * 2 + 0) * nprimes + pi) * N + k];
                ka[j] = key[((size_t(j) * 2 + 1) * nprimes + pi) * N + k];
            }
        }
        const size_t out = size_t(tt) * N + scat[k];
        const uint64_t *dg = digits + size_t(tt) * N + k;
        for (int b = 0; b < nb; ++b) {
            uint64_t d[KD];
#pragma unroll
            for (int j = 0; j < KD; ++j)
                if (DNUM > 0 || j < dnum) d[j] = dg[size_t(j) * nt * N];
            accc a0{0, 0, 0, 0, 0}, a1{0, 0, 0, 0, 0};
#pragma unroll
            for (int j = 0; j < KD; ++j) {
                if (DNUM > 0 || j < dnum) {
                    macc(a0, d[j], kb[j]);
                    macc(a1, d[j], ka[j]);
                }
            }
            // P c0 joins the sum as one more product (pm = P 2^64 mod q, c0 < q)
            if (lowq) macc(a0, c0.p[b][size_t(tt) * N + k], pm);
            uint64_t *o = dst.p[b] + out;
            o[0] = redc_accc<KD + 1>(a0, P);
            o[size_t(nt) * N] = redc_accc<KD>(a1, P);
            dg += dig_bs;
        }
    }
}

// The same for up to kMaxRot rotations of the batch in one launch: block id
// -> (rotation r, tile-limb pair) with the pair's low 3 bits equal to id mod
// 8, so the r blocks of one 256-coefficient tile of one limb are dispatched
// within 8 nrot consecutive ids to the same XCD (workgroups go round-robin
// over the 8 XCDs) and all but the first find the tile's digits in that XCD's
// L2: the digits cross HBM about once instead of once per rotation.  Output
// of rotation r for input b at dst.p[b] + off[r] (the same layout as above).
constexpr int kMaxRot = 8;
struct KipRot {
    const uint64_t *key[kMaxRot];
    const uint32_t *scat[kMaxRot];
    int64_t off[kMaxRot];
};
template <int DNUM>
__global__ __launch_bounds__(256) void k_kip_ext_rot(const uint64_t *__restrict__ digits, int nb, int dnum_rt, int nt,
                                                     int nl, int nrot, KipRot kr, int nprimes, LimbMap map, Ptrs c0,
                                                     Ptrs dst, const uint64_t *__restrict__ pmod,
                                                     const Prime *__restrict__ primes, int logN) {
    const size_t N = size_t(1) << logN;
    const unsigned ntile = unsigned(N >> 8);
    const unsigned id = blockIdx.x, r = (id >> 3) % unsigned(nrot);
    const unsigned tl = (id / (8u * unsigned(nrot))) * 8u + (id & 7u);
    const int tt = int(tl / ntile);
    const size_t k = size_t(tl % ntile) * 256 + threadIdx.x;
    const int dnum = DNUM > 0 ? DNUM : dnum_rt;
    const int pi = map.prime(tt);
    const Prime P = primes[pi];
    const size_t dig_bs = size_t(dnum) * nt * N;
    const bool lowq = tt < nl;
    const uint64_t pm = lowq ? mul_shoup(pmod[2 * tt], P.r2, P.r2p, P.q) : 0;  // P 2^64 mod q
    const uint64_t *key = kr.key[r];
    constexpr int KD = DNUM > 0 ? DNUM : kMaxDnum;
    uint64_t kb[KD], ka[KD];
#pragma unroll
    for (int j = 0; j < KD; ++j) {
        if (DNUM > 0 || j < dnum) {
            kb[j] = key[((size_t(j) * 2 + 0) * nprimes + pi) * N + k];
            ka[j] = key[((size_t(j) * 2 + 1) * nprimes + pi) * N + k];
        }
    }
    const int64_t out = kr.off[r] + int64_t(tt) * int64_t(N) + int64_t(kr.scat[r][k]);
    const uint64_t *dg = digits + size_t(tt) * N + k;
    // the digits (and c0 word) of input b + 1 are loaded while input b's
    // products run; two buffers swap roles (a register copy would wait for
    // its load)
    auto load = [&](uint64_t(&d)[KD + 1], int b) {
        if (b >= nb) return;
#pragma unroll
        for (int j = 0; j < KD; ++j)
            if (DNUM > 0 || j < dnum) d[j] = dg[size_t(b) * dig_bs + size_t(j) * nt * N];
        if (lowq) d[KD] = c0.p[b][size_t(tt) * N + k];
    };
    auto body = [&](const uint64_t(&d)[KD + 1], int b) {
        accc a0{0, 0, 0, 0, 0}, a1{0, 0, 0, 0, 0};
#pragma unroll
        for (int j = 0; j < KD; ++j) {
            if (DNUM > 0 || j < dnum) {
                macc(a0, d[j], kb[j]);
                macc(a1, d[j], ka[j]);
            }
        }
        // P c0 joins the sum as one more product (pm = P 2^64 mod q, c0 < q)
        if (lowq) macc(a0, d[KD], pm);
        uint64_t *o = dst.p[b] + out;
        o[0] = redc_accc<KD + 1>(a0, P);
        o[size_t(nt) * N] = redc_accc<KD>(a1, P);
    };
    uint64_t da[KD + 1], db[KD + 1];
    load(da, 0);
    for (int b = 0; b < nb; b += 2) {
        load(db, b + 1);
        body(da, b);
        load(da, b + 2);
        if (b + 1 < nb) body(db, b + 1);
    }
}
using KipRotFn = void (*)(const uint64_t *, int, int, int, int, int, KipRot, int, LimbMap, Ptrs, Ptrs,
                          const uint64_t *, const Prime *, int);
KipRotFn kip_rot_kernel(int dnum) {
    switch (dnum) {
        case 1: return k_kip_ext_rot<1>;
        case 2: return k_kip_ext_rot<2>;
        case 3: return k_kip_ext_rot<3>;
        case 4: return k_kip_ext_rot<4>;
        case 5: return k_kip_ext_rot<5>;
        case 6: return k_kip_ext_rot<6>;
        case 7: return k_kip_ext_rot<7>;
        case 8: return k_kip_ext_rot<8>;
        default: return k_kip_ext_rot<0>;
    }
}

using KipExtFn = void (*)(const uint64_t *, int, int, int, int, const uint64_t *, int, LimbMap, const uint32_t *,
                          Ptrs, Ptrs, const uint64_t *, const Prime *, int);
KipExtFn kip_ext_kernel(int dnum) {
    switch (dnum) {
        case 1: return k_kip_ext<1>;
        case 2: return k_kip_ext<2>;
        case 3: return k_kip_ext<3>;
        case 4: return k_kip_ext<4>;
        case 5: return k_kip_ext<5>;
        case 6: return k_kip_ext<6>;
        case 7: return k_kip_ext<7>;
        case 8: return k_kip_ext<8>;
        default: return k_kip_ext<0>;
    }
}

// dst.p[b] = [2][nt][N]: P * in.p[b] on the Q limbs, zeros on the P limbs
__global__ __launch_bounds__(256) void k_lift_P(Ptrs in, Ptrs dst, int nl, int nt, const uint64_t *__restrict__ pmod,
                                                const Prime *__restrict__ primes, int logN) {
    const int tt = blockIdx.y, b = blockIdx.z >> 1, p = blockIdx.z & 1;
    const size_t N = size_t(1) << logN;
    uint64_t *o = dst.p[b] + (size_t(p) * nt + tt) * N;
    if (tt >= nl) {
        for (size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x; k < N; k += size_t(gridDim.x) * blockDim.x)
            o[k] = 0;
        return;
    }
    const uint64_t q = primes[tt].q, pm = pmod[2 * tt], pmp = pmod[2 * tt + 1];
    const uint64_t *x = in.p[b] + (size_t(p) * nl + tt) * N;
    for (size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x; k < N; k += size_t(gridDim.x) * blockDim.x)
        o[k] = mul_shoup(x[k], pm, pmp, q);
}

// rescale lift for a batch: top[b][p] (coefficient form) -> lift[b][p][i] = centred(top) mod q_i
__global__ __launch_bounds__(256) void k_rescale_lift_b(const uint64_t *__restrict__ top, int npoly,
                                                        uint64_t *__restrict__ lift, int level,
                                                        const Prime *__restrict__ primes, int logN) {
    const int i = blockIdx.y, bp = blockIdx.z;
    const size_t N = size_t(1) << logN;
    const uint64_t ql = primes[level].q, half = ql >> 1;
    const Prime P = primes[i];
    const uint64_t qlm = reduce64(ql, P);
    const uint64_t *t = top + size_t(bp) * N;
    uint64_t *o = lift + (size_t(bp) * level + i) * N;
    for (size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x; k < N; k += size_t(gridDim.x) * blockDim.x) {
        const uint64_t v = t[k];
        const uint64_t vm = reduce64(v, P);
        o[k] = v > half ? sub_mod(vm, qlm, P.q) : vm;
    }
}

__global__ __launch_bounds__(256) void k_rescale_combine_b(Ptrs in, int npoly, const uint64_t *__restrict__ lift,
                                                           Ptrs out, int level, const uint64_t *__restrict__ rinv,
                                                           const Prime *__restrict__ primes, int logN, int nq) {
    const int i = blockIdx.y, bp = blockIdx.z;
    const int b = bp / npoly, p = bp - b * npoly;
    const size_t N = size_t(1) << logN;
    const uint64_t q = primes[i].q;
    const uint64_t iv = rinv[(size_t(level) * nq + i) * 2], ivp = rinv[(size_t(level) * nq + i) * 2 + 1];
    const uint64_t *x = in.p[b] + (size_t(p) * (level + 1) + i) * N;
    const uint64_t *t = lift + (size_t(bp) * level + i) * N;
    uint64_t *o = out.p[b] + (size_t(p) * level + i) * N;
    for (size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x; k < N; k += size_t(gridDim.x) * blockDim.x)
        o[k] = mul_shoup(sub_mod(x[k], t[k], q), iv, ivp, q);
}

__global__ __launch_bounds__(256) void k_ew_b(int op, Ptrs out, Ptrs a, Ptrs bb, int has_b, int nl,
                                              const Prime *__restrict__ primes, int logN) {
    const int limb = blockIdx.y % nl, poly = blockIdx.y / nl, b = blockIdx.z;
    const size_t N = size_t(1) << logN;
    const Prime P = primes[limb];
    const size_t off = (size_t(poly) * nl + limb) * N;
    const uint64_t *al = a.p[b] + off;
    const uint64_t *bl = has_b ? bb.p[b] + off : nullptr;
    uint64_t *ol = out.p[b] + off;
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

}  // namespace

int gather(const Ptrs &src, size_t src_off, uint64_t *dst, size_t dst_bs, size_t words, int nb, hipStream_t s) {
    if (nb <= 0) return CKC_OK;
    CKC_PROF(PK_COPY, s, 16.0 * double(words) * nb, 0.0);
    hipLaunchKernelGGL(k_gather, dim3(unsigned(std::min<size_t>((words + 255) / 256, 1024)), unsigned(nb)), dim3(256),
                       0, s, src, src_off, dst, dst_bs, words);
    CKC_HIP(hipGetLastError());
    return CKC_OK;
}

namespace {
// ModUp of nb inputs, read contiguously (x + b xs) or through a pointer
// table (xp->p[b] + x_off)
int ks_modup_impl(ckc_ctx *c, const uint64_t *x, size_t xs, const Ptrs *xp, size_t x_off, int nb, int level,
                  uint64_t *digits, hipStream_t s) {
    const size_t N = c->N;
    const int nl = level + 1, dnum = c->dnum_at(level);
    CKC_REQUIRE(dnum <= kMaxDnum, CKC_EUNSUPPORTED, "too many key-switching digits");
    int rc = CKC_OK;
    const uint64_t *scale = modup_scale(c, level, &rc);
    if (!scale) return rc;
    // coefficient form, already multiplied by each limb's (D_j / q_i)^-1
    DevBuf coeff;
    CKC_TRY(coeff.alloc(8 * N * nl * nb, s));
    if (xp)
        CKC_TRY(ntt_inverse_ptrs(c, coeff.u64(), nl, qmap(), nb, size_t(nl) * N, s, scale, *xp, x_off));
    else
        CKC_TRY(ntt_inverse(c, coeff.u64(), nl, qmap(), nb, size_t(nl) * N, s, scale, x, xs));
    // digit j: its own limbs are those of x; every other limb of Q u P is the
    // conversion of the digit, transformed (all digits in one launch pair)
    const BconvTable *tabs[kMaxDnum];
    for (int j = 0; j < dnum; ++j) {
        tabs[j] = modup_table(c, level, j, &rc);
        if (!tabs[j]) return rc;
    }
    return ntt_modup(c, digits, level, nb, coeff.u64(), size_t(nl) * N, x, xs, tabs, s, xp, x_off);
}
}  // namespace

int ks_modup_b(ckc_ctx *c, const uint64_t *x, size_t xs, int nb, int level, uint64_t *digits, hipStream_t s) {
    return ks_modup_impl(c, x, xs, nullptr, 0, nb, level, digits, s);
}

int ks_modup_p(ckc_ctx *c, const Ptrs &xp, size_t x_off, int nb, int level, uint64_t *digits, hipStream_t s) {
    return ks_modup_impl(c, nullptr, 0, &xp, x_off, nb, level, digits, s);
}

int ks_apply_b(ckc_ctx *c, const uint64_t *digits, int nb, int level, const uint64_t *key, uint64_t g,
               const Ptrs *add0, const Ptrs *add1, bool perm_add0, const Ptrs &out0, const Ptrs &out1,
               hipStream_t s) {
    const size_t N = c->N;
    const int nl = level + 1, np = c->np, nt = nl + np, dnum = c->dnum_at(level);
    const uint32_t *perm = nullptr, *scat = nullptr;
    if (g != 1) {
        int rc;
        perm = (const uint32_t *)galois_table(c, g, &rc);
        if (!perm) return rc;
        scat = (const uint32_t *)galois_table(c, galois_inverse(c, g), &rc);
        if (!scat) return rc;
    }
    DevBuf acc, pl, conv;
    CKC_TRY(acc.alloc(8 * N * nl * 2 * nb, s));
    CKC_TRY(pl.alloc(8 * N * np * 2 * nb, s));
    CKC_TRY(conv.alloc(8 * N * nl * 2 * nb, s));
    const LimbMap ext{nl, c->nq};
    {
        // algorithmic bytes: every digit word, every key word and every output word once
        const double bytes = 8.0 * N * nt * (double(nb) * dnum + 2.0 * dnum + 2.0 * nb);
        CKC_PROF(PK_KIP, s, bytes, 2.0 * N * nt * dnum * nb);
        count_variant("kip_b", dnum <= 8 ? dnum : 0);
        hipLaunchKernelGGL(kip_kernel(dnum), dim3(unsigned(N / 256), unsigned(nt)), dim3(256), 0, s, digits, nb, dnum,
                           nt, nl, key, c->nprimes(), ext, scat, acc.u64(), pl.u64(), c->dprimes(), c->logN);
    }
    CKC_HIP(hipGetLastError());
    // ModDown: P limbs of every output (2 nb of them) to coefficient form,
    // pre-scaled by (P/p_k)^-1; their conversion to Q feeds the forward NTT,
    // whose last pass forms (acc - conversion) P^-1 + addend
    const LimbMap pmap{0, c->nq};
    CKC_TRY(ntt_inverse(c, pl.u64(), np, pmap, 2 * nb, size_t(np) * N, s, c->p_to_q.iscale.u64()));
    Ptrs none{};
    const BconvIn in{pl.u64(), size_t(np) * N, np, c->p_to_q.hat.u64(), c->p_to_q.neg_s.u64(),
                     c->p_to_q.s_half.u64(), nullptr, 0, -1, -1};
    const CombineOut co{acc.u64(), size_t(nl) * N, c->pinv.u64(), add0 ? *add0 : none, add1 ? *add1 : none, out0,
                        out1, add0 ? 1 : 0, add1 ? 1 : 0, perm_add0 ? perm : nullptr};
    CKC_TRY(ntt_forward_ex(c, conv.u64(), nl, qmap(), 2 * nb, size_t(nl) * N, s, -1, -1, &in, &co));
    return CKC_OK;
}

int rescale_b(ckc_ctx *c, const Ptrs &in, const Ptrs &out, int nb, int npoly, int level, hipStream_t s) {
    const size_t N = c->N;
    const int nl = level + 1, nbp = nb * npoly;
    DevBuf top, lift;
    CKC_TRY(top.alloc(8 * N * nbp, s));
    CKC_TRY(lift.alloc(8 * N * nbp * level, s));
    // gather the top limb of every polynomial: [b][p]
    for (int p = 0; p < npoly; ++p)
        CKC_TRY(gather(in, (size_t(p) * nl + level) * N, top.u64() + size_t(p) * N, size_t(npoly) * N, N, nb, s));
    const LimbMap one{0, level};
    CKC_TRY(ntt_inverse(c, top.u64(), 1, one, nbp, N, s));
    {
        CKC_PROF(PK_RESCALE, s, 8.0 * N * nbp * (1.0 + level), 0.0);
        hipLaunchKernelGGL(k_rescale_lift_b, dim3(tiles(N), unsigned(level), unsigned(nbp)), dim3(256), 0, s,
                           top.u64(), npoly, lift.u64(), level, c->dprimes(), c->logN);
    }
    CKC_HIP(hipGetLastError());
    CKC_TRY(ntt_forward(c, lift.u64(), level, qmap(), nbp, size_t(level) * N, s));
    {
        CKC_PROF(PK_RESCALE, s, 8.0 * N * nbp * 3.0 * level, 0.0);
        hipLaunchKernelGGL(k_rescale_combine_b, dim3(tiles(N), unsigned(level), unsigned(nbp)), dim3(256), 0, s, in,
                           npoly, lift.u64(), out, level, c->rescale_inv.u64(), c->dprimes(), c->logN, c->nq);
    }
    CKC_HIP(hipGetLastError());
    return CKC_OK;
}

int ew_b(ckc_ctx *c, EwOp op, const Ptrs &out, const Ptrs &a, const Ptrs *b, int nb, int npoly, int nl,
         hipStream_t s) {
    if (nb <= 0) return CKC_OK;
    Ptrs none{};
    CKC_PROF(PK_EW, s, 8.0 * c->N * nl * npoly * nb * (b ? 3.0 : 2.0), 0.0);
    hipLaunchKernelGGL(k_ew_b, dim3(tiles(c->N), unsigned(nl * npoly), unsigned(nb)), dim3(256), 0, s, int(op), out, a,
                       b ? *b : none, b ? 1 : 0, nl, c->dprimes(), c->logN);
    CKC_HIP(hipGetLastError());
    return CKC_OK;
}

// Hoisted rotations of nb inputs (pointer table) for every nonzero step;
// results to dst(b, step index) pointers.  The identity step is a copy.
int hoisted_group(ckc_ctx *c, const ckc_evk *evk, const Ptrs &in, int nb, int level, const std::vector<int32_t> &steps,
                  const std::vector<Ptrs> &dst, hipStream_t s) {
    const size_t N = c->N;
    const int nl = level + 1, nt = nl + c->np, dnum = c->dnum_at(level);
    const size_t pw = size_t(nl) * N;
    bool any = false;
    for (int32_t st : steps) any |= galois_element(c, st) != 1;
    DevBuf digits;
    if (any) {
        // ModUp of every input's c1, read in place
        CKC_TRY(digits.alloc(8 * N * nt * dnum * nb, s));
        CKC_TRY(ks_modup_p(c, in, pw, nb, level, digits.u64(), s));
    }
    for (size_t si = 0; si < steps.size(); ++si) {
        const uint64_t g = galois_element(c, steps[si]);
        if (g == 1) {
            CKC_PROF(PK_COPY, s, 16.0 * 2 * pw * nb, 0.0);
            hipLaunchKernelGGL(k_copy_pp, dim3(1024, unsigned(nb)), dim3(256), 0, s, in, dst[si], 2 * pw);
            CKC_HIP(hipGetLastError());
            continue;
        }
        auto it = evk->galois.find(g);
        CKC_REQUIRE(it != evk->galois.end(), CKC_ENOKEY, "missing Galois key for step " + std::to_string(steps[si]));
        Ptrs o1;
        for (int b = 0; b < nb; ++b) o1.p[b] = dst[si].p[b] + pw;
        CKC_TRY(ks_apply_b(c, digits.u64(), nb, level, it->second->u64(), g, &in, nullptr, true, dst[si], o1, s));
    }
    return CKC_OK;
}

int hoisted_group_ext(ckc_ctx *c, const ckc_evk *evk, const Ptrs &in, int nb, int level,
                      const std::vector<int32_t> &steps, const std::vector<Ptrs> &dst, hipStream_t s) {
    const size_t N = c->N;
    const int nl = level + 1, np = c->np, nt = nl + np, dnum = c->dnum_at(level);
    const size_t pw = size_t(nl) * N;
    bool any = false;
    for (int32_t st : steps) any |= galois_element(c, st) != 1;
    DevBuf digits;
    if (any) {
        // ModUp of every input's c1, read in place
        CKC_TRY(digits.alloc(8 * N * nt * dnum * nb, s));
        CKC_TRY(ks_modup_p(c, in, pw, nb, level, digits.u64(), s));
    }
    const LimbMap ext{nl, c->nq};
    // rotations whose outputs sit at one offset from the first step's for
    // every input (the convolution's layout) share one launch
    std::vector<size_t> fused;
    const bool tiles8 = ((N >> 8) * size_t(nt)) % 8 == 0 && (N >> 8) > 0;
    for (size_t si = 0; si < steps.size(); ++si) {
        if (galois_element(c, steps[si]) == 1 || !tiles8 || fused.size() == size_t(kMaxRot)) continue;
        const ptrdiff_t d0 = dst[si].p[0] - dst[0].p[0];
        bool same = true;
        for (int b = 1; b < nb && same; ++b) same = dst[si].p[b] - dst[0].p[b] == d0;
        if (same) fused.push_back(si);
    }
    if (fused.size() < 2) fused.clear();
    if (!fused.empty()) {
        KipRot kr{};
        for (size_t r = 0; r < fused.size(); ++r) {
            const uint64_t g = galois_element(c, steps[fused[r]]);
            auto it = evk->galois.find(g);
            CKC_REQUIRE(it != evk->galois.end(), CKC_ENOKEY,
                        "missing Galois key for step " + std::to_string(steps[fused[r]]));
            int rc;
            kr.scat[r] = (const uint32_t *)galois_table(c, galois_inverse(c, g), &rc);
            if (!kr.scat[r]) return rc;
            kr.key[r] = it->second->u64();
            kr.off[r] = int64_t(dst[fused[r]].p[0] - dst[0].p[0]);
        }
        const int nrot = int(fused.size());
        // algorithmic bytes: digits once, every key, c0 (Q limbs) and both
        // outputs of every rotation once
        const double bytes =
            8.0 * N * (nt * (double(nb) * dnum + nrot * (2.0 * dnum + 2.0 * nb)) + double(nb) * nl);
        CKC_PROF(PK_KIP, s, bytes, 2.0 * N * nt * dnum * nb * nrot);
        const unsigned blocks = unsigned((N >> 8) * size_t(nt) * size_t(nrot));
        count_variant("kip_ext_rot", dnum <= 8 ? dnum : 0);
        hipLaunchKernelGGL(kip_rot_kernel(dnum), dim3(blocks), dim3(256), 0, s, digits.u64(), nb, dnum, nt, nl, nrot,
                           kr, c->nprimes(), ext, in, dst[0], c->pmod.u64(), c->dprimes(), c->logN);
        CKC_HIP(hipGetLastError());
    }
    for (size_t si = 0; si < steps.size(); ++si) {
        if (std::find(fused.begin(), fused.end(), si) != fused.end()) continue;
        const uint64_t g = galois_element(c, steps[si]);
        if (g == 1) {
            CKC_PROF(PK_EW, s, 8.0 * N * nb * 2 * (nl + nt), 0.0);
            hipLaunchKernelGGL(k_lift_P, dim3(tiles(N), unsigned(nt), unsigned(2 * nb)), dim3(256), 0, s, in, dst[si],
                               nl, nt, c->pmod.u64(), c->dprimes(), c->logN);
            CKC_HIP(hipGetLastError());
            continue;
        }
        auto it = evk->galois.find(g);
        CKC_REQUIRE(it != evk->galois.end(), CKC_ENOKEY, "missing Galois key for step " + std::to_string(steps[si]));
        int rc;
        const uint32_t *scat = (const uint32_t *)galois_table(c, galois_inverse(c, g), &rc);
        if (!scat) return rc;
        {
            // algorithmic bytes: digits, key, c0 (Q limbs) and both outputs once
            const double bytes = 8.0 * N * (nt * (double(nb) * dnum + 2.0 * dnum + 2.0 * nb) + double(nb) * nl);
            CKC_PROF(PK_KIP, s, bytes, 2.0 * N * nt * dnum * nb);
            count_variant("kip_ext", dnum <= 8 ? dnum : 0);
            hipLaunchKernelGGL(kip_ext_kernel(dnum), dim3(unsigned(N / 256), unsigned(nt)), dim3(256), 0, s,
                               digits.u64(), nb, dnum, nt, nl, it->second->u64(), c->nprimes(), ext, scat, in,
                               dst[si], c->pmod.u64(), c->dprimes(), c->logN);
        }
        CKC_HIP(hipGetLastError());
    }
    return CKC_OK;
}

int moddown_b(ckc_ctx *c, const uint64_t *y, int n, int level, const Ptrs *add0, const Ptrs &out0, const Ptrs &out1,
              hipStream_t s) {
    if (n <= 0) return CKC_OK;
    CKC_REQUIRE(n <= kMaxBatch, CKC_EINVAL, "moddown_b: at most 64 ciphertexts per call");
    const size_t N = c->N;
    const int nl = level + 1, np = c->np, nt = nl + np;
    DevBuf pl, conv;
    CKC_TRY(pl.alloc(8 * N * np * 2 * n, s));
    CKC_TRY(conv.alloc(8 * N * nl * 2 * n, s));
    const LimbMap pmap{0, c->nq};
    // P limbs of every polynomial -> coefficient form, scaled by (P/p_k)^-1
    CKC_TRY(ntt_inverse(c, pl.u64(), np, pmap, 2 * n, size_t(np) * N, s, c->p_to_q.iscale.u64(), y + size_t(nl) * N,
                        size_t(nt) * N));
    Ptrs none{};
    const BconvIn in{pl.u64(), size_t(np) * N, np, c->p_to_q.hat.u64(), c->p_to_q.neg_s.u64(),
                     c->p_to_q.s_half.u64(), nullptr, 0, -1, -1};
    const CombineOut co{y, size_t(nt) * N, c->pinv.u64(), add0 ? *add0 : none, none, out0, out1, add0 ? 1 : 0, 0,
                        nullptr};
    return ntt_forward_ex(c, conv.u64(), nl, qmap(), 2 * n, size_t(nl) * N, s, -1, -1, &in, &co);
}
