// Client-side kernels: encoding FFT (FP64), decoding, counter-based sampling,
// key generation, encryption and decryption.
//
// Encoding (Section 2.2): the N/2 slots sit at the roots zeta^(5^j),
// zeta = e^(i pi/N).  Writing 5^j mod 2N = 1 + 4 t_j, slot values are the
// length-n (n = N/2) DFT of w_k zeta^k read at index t_j, where the plaintext
// polynomial has m_k = Re w_k and m_{k+n} = Im w_k.  Encoding scatters the
// slots to y[t_j], runs an unnormalised inverse DFT (iterative radix-2
// decimation in time, bit-reversed input), twists by zeta^-k / n, scales by
// Delta and rounds half away from zero.  The FFT has one fixed operation order,
// is compiled without FMA contraction, and its twiddle tables come from a
// fixed series evaluation (not libm), so the rounded integers are a
// deterministic function of the slots.
#include <math.h>

#include <algorithm>

#include "ckc_internal.h"

namespace {

// ---------------------------------------------------------------- PRNG
constexpr uint64_t kGamma = 0x9e3779b97f4a7c15ull;
enum { TAG_SECRET = 1, TAG_KEY_A = 2, TAG_KEY_E = 3, TAG_ENC_A = 4, TAG_ENC_E = 5 };

CKC_HD uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}
// SplitMix64 (Steele, Lea, Flood 2014): stream key, then draw j = mix(key + (j+1) gamma)
uint64_t stream_key(uint64_t seed, uint64_t tag, uint64_t idx) { return mix64(mix64(seed + tag * kGamma) + idx * kGamma); }
__device__ __forceinline__ uint64_t draw(uint64_t key, uint64_t j) { return mix64(key + (j + 1) * kGamma); }
__device__ __forceinline__ int cbd21(uint64_t u) {
    return __popcll(u & 0x1fffffull) - __popcll((u >> 21) & 0x1fffffull);
}
__device__ __forceinline__ uint64_t from_small(int v, uint64_t q) { return v >= 0 ? uint64_t(v) : q - uint64_t(-v); }

// uniform residues: out[t][k] = floor(draw(key, prime(t) N + k) * q / 2^64)
__global__ void k_sample_uniform(uint64_t *__restrict__ out, int nlimbs, LimbMap map, uint64_t key,
                                 const Prime *__restrict__ primes, int logN) {
    const int t = blockIdx.y;
    const size_t N = size_t(1) << logN;
    const int pi = map.prime(t);
    const uint64_t q = primes[pi].q;
    for (size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x; k < N; k += size_t(gridDim.x) * blockDim.x)
        out[size_t(t) * N + k] = mulhi64(draw(key, uint64_t(pi) * N + k), q);
}

// centred binomial (eta = 21), one draw per coefficient, residues per limb
__global__ void k_sample_cbd(uint64_t *__restrict__ out, int nlimbs, LimbMap map, uint64_t key,
                             const Prime *__restrict__ primes, int logN) {
    const int t = blockIdx.y;
    const size_t N = size_t(1) << logN;
    const uint64_t q = primes[map.prime(t)].q;
    for (size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x; k < N; k += size_t(gridDim.x) * blockDim.x)
        out[size_t(t) * N + k] = from_small(cbd21(draw(key, k)), q);
}

// ternary secret: s_k = {0, 1, -1}[floor(3 u / 2^64)]
__global__ void k_sample_ternary(int8_t *__restrict__ s, uint64_t key, int logN) {
    const size_t N = size_t(1) << logN;
    for (size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x; k < N; k += size_t(gridDim.x) * blockDim.x) {
        const int t = int(mulhi64(draw(key, k), 3));
        s[k] = int8_t(t == 2 ? -1 : t);
    }
}

__global__ void k_small_to_limbs(const int8_t *__restrict__ s, uint64_t *__restrict__ out, int nlimbs, LimbMap map,
                                 const Prime *__restrict__ primes, int logN) {
    const int t = blockIdx.y;
    const size_t N = size_t(1) << logN;
    const uint64_t q = primes[map.prime(t)].q;
    for (size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x; k < N; k += size_t(gridDim.x) * blockDim.x)
        out[size_t(t) * N + k] = from_small(s[k], q);
}

// key row: b = -a s + e + [t in digit] (P mod q_t) s'   (NTT form, all primes)
__global__ void k_keygen_combine(uint64_t *__restrict__ b, const uint64_t *__restrict__ a,
                                 const uint64_t *__restrict__ e, const uint64_t *__restrict__ s,
                                 const uint64_t *__restrict__ sp, const uint64_t *__restrict__ pmod, int dlo,
                                 int dhi, const Prime *__restrict__ primes, int logN) {
    const int t = blockIdx.y;
    const size_t N = size_t(1) << logN;
    const Prime P = primes[t];
    const bool in_digit = t >= dlo && t < dhi;
    const uint64_t pm = pmod[t];
    for (size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x; k < N; k += size_t(gridDim.x) * blockDim.x) {
        const size_t i = size_t(t) * N + k;
        uint64_t r = sub_mod(e[i], mul_mod(a[i], s[i], P), P.q);
        if (in_digit) r = add_mod(r, mul_mod(pm, sp[i], P), P.q);
        b[i] = r;
    }
}

// evaluation keys are kept times 2^64 mod q (Montgomery form): the key inner
// products end in one Montgomery reduction per output instead of a 128-bit
// reduction (x -> x 2^64 mod q is a Shoup product by r2 = 2^64 mod q)
__global__ void k_to_montgomery(uint64_t *__restrict__ x, int nlimbs_per_row, const Prime *__restrict__ primes,
                                int logN) {
    const size_t N = size_t(1) << logN;
    const int row = blockIdx.y;
    const Prime P = primes[row % nlimbs_per_row];
    uint64_t *r = x + size_t(row) * N;
    for (size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x; k < N; k += size_t(gridDim.x) * blockDim.x)
        r[k] = mul_shoup(r[k], P.r2, P.r2p, P.q);
}

// c0 = m - a s + e over the Q limbs (NTT form)
__global__ void k_encrypt_combine(uint64_t *__restrict__ c0, const uint64_t *__restrict__ m,
                                  const uint64_t *__restrict__ a, const uint64_t *__restrict__ e,
                                  const uint64_t *__restrict__ s, const Prime *__restrict__ primes, int logN) {
    const int t = blockIdx.y;
    const size_t N = size_t(1) << logN;
    const Prime P = primes[t];
    for (size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x; k < N; k += size_t(gridDim.x) * blockDim.x) {
        const size_t i = size_t(t) * N + k;
        c0[i] = add_mod(sub_mod(m[i], mul_mod(a[i], s[i], P), P.q), e[i], P.q);
    }
}

// m = c0 + c1 s (+ c2 s^2)
__global__ void k_decrypt(uint64_t *__restrict__ m, const uint64_t *__restrict__ ct, int nl, int npoly,
                          const uint64_t *__restrict__ s, const Prime *__restrict__ primes, int logN) {
    const int t = blockIdx.y;
    const size_t N = size_t(1) << logN;
    const Prime P = primes[t];
    for (size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x; k < N; k += size_t(gridDim.x) * blockDim.x) {
        const size_t i = size_t(t) * N + k;
        const uint64_t sv = s[i];
        uint64_t r = add_mod(ct[i], mul_mod(ct[size_t(nl) * N + i], sv, P), P.q);
        if (npoly == 3) r = add_mod(r, mul_mod(mul_mod(ct[size_t(2 * nl) * N + i], sv, P), sv, P), P.q);
        m[i] = r;
    }
}

// ---------------------------------------------------------------- FFT (FP64)
#pragma clang fp contract(off)

__global__ void k_fft_scatter(const double *__restrict__ z, size_t nslots, const uint32_t *__restrict__ idx,
                              double2 *__restrict__ y, size_t n) {
    for (size_t j = size_t(blockIdx.x) * blockDim.x + threadIdx.x; j < n; j += size_t(gridDim.x) * blockDim.x)
        if (j < nslots) y[idx[j]] = make_double2(z[j], 0.0);
}

__global__ void k_bitrev(const double2 *__restrict__ in, double2 *__restrict__ out, int logn) {
    const size_t n = size_t(1) << logn;
    for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x) {
        const uint32_t r = __brev(uint32_t(i)) >> (32 - logn);
        out[r] = in[i];
    }
}

// one radix-2 DIT stage of length `len`: twiddle exponent e = j * (n / len)
__global__ void k_fft_stage(double2 *__restrict__ a, const double2 *__restrict__ w, size_t n, size_t len,
                            int inverse) {
    const size_t half = len >> 1, step = n / len;
    for (size_t b = size_t(blockIdx.x) * blockDim.x + threadIdx.x; b < n / 2; b += size_t(gridDim.x) * blockDim.x) {
        const size_t i = (b / half) * len, j = b % half;
        const double2 tw = w[j * step];
        const double wr = tw.x, wi = inverse ? -tw.y : tw.y;
        const double2 x = a[i + j + half];
        const double vr = x.x * wr - x.y * wi;
        const double vi = x.x * wi + x.y * wr;
        const double2 u = a[i + j];
        a[i + j] = make_double2(u.x + vr, u.y + vi);
        a[i + j + half] = make_double2(u.x - vr, u.y - vi);
    }
}

// exact residue of an integer-valued double modulo q
__device__ uint64_t dint_mod(double v, const Prime &P) {
    const double av = fabs(v);
    uint64_t r;
    if (av < 9.2e18) {
        r = reduce64(uint64_t(av), P);
    } else {
        int e;
        const double mant = frexp(av, &e);
        const uint64_t M = uint64_t(ldexp(mant, 53));
        uint64_t pw = 1, base = 2 % P.q;
        unsigned ex = unsigned(e - 53);
        while (ex) {
            if (ex & 1) pw = mul_mod(pw, base, P);
            base = mul_mod(base, base, P);
            ex >>= 1;
        }
        r = mul_mod(reduce64(M, P), pw, P);
    }
    return v < 0 ? neg_mod(r, P.q) : r;
}

// twist by (cos, -sin)(pi k / N) / n, scale, round, reduce into every limb
__global__ void k_encode_finish(const double2 *__restrict__ Y, const double2 *__restrict__ twist, double delta,
                                uint64_t *__restrict__ m, int nl, LimbMap map, const Prime *__restrict__ primes,
                                int logN) {
    const size_t N = size_t(1) << logN, n = N / 2;
    const double inv_n = 1.0 / double(n);
    for (size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x; k < n; k += size_t(gridDim.x) * blockDim.x) {
        const double2 tw = twist[k];
        const double tr = tw.x * inv_n, ti = -tw.y * inv_n;
        const double2 y = Y[k];
        const double wr = y.x * tr - y.y * ti;
        const double wi = y.x * ti + y.y * tr;
        const double a = round(delta * wr), b = round(delta * wi);
        for (int t = 0; t < nl; ++t) {
            const Prime P = primes[map.prime(t)];
            m[size_t(t) * N + k] = dint_mod(a, P);
            m[size_t(t) * N + k + n] = dint_mod(b, P);
        }
    }
}

// decode start: centred lift of the q_0 limb, twist by zeta^k
__global__ void k_decode_start(const uint64_t *__restrict__ m0, const double2 *__restrict__ twist,
                               double2 *__restrict__ c, uint64_t q0, int logN) {
    const size_t N = size_t(1) << logN, n = N / 2;
    const uint64_t half = q0 >> 1;
    for (size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x; k < n; k += size_t(gridDim.x) * blockDim.x) {
        const uint64_t x = m0[k], y = m0[k + n];
        const double ar = x > half ? -double(q0 - x) : double(x);
        const double ai = y > half ? -double(q0 - y) : double(y);
        const double2 tw = twist[k];
        c[k] = make_double2(ar * tw.x - ai * tw.y, ar * tw.y + ai * tw.x);
    }
}

__global__ void k_decode_gather(const double2 *__restrict__ Z, const uint32_t *__restrict__ idx, double scale,
                                double *__restrict__ out, size_t nslots) {
    for (size_t j = size_t(blockIdx.x) * blockDim.x + threadIdx.x; j < nslots; j += size_t(gridDim.x) * blockDim.x)
        out[j] = Z[idx[j]].x / scale;
}

#pragma clang fp contract(on)

unsigned tiles(size_t work) { return unsigned(std::max<size_t>(1, std::min<size_t>((work + 255) / 256, 1024))); }

int fft_run(const ckc_ctx *c, double2 *buf, double2 *tmp, int inverse, hipStream_t s) {
    const int logn = c->logN - 1;
    const size_t n = size_t(1) << logn;
    hipLaunchKernelGGL(k_bitrev, dim3(tiles(n)), dim3(256), 0, s, buf, tmp, logn);
    for (size_t len = 2; len <= n; len <<= 1)
        hipLaunchKernelGGL(k_fft_stage, dim3(tiles(n / 2)), dim3(256), 0, s, tmp, (const double2 *)c->fft_w.p, n,
                           len, inverse);
    CKC_HIP(hipGetLastError());
    return CKC_OK;
}

}  // namespace

int copy_limbs(const uint64_t *src, size_t src_ps, uint64_t *dst, size_t dst_ps, size_t words, int npoly,
               hipStream_t s);

// ---------------------------------------------------------------- encode / decode
int encode_impl(ckc_ctx *c, const double *slots_h, size_t nslots, int level, double scale, uint64_t *m,
                hipStream_t s, bool ext) {
    const size_t N = c->N, n = N / 2;
    DevBuf zb, yb, tb;
    CKC_TRY(zb.alloc(8 * std::max<size_t>(nslots, 1), s));
    CKC_TRY(yb.alloc(16 * n, s));
    CKC_TRY(tb.alloc(16 * n, s));
    if (nslots) CKC_HIP(hipMemcpyAsync(zb.p, slots_h, 8 * nslots, hipMemcpyHostToDevice, s));
    CKC_HIP(hipMemsetAsync(yb.p, 0, 16 * n, s));
    hipLaunchKernelGGL(k_fft_scatter, dim3(tiles(n)), dim3(256), 0, s, (const double *)zb.p, nslots,
                       (const uint32_t *)c->slot_idx.p, (double2 *)yb.p, n);
    CKC_TRY(fft_run(c, (double2 *)yb.p, (double2 *)tb.p, 1, s));
    // the integer coefficients reduced into q_0..q_level (and, for ext, every P prime)
    const int nlimbs = level + 1 + (ext ? c->np : 0);
    const LimbMap map = ext ? LimbMap{level + 1, c->nq} : qmap();
    hipLaunchKernelGGL(k_encode_finish, dim3(tiles(n)), dim3(256), 0, s, (const double2 *)tb.p,
                       (const double2 *)c->twist.p, scale, m, nlimbs, map, c->dprimes(), c->logN);
    CKC_HIP(hipGetLastError());
    CKC_TRY(ntt_forward(c, m, nlimbs, map, 1, 0, s));
    // the host array must stay valid until the copy ran
    CKC_HIP(hipStreamSynchronize(s));
    return CKC_OK;
}

int decode_impl(ckc_ctx *c, const uint64_t *m, double scale, double *out_h, size_t nslots, hipStream_t s) {
    const size_t N = c->N, n = N / 2;
    DevBuf lb, cb, tb, ob;
    CKC_TRY(lb.alloc(8 * N, s));
    CKC_TRY(cb.alloc(16 * n, s));
    CKC_TRY(tb.alloc(16 * n, s));
    CKC_TRY(ob.alloc(8 * std::max<size_t>(nslots, 1), s));
    CKC_TRY(copy_limbs(m, 0, lb.u64(), 0, N, 1, s));
    CKC_TRY(ntt_inverse(c, lb.u64(), 1, qmap(), 1, 0, s));
    hipLaunchKernelGGL(k_decode_start, dim3(tiles(n)), dim3(256), 0, s, lb.u64(), (const double2 *)c->twist.p,
                       (double2 *)cb.p, c->mods[0], c->logN);
    CKC_TRY(fft_run(c, (double2 *)cb.p, (double2 *)tb.p, 0, s));
    hipLaunchKernelGGL(k_decode_gather, dim3(tiles(nslots)), dim3(256), 0, s, (const double2 *)tb.p,
                       (const uint32_t *)c->slot_idx.p, scale, (double *)ob.p, nslots);
    CKC_HIP(hipGetLastError());
    if (nslots) CKC_HIP(hipMemcpyAsync(out_h, ob.p, 8 * nslots, hipMemcpyDeviceToHost, s));
    CKC_HIP(hipStreamSynchronize(s));
    return CKC_OK;
}

// ---------------------------------------------------------------- keys
int secret_impl(ckc_ctx *c, ckc_sk *sk, uint64_t seed, hipStream_t s) {
    const size_t N = c->N;
    const int np = c->nprimes();
    DevBuf sb;
    CKC_TRY(sb.alloc(N, s));
    hipLaunchKernelGGL(k_sample_ternary, dim3(tiles(N)), dim3(256), 0, s, (int8_t *)sb.p,
                       stream_key(seed, TAG_SECRET, 0), c->logN);
    CKC_TRY(sk->s_ntt.alloc(8 * N * np));
    hipLaunchKernelGGL(k_small_to_limbs, dim3(tiles(N), unsigned(np)), dim3(256), 0, s, (const int8_t *)sb.p,
                       sk->s_ntt.u64(), np, qmap(), c->dprimes(), c->logN);
    CKC_HIP(hipGetLastError());
    sk->s.resize(N);
    CKC_HIP(hipMemcpyAsync(sk->s.data(), sb.p, N, hipMemcpyDeviceToHost, s));
    CKC_TRY(ntt_forward(c, sk->s_ntt.u64(), np, qmap(), 1, 0, s));
    CKC_HIP(hipStreamSynchronize(s));
    sk->seed = seed;
    return CKC_OK;
}

// key[j][2][nprimes][N] switching s' (NTT form, every prime) -> s, stored
// times 2^64 mod q
int switch_key_impl(ckc_ctx *c, const ckc_sk *sk, uint64_t key_id, const uint64_t *sprime, uint64_t *key,
                    hipStream_t s) {
    const size_t N = c->N;
    const int np = c->nprimes();
    const int dnum = c->dnum_at(c->nq - 1);
    std::vector<uint64_t> pmod(np);
    for (int t = 0; t < np; ++t) {
        const uint64_t q = c->mods[t];
        uint64_t pm = 1 % q;
        for (int i = 0; i < c->np; ++i) pm = (uint64_t)(((unsigned __int128)pm * (c->mods[c->nq + i] % q)) % q);
        pmod[t] = pm;
    }
    DevBuf pmd, eb;
    CKC_TRY(pmd.alloc(8 * np, s));
    CKC_TRY(eb.alloc(8 * N * np, s));
    CKC_HIP(hipMemcpyAsync(pmd.p, pmod.data(), 8 * np, hipMemcpyHostToDevice, s));
    for (int j = 0; j < dnum; ++j) {
        uint64_t *b = key + (size_t(j) * 2 + 0) * np * N;
        uint64_t *a = key + (size_t(j) * 2 + 1) * np * N;
        hipLaunchKernelGGL(k_sample_uniform, dim3(tiles(N), unsigned(np)), dim3(256), 0, s, a, np, qmap(),
                           stream_key(sk->seed, TAG_KEY_A, key_id * 64 + uint64_t(j)), c->dprimes(), c->logN);
        hipLaunchKernelGGL(k_sample_cbd, dim3(tiles(N), unsigned(np)), dim3(256), 0, s, eb.u64(), np, qmap(),
                           stream_key(sk->seed, TAG_KEY_E, key_id * 64 + uint64_t(j)), c->dprimes(), c->logN);
        CKC_HIP(hipGetLastError());
        CKC_TRY(ntt_forward(c, a, np, qmap(), 1, 0, s));
        CKC_TRY(ntt_forward(c, eb.u64(), np, qmap(), 1, 0, s));
        const int dlo = j * c->alpha, dhi = std::min(dlo + c->alpha, c->nq);
        hipLaunchKernelGGL(k_keygen_combine, dim3(tiles(N), unsigned(np)), dim3(256), 0, s, b, a, eb.u64(),
                           sk->s_ntt.u64(), sprime, (const uint64_t *)pmd.p, dlo, dhi, c->dprimes(), c->logN);
        CKC_HIP(hipGetLastError());
    }
    // rows [dnum][2][np], row r over prime r mod np
    hipLaunchKernelGGL(k_to_montgomery, dim3(tiles(N), unsigned(dnum * 2 * np)), dim3(256), 0, s, key, np,
                       c->dprimes(), c->logN);
    CKC_HIP(hipGetLastError());
    CKC_HIP(hipStreamSynchronize(s));
    return CKC_OK;
}

int encrypt_impl(ckc_ctx *c, const ckc_sk *sk, const uint64_t *m, int level, uint64_t stream_id, uint64_t *ct,
                 hipStream_t s) {
    const size_t N = c->N;
    const int nl = level + 1;
    DevBuf eb, c0;
    CKC_TRY(eb.alloc(8 * N * nl, s));
    CKC_TRY(c0.alloc(8 * N * nl, s));
    uint64_t *c1 = ct + size_t(nl) * N;
    hipLaunchKernelGGL(k_sample_uniform, dim3(tiles(N), unsigned(nl)), dim3(256), 0, s, c1, nl, qmap(),
                       stream_key(sk->seed, TAG_ENC_A, stream_id), c->dprimes(), c->logN);
    hipLaunchKernelGGL(k_sample_cbd, dim3(tiles(N), unsigned(nl)), dim3(256), 0, s, eb.u64(), nl, qmap(),
                       stream_key(sk->seed, TAG_ENC_E, stream_id), c->dprimes(), c->logN);
    CKC_HIP(hipGetLastError());
    CKC_TRY(ntt_forward(c, c1, nl, qmap(), 1, 0, s));
    CKC_TRY(ntt_forward(c, eb.u64(), nl, qmap(), 1, 0, s));
    // m may alias ct[0]; build c0 in a temporary first
    hipLaunchKernelGGL(k_encrypt_combine, dim3(tiles(N), unsigned(nl)), dim3(256), 0, s, c0.u64(), m, c1, eb.u64(),
                       sk->s_ntt.u64(), c->dprimes(), c->logN);
    CKC_HIP(hipGetLastError());
    CKC_TRY(copy_limbs(c0.u64(), 0, ct, 0, N * nl, 1, s));
    return CKC_OK;
}

int decrypt_impl(ckc_ctx *c, const ckc_sk *sk, const uint64_t *ct, int level, int npoly, uint64_t *m,
                 hipStream_t s) {
    const size_t N = c->N;
    const int nl = level + 1;
    hipLaunchKernelGGL(k_decrypt, dim3(tiles(N), unsigned(nl)), dim3(256), 0, s, m, ct, nl, npoly, sk->s_ntt.u64(),
                       c->dprimes(), c->logN);
    CKC_HIP(hipGetLastError());
    return CKC_OK;
}
