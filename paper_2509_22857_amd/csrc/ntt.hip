// Negacyclic NTT / INTT over 64-bit RNS limbs for gfx950.
//
// Forward: merged-twiddle Cooley-Tukey (the psi twist folded into a
// bit-reversed table tw[k] = psi^bitrev(k)); natural-order input, output
// index k holds a(psi^(2 bitrev(k) + 1)).  Inverse: Gentleman-Sande with
// itw[k] = psi^-bitrev(k), then a multiply by N^-1.
//
// A limb of N = 2^logN words is split as N1 x N2 with N2 = 256: the stages
// whose butterfly distance is a multiple of N2 only mix words of one column
// (stride N2), the remaining log2(N2) stages only mix words inside one
// contiguous run of N2.  Each pass stages 4096 words (32 KiB) per workgroup
// through LDS and runs its stages there, so a transform reads and writes the
// limb twice.
#include "ckc_internal.h"
#include "prof.h"

namespace {

constexpr int kThreads = 256;
constexpr int kElems = 4096;
constexpr int kLogN2 = 8;
constexpr int kN2 = 1 << kLogN2;

// ---------------------------------------------------------------- columns
template <bool INVERSE>
__global__ __launch_bounds__(kThreads) void k_ntt_cols(uint64_t *__restrict__ data, size_t batch_stride,
                                                       LimbMap map, const Prime *__restrict__ primes,
                                                       const uint64_t *__restrict__ tw,
                                                       const uint64_t *__restrict__ twp,
                                                       const uint64_t *__restrict__ ninv, int logN,
                                                       int skip_lo, int skip_hi) {
    __shared__ uint64_t s[kElems];
    const int limb = blockIdx.y;
    if (limb >= skip_lo && limb < skip_hi) return;
    const int pi = map.prime(limb);
    const uint64_t q = primes[pi].q;
    const size_t N = size_t(1) << logN;
    uint64_t *a = data + size_t(blockIdx.z) * batch_stride + size_t(limb) * N;
    const int logN1 = logN - kLogN2;
    const int N1 = 1 << logN1;
    const int logC = 12 - logN1;  // columns per workgroup = kElems / N1
    const int C = 1 << logC;
    const int col0 = blockIdx.x * C;
    const uint64_t *W = tw + size_t(pi) * N;
    const uint64_t *Wp = twp + size_t(pi) * N;

    for (int e = threadIdx.x; e < kElems; e += kThreads) {
        const int c = e & (C - 1), r = e >> logC;
        s[e] = a[size_t(r) * kN2 + col0 + c];
    }
    __syncthreads();
    if (!INVERSE) {
        for (int m = 1; m < N1; m <<= 1) {
            const int tr = N1 / (2 * m);
            for (int b = threadIdx.x; b < kElems / 2; b += kThreads) {
                const int c = b & (C - 1), pr = b >> logC;
                const int i = pr / tr, r = i * 2 * tr + (pr - i * tr);
                const uint64_t w = W[m + i], wp = Wp[m + i];
                const int lo = (r << logC) + c, hi = ((r + tr) << logC) + c;
                const uint64_t U = s[lo];
                const uint64_t V = mul_shoup(s[hi], w, wp, q);
                s[lo] = add_mod(U, V, q);
                s[hi] = sub_mod(U, V, q);
            }
            __syncthreads();
        }
        for (int e = threadIdx.x; e < kElems; e += kThreads) {
            const int c = e & (C - 1), r = e >> logC;
            a[size_t(r) * kN2 + col0 + c] = s[e];
        }
    } else {
        for (int tr = 1; tr < N1; tr <<= 1) {
            const int h = N1 / (2 * tr);
            for (int b = threadIdx.x; b < kElems / 2; b += kThreads) {
                const int c = b & (C - 1), pr = b >> logC;
                const int i = pr / tr, r = i * 2 * tr + (pr - i * tr);
                const uint64_t w = W[h + i], wp = Wp[h + i];
                const int lo = (r << logC) + c, hi = ((r + tr) << logC) + c;
                const uint64_t U = s[lo], V = s[hi];
                s[lo] = add_mod(U, V, q);
                s[hi] = mul_shoup(sub_mod(U, V, q), w, wp, q);
            }
            __syncthreads();
        }
        const uint64_t ni = ninv[2 * pi], nip = ninv[2 * pi + 1];
        for (int e = threadIdx.x; e < kElems; e += kThreads) {
            const int c = e & (C - 1), r = e >> logC;
            a[size_t(r) * kN2 + col0 + c] = mul_shoup(s[e], ni, nip, q);
        }
    }
}

// ---------------------------------------------------------------- rows
template <bool INVERSE>
__global__ __launch_bounds__(kThreads) void k_ntt_rows(uint64_t *__restrict__ data, size_t batch_stride,
                                                       LimbMap map, const Prime *__restrict__ primes,
                                                       const uint64_t *__restrict__ tw,
                                                       const uint64_t *__restrict__ twp, int logN,
                                                       int skip_lo, int skip_hi) {
    __shared__ uint64_t s[kElems];
    const int limb = blockIdx.y;
    if (limb >= skip_lo && limb < skip_hi) return;
    const int pi = map.prime(limb);
    const uint64_t q = primes[pi].q;
    const size_t N = size_t(1) << logN;
    const size_t base = size_t(blockIdx.x) * kElems;
    uint64_t *a = data + size_t(blockIdx.z) * batch_stride + size_t(limb) * N + base;
    const uint64_t *W = tw + size_t(pi) * N;
    const uint64_t *Wp = twp + size_t(pi) * N;

    for (int e = threadIdx.x; e < kElems; e += kThreads) s[e] = a[e];
    __syncthreads();
    if (!INVERSE) {
        // stages m = N/N2 .. N/2, distance t = N/(2m) = N2/2 .. 1
        for (int t = kN2 / 2; t >= 1; t >>= 1) {
            const size_t m = N / (2 * size_t(t));
            for (int b = threadIdx.x; b < kElems / 2; b += kThreads) {
                const int il = b / t, off = b - il * t;
                const int lo = il * 2 * t + off, hi = lo + t;
                const size_t gi = (base / (2 * size_t(t))) + il;
                const uint64_t w = W[m + gi], wp = Wp[m + gi];
                const uint64_t U = s[lo];
                const uint64_t V = mul_shoup(s[hi], w, wp, q);
                s[lo] = add_mod(U, V, q);
                s[hi] = sub_mod(U, V, q);
            }
            __syncthreads();
        }
    } else {
        for (int t = 1; t < kN2; t <<= 1) {
            const size_t h = N / (2 * size_t(t));
            for (int b = threadIdx.x; b < kElems / 2; b += kThreads) {
                const int il = b / t, off = b - il * t;
                const int lo = il * 2 * t + off, hi = lo + t;
                const size_t gi = (base / (2 * size_t(t))) + il;
                const uint64_t w = W[h + gi], wp = Wp[h + gi];
                const uint64_t U = s[lo], V = s[hi];
                s[lo] = add_mod(U, V, q);
                s[hi] = mul_shoup(sub_mod(U, V, q), w, wp, q);
            }
            __syncthreads();
        }
    }
    for (int e = threadIdx.x; e < kElems; e += kThreads) a[e] = s[e];
}

}  // namespace

int ntt_forward(const ckc_ctx *c, uint64_t *d, int nlimbs, LimbMap map, int nbatch, size_t batch_stride,
                hipStream_t s, int skip_lo, int skip_hi) {
    if (nlimbs <= 0 || nbatch <= 0) return CKC_OK;
    CKC_REQUIRE(c->logN >= 12 && c->logN <= 17, CKC_EUNSUPPORTED, "NTT supports 2^12 <= N <= 2^17");
    dim3 grid(unsigned(c->N / kElems), unsigned(nlimbs), unsigned(nbatch));
    const int active = nlimbs - ((skip_lo >= 0 && skip_hi > skip_lo) ? (skip_hi - skip_lo) : 0);
    CKC_PROF(PK_NTT_FWD, s, 16.0 * double(c->N) * active * nbatch, 0.5 * double(c->N) * c->logN * active * nbatch);
    hipLaunchKernelGGL(k_ntt_cols<false>, grid, dim3(kThreads), 0, s, d, batch_stride, map, c->dprimes(),
                       c->tw.u64(), c->twp.u64(), c->ninv.u64(), c->logN, skip_lo, skip_hi);
    hipLaunchKernelGGL(k_ntt_rows<false>, grid, dim3(kThreads), 0, s, d, batch_stride, map, c->dprimes(),
                       c->tw.u64(), c->twp.u64(), c->logN, skip_lo, skip_hi);
    CKC_HIP(hipGetLastError());
    return CKC_OK;
}

int ntt_inverse(const ckc_ctx *c, uint64_t *d, int nlimbs, LimbMap map, int nbatch, size_t batch_stride,
                hipStream_t s) {
    if (nlimbs <= 0 || nbatch <= 0) return CKC_OK;
    CKC_REQUIRE(c->logN >= 12 && c->logN <= 17, CKC_EUNSUPPORTED, "NTT supports 2^12 <= N <= 2^17");
    dim3 grid(unsigned(c->N / kElems), unsigned(nlimbs), unsigned(nbatch));
    CKC_PROF(PK_NTT_INV, s, 16.0 * double(c->N) * nlimbs * nbatch, 0.5 * double(c->N) * c->logN * nlimbs * nbatch);
    hipLaunchKernelGGL(k_ntt_rows<true>, grid, dim3(kThreads), 0, s, d, batch_stride, map, c->dprimes(),
                       c->itw.u64(), c->itwp.u64(), c->logN, -1, -1);
    hipLaunchKernelGGL(k_ntt_cols<true>, grid, dim3(kThreads), 0, s, d, batch_stride, map, c->dprimes(),
                       c->itw.u64(), c->itwp.u64(), c->ninv.u64(), c->logN, -1, -1);
    CKC_HIP(hipGetLastError());
    return CKC_OK;
}
