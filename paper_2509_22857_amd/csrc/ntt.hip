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


// ---------------------------------------------------------------- radix-16
// Register-resident variant for N = 2^12 and 2^16.  Every thread holds 16
// words and runs four butterfly stages in registers (a radix-16 block); a
// 256-point pass is two such blocks with one LDS exchange between them.
// Harvey's lazy reduction keeps values in [0, 4q) (forward) or [0, 2q)
// (inverse) between stages; the last stage reduces into [0, q).
__device__ __forceinline__ void ct_bfly(uint64_t &X, uint64_t &Y, uint64_t w, uint64_t wp, uint64_t q, uint64_t q2) {
    const uint64_t x = X >= q2 ? X - q2 : X;
    const uint64_t t = mul_shoup_lazy(Y, w, wp, q);
    X = x + t;
    Y = x - t + q2;
}
__device__ __forceinline__ void gs_bfly(uint64_t &X, uint64_t &Y, uint64_t w, uint64_t wp, uint64_t q, uint64_t q2) {
    uint64_t s = X + Y;
    s = s >= q2 ? s - q2 : s;
    const uint64_t d = X - Y + q2;
    X = s;
    Y = mul_shoup_lazy(d, w, wp, q);
}
// stage s pairs j, j + (8 >> s) inside groups g of 2 (8 >> s); twiddle index idx(s, g)
template <class F>
__device__ __forceinline__ void ct16(uint64_t (&x)[16], const uint64_t *W, const uint64_t *Wp, F idx, uint64_t q,
                                     uint64_t q2) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int d = 8 >> s;
#pragma unroll
        for (int g = 0; g < (1 << s); ++g) {
            const size_t i = idx(s, g);
            const uint64_t w = W[i], wp = Wp[i];
#pragma unroll
            for (int k = 0; k < d; ++k) ct_bfly(x[g * 2 * d + k], x[g * 2 * d + k + d], w, wp, q, q2);
        }
    }
}
// stage s pairs j, j + (1 << s) inside groups g of 2 (1 << s)
template <class F>
__device__ __forceinline__ void gs16(uint64_t (&x)[16], const uint64_t *W, const uint64_t *Wp, F idx, uint64_t q,
                                     uint64_t q2) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int d = 1 << s;
#pragma unroll
        for (int g = 0; g < (8 >> s); ++g) {
            const size_t i = idx(s, g);
            const uint64_t w = W[i], wp = Wp[i];
#pragma unroll
            for (int k = 0; k < d; ++k) gs_bfly(x[g * 2 * d + k], x[g * 2 * d + k + d], w, wp, q, q2);
        }
    }
}
__device__ __forceinline__ uint64_t full_reduce4(uint64_t x, uint64_t q, uint64_t q2) {
    x = x >= q2 ? x - q2 : x;
    return x >= q ? x - q : x;
}

// columns pass: the first log2(N1) stages (N1 = N / 256 rows of 256 columns)
// forward: rows r0 + RS*j (RS = N1/16) then, for N1 = 256, rows 16*r0' + j.
template <bool INVERSE>
__global__ __launch_bounds__(kThreads) void k_ntt16_cols(uint64_t *__restrict__ data, size_t batch_stride, LimbMap map,
                                                         const Prime *__restrict__ primes,
                                                         const uint64_t *__restrict__ tw,
                                                         const uint64_t *__restrict__ twp,
                                                         const uint64_t *__restrict__ ninv, int logN, int skip_lo,
                                                         int skip_hi) {
    __shared__ uint64_t s[kElems + 16];
    const int limb = blockIdx.y;
    if (limb >= skip_lo && limb < skip_hi) return;
    const int pi = map.prime(limb);
    const uint64_t q = primes[pi].q, q2 = 2 * q;
    const size_t N = size_t(1) << logN;
    uint64_t *a = data + size_t(blockIdx.z) * batch_stride + size_t(limb) * N;
    const uint64_t *W = tw + size_t(pi) * N;
    const uint64_t *Wp = twp + size_t(pi) * N;
    const int N1 = int(N >> 8);
    const int RS = N1 >> 4;          // 1 or 16
    const int C = kElems / N1;       // 256 or 16 columns per workgroup
    const int col0 = blockIdx.x * C;
    const int tid = threadIdx.x;
    const int c = tid % C, r0 = tid / C;
    uint64_t x[16];
    auto lds = [](int row, int col) { return row * 16 + col + (row >> 4); };  // N1 = 256 layout, padded
    if (!INVERSE) {
#pragma unroll
        for (int j = 0; j < 16; ++j) x[j] = a[size_t(r0 + RS * j) * kN2 + col0 + c];
        ct16(x, W, Wp, [](int st, int g) { return size_t((1 << st) + g); }, q, q2);
        if (N1 == 256) {
#pragma unroll
            for (int j = 0; j < 16; ++j) s[lds(r0 + 16 * j, c)] = x[j];
            __syncthreads();
#pragma unroll
            for (int j = 0; j < 16; ++j) x[j] = s[lds(16 * r0 + j, c)];
            ct16(x, W, Wp, [r0](int st, int g) { return size_t((16 << st) + (r0 << st) + g); }, q, q2);
#pragma unroll
            for (int j = 0; j < 16; ++j) a[size_t(16 * r0 + j) * kN2 + col0 + c] = x[j];
        } else {
#pragma unroll
            for (int j = 0; j < 16; ++j) a[size_t(j) * kN2 + col0 + c] = x[j];
        }
    } else {
        const uint64_t ni = ninv[2 * pi], nip = ninv[2 * pi + 1];
        if (N1 == 256) {
#pragma unroll
            for (int j = 0; j < 16; ++j) x[j] = a[size_t(16 * r0 + j) * kN2 + col0 + c];
            gs16(x, W, Wp, [r0](int st, int g) { return size_t((128 >> st) + r0 * (8 >> st) + g); }, q, q2);
#pragma unroll
            for (int j = 0; j < 16; ++j) s[lds(16 * r0 + j, c)] = x[j];
            __syncthreads();
#pragma unroll
            for (int j = 0; j < 16; ++j) x[j] = s[lds(r0 + 16 * j, c)];
        } else {
#pragma unroll
            for (int j = 0; j < 16; ++j) x[j] = a[size_t(j) * kN2 + col0 + c];
        }
        gs16(x, W, Wp, [](int st, int g) { return size_t((8 >> st) + g); }, q, q2);
#pragma unroll
        for (int j = 0; j < 16; ++j) a[size_t(r0 + RS * j) * kN2 + col0 + c] = mul_shoup(x[j], ni, nip, q);
    }
}

// rows pass: the last 8 stages inside contiguous runs of 256 words.
// mapping A: element 256 b + x0 + 16 j; mapping B: element 256 b + 16 x0 + j.
template <bool INVERSE>
__global__ __launch_bounds__(kThreads) void k_ntt16_rows(uint64_t *__restrict__ data, size_t batch_stride, LimbMap map,
                                                         const Prime *__restrict__ primes,
                                                         const uint64_t *__restrict__ tw,
                                                         const uint64_t *__restrict__ twp, int logN, int skip_lo,
                                                         int skip_hi) {
    __shared__ uint64_t s[kElems + kElems / 16];
    const int limb = blockIdx.y;
    if (limb >= skip_lo && limb < skip_hi) return;
    const int pi = map.prime(limb);
    const uint64_t q = primes[pi].q, q2 = 2 * q;
    const size_t N = size_t(1) << logN;
    const size_t base = size_t(blockIdx.x) * kElems;
    uint64_t *a = data + size_t(blockIdx.z) * batch_stride + size_t(limb) * N + base;
    const uint64_t *W = tw + size_t(pi) * N;
    const uint64_t *Wp = twp + size_t(pi) * N;
    const int tid = threadIdx.x;
    const int x0 = tid & 15, b = tid >> 4;
    const size_t G = blockIdx.x * 16 + b;      // global 256-run index
    const size_t Gp = 16 * G + x0;             // global 16-group index (mapping B)
    auto pad = [](int e) { return e + (e >> 4); };
    uint64_t x[16];
    if (!INVERSE) {
#pragma unroll
        for (int j = 0; j < 16; ++j) x[j] = a[256 * b + x0 + 16 * j];
        const size_t m1 = N >> 8;
        ct16(x, W, Wp, [m1, G](int st, int g) { return (m1 << st) + (G << st) + g; }, q, q2);
#pragma unroll
        for (int j = 0; j < 16; ++j) s[pad(256 * b + x0 + 16 * j)] = x[j];
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 16; ++j) x[j] = s[pad(256 * b + 16 * x0 + j)];
        const size_t m2 = N >> 4;
        ct16(x, W, Wp, [m2, Gp](int st, int g) { return (m2 << st) + (Gp << st) + g; }, q, q2);
#pragma unroll
        for (int j = 0; j < 16; ++j) s[pad(256 * b + 16 * x0 + j)] = full_reduce4(x[j], q, q2);
        __syncthreads();
        for (int e = tid; e < kElems; e += kThreads) a[e] = s[pad(e)];
    } else {
        for (int e = tid; e < kElems; e += kThreads) s[pad(e)] = a[e];
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 16; ++j) x[j] = s[pad(256 * b + 16 * x0 + j)];
        const size_t h2 = N >> 1;
        gs16(x, W, Wp, [h2, Gp](int st, int g) { return (h2 >> st) + Gp * (8 >> st) + g; }, q, q2);
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 16; ++j) s[pad(256 * b + 16 * x0 + j)] = x[j];
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 16; ++j) x[j] = s[pad(256 * b + x0 + 16 * j)];
        const size_t h1 = N >> 5;
        gs16(x, W, Wp, [h1, G](int st, int g) { return (h1 >> st) + G * (8 >> st) + g; }, q, q2);
#pragma unroll
        for (int j = 0; j < 16; ++j) a[256 * b + x0 + 16 * j] = x[j];
    }
}

}  // namespace

int ntt_forward(const ckc_ctx *c, uint64_t *d, int nlimbs, LimbMap map, int nbatch, size_t batch_stride,
                hipStream_t s, int skip_lo, int skip_hi) {
    if (nlimbs <= 0 || nbatch <= 0) return CKC_OK;
    CKC_REQUIRE(c->logN >= 12 && c->logN <= 17, CKC_EUNSUPPORTED, "NTT supports 2^12 <= N <= 2^17");
    dim3 grid(unsigned(c->N / kElems), unsigned(nlimbs), unsigned(nbatch));
    const int active = nlimbs - ((skip_lo >= 0 && skip_hi > skip_lo) ? (skip_hi - skip_lo) : 0);
    CKC_PROF(PK_NTT_FWD, s, 16.0 * double(c->N) * active * nbatch, 0.5 * double(c->N) * c->logN * active * nbatch);
    if (c->logN == 16 || c->logN == 12) {
        hipLaunchKernelGGL(k_ntt16_cols<false>, grid, dim3(kThreads), 0, s, d, batch_stride, map, c->dprimes(),
                           c->tw.u64(), c->twp.u64(), c->ninv.u64(), c->logN, skip_lo, skip_hi);
        hipLaunchKernelGGL(k_ntt16_rows<false>, grid, dim3(kThreads), 0, s, d, batch_stride, map, c->dprimes(),
                           c->tw.u64(), c->twp.u64(), c->logN, skip_lo, skip_hi);
    } else {
        hipLaunchKernelGGL(k_ntt_cols<false>, grid, dim3(kThreads), 0, s, d, batch_stride, map, c->dprimes(),
                           c->tw.u64(), c->twp.u64(), c->ninv.u64(), c->logN, skip_lo, skip_hi);
        hipLaunchKernelGGL(k_ntt_rows<false>, grid, dim3(kThreads), 0, s, d, batch_stride, map, c->dprimes(),
                           c->tw.u64(), c->twp.u64(), c->logN, skip_lo, skip_hi);
    }
    CKC_HIP(hipGetLastError());
    return CKC_OK;
}

int ntt_inverse(const ckc_ctx *c, uint64_t *d, int nlimbs, LimbMap map, int nbatch, size_t batch_stride,
                hipStream_t s) {
    if (nlimbs <= 0 || nbatch <= 0) return CKC_OK;
    CKC_REQUIRE(c->logN >= 12 && c->logN <= 17, CKC_EUNSUPPORTED, "NTT supports 2^12 <= N <= 2^17");
    dim3 grid(unsigned(c->N / kElems), unsigned(nlimbs), unsigned(nbatch));
    CKC_PROF(PK_NTT_INV, s, 16.0 * double(c->N) * nlimbs * nbatch, 0.5 * double(c->N) * c->logN * nlimbs * nbatch);
    if (c->logN == 16 || c->logN == 12) {
        hipLaunchKernelGGL(k_ntt16_rows<true>, grid, dim3(kThreads), 0, s, d, batch_stride, map, c->dprimes(),
                           c->itw.u64(), c->itwp.u64(), c->logN, -1, -1);
        hipLaunchKernelGGL(k_ntt16_cols<true>, grid, dim3(kThreads), 0, s, d, batch_stride, map, c->dprimes(),
                           c->itw.u64(), c->itwp.u64(), c->ninv.u64(), c->logN, -1, -1);
    } else {
        hipLaunchKernelGGL(k_ntt_rows<true>, grid, dim3(kThreads), 0, s, d, batch_stride, map, c->dprimes(),
                           c->itw.u64(), c->itwp.u64(), c->logN, -1, -1);
        hipLaunchKernelGGL(k_ntt_cols<true>, grid, dim3(kThreads), 0, s, d, batch_stride, map, c->dprimes(),
                           c->itw.u64(), c->itwp.u64(), c->ninv.u64(), c->logN, -1, -1);
    }
    CKC_HIP(hipGetLastError());
    return CKC_OK;
}
