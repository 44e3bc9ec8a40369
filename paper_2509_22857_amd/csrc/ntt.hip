// Negacyclic NTT / INTT over 64-bit RNS limbs for gfx950.
//
// Forward: merged-twiddle Cooley-Tukey (the psi twist folded into a
// bit-reversed table tw[k] = psi^bitrev(k)); natural-order input, output
// index k holds a(psi^(2 bitrev(k) + 1)).  Inverse: Gentleman-Sande with
// itw[k] = psi^-bitrev(k), then a multiply by N^-1 (or by a per-limb
// constant that already contains N^-1).
//
// A limb of N = 2^logN words is split as N1 x N2 with N2 = 256: the stages
// whose butterfly distance is a multiple of N2 only mix words of one column
// (stride N2), the remaining log2(N2) stages only mix words inside one
// contiguous run of N2.  Each pass stages 4096 words (32 KiB) per workgroup
// through LDS and runs its stages there, so a transform reads and writes the
// limb twice.
//
// The passes take their input and give their output through load / store
// functors, so the key-switching steps around a transform run inside it:
// the first forward pass can compute its input by fast basis conversion from
// a few coefficient-form source limbs (ModUp and ModDown), and the last
// forward pass can finish ModDown ((acc - x) P^-1 + addend) instead of
// storing x.  The arithmetic of the transform itself is the same in every
// variant.
#include "batch.h"
#include "prof.h"

namespace {

constexpr int kThreads = 256;
constexpr int kElems = 4096;
constexpr int kLogN2 = 8;
constexpr int kN2 = 1 << kLogN2;

// ---------------------------------------------------------------- generic sizes
// columns pass: stages with distance >= N2.  Loads / stores address words of
// the limb by index (row * N2 + column).
template <class Ld, class St>
__device__ __forceinline__ void cols_generic(Ld ld, St st, bool inverse, uint64_t *s, const uint64_t *W,
                                             const uint64_t *Wp, uint64_t q, int logN, int col0, uint64_t sc,
                                             uint64_t scp) {
    const int logN1 = logN - kLogN2;
    const int N1 = 1 << logN1;
    const int logC = 12 - logN1;  // columns per workgroup = kElems / N1
    const int C = 1 << logC;
    for (int e = threadIdx.x; e < kElems; e += kThreads) {
        const int c = e & (C - 1), r = e >> logC;
        s[e] = ld(size_t(r) * kN2 + col0 + c);
    }
    __syncthreads();
    if (!inverse) {
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
            st(size_t(r) * kN2 + col0 + c, s[e]);
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
        for (int e = threadIdx.x; e < kElems; e += kThreads) {
            const int c = e & (C - 1), r = e >> logC;
            st(size_t(r) * kN2 + col0 + c, mul_shoup(s[e], sc, scp, q));
        }
    }
}

// rows pass: the last 8 stages inside contiguous runs of 256 words; loads and
// stores address words of the workgroup's 4096-word tile.
template <class Ld, class St>
__device__ __forceinline__ void rows_generic(Ld ld, St st, bool inverse, uint64_t *s, const uint64_t *W,
                                             const uint64_t *Wp, uint64_t q, size_t N, size_t base) {
    for (int e = threadIdx.x; e < kElems; e += kThreads) s[e] = ld(e);
    __syncthreads();
    if (!inverse) {
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
    for (int e = threadIdx.x; e < kElems; e += kThreads) st(e, s[e]);
}

// ---------------------------------------------------------------- radix-16
// Register-resident variant for N = 2^12 and 2^16.  Every thread holds 16
// words and runs four butterfly stages in registers (a radix-16 block); a
// 256-point pass is two such blocks with one LDS exchange between them.
// Harvey's lazy reduction keeps values in [0, 4q) (forward) or [0, 2q)
// (inverse) between stages; the last stage reduces into [0, q).
//
// Each butterfly is one block of instructions over four fixed scratch pairs
// v56..v63 (clobbered, so the compiler keeps nothing there across it):
//  * the Shoup quotient qh = hi64(Y w') exactly: A = y1 p0 + hi32(y0 p0)
//    (no overflow), A' = y0 p1 + A with its carry k out of 2^64, then
//    qh = y1 p1 + (hi32(A') + k 2^32) as one multiply-add whose addend pair
//    is {hi32(A'), k};
//  * t = Y w - qh q mod 2^64 as Y w + qh (2^64 - q): multiply-adds and
//    low-word products only, no 64-bit subtraction;
//  * conditional subtractions of 2q through a mask-selected pair added with
//    one 64-bit add, and x - t + 2q as x + (2q + 1) + ~t.
// gfx950 needs two instructions between a vector write of a scalar register
// and its read (carry-in or mask); the orders below keep that distance.  The
// compiler's own code for the same formulas spends ~30 instructions per
// butterfly (half a dozen of them register moves building multiply-add
// addend pairs), these 24 and 25.
#define CKC_BFLY_CLOBBERS "v56", "v57", "v58", "v59", "v60", "v61", "v62", "v63"
// The modulus' constants are wave-uniform and stay in scalar registers (every
// instruction below reads at most one); twiddles are scalar too where the
// whole wave uses the same ones (UT), else per lane.  The forward block reads
// no input after writing an output, so outputs may reuse input registers.
#define CKC_CT_BODY                                         \
    "v_cmp_ge_u64_e64 %[m], %[X], %[q2]\n\t"                \
    "v_mul_hi_u32 v56, %[y0], %[p0]\n\t"                    \
    "v_mov_b32 v57, 0\n\t"                                  \
    "v_mad_u64_u32 v[56:57], %[j], %[y1], %[p0], v[56:57]\n\t" \
    "v_mad_u64_u32 v[58:59], %[j], %[y0], %[w0], 0\n\t"     \
    "v_mad_u64_u32 v[56:57], %[k], %[y0], %[p1], v[56:57]\n\t" \
    "v_mul_lo_u32 v60, %[y0], %[w1]\n\t"                    \
    "v_mul_lo_u32 v61, %[y1], %[w0]\n\t"                    \
    "v_mov_b32 v56, v57\n\t"                                \
    "v_addc_co_u32_e64 v57, %[j], 0, 0, %[k]\n\t"           \
    "v_mad_u64_u32 v[56:57], %[j], %[y1], %[p1], v[56:57]\n\t" \
    "v_add3_u32 v59, v59, v60, v61\n\t"                     \
    "v_mad_u64_u32 v[58:59], %[j], v56, %[qn0], v[58:59]\n\t" \
    "v_mul_lo_u32 v60, v56, %[qn1]\n\t"                     \
    "v_mul_lo_u32 v61, v57, %[qn0]\n\t"                     \
    "v_cndmask_b32_e64 v62, 0, %[nq2lo], %[m]\n\t"          \
    "v_cndmask_b32_e64 v63, 0, %[nq2hi], %[m]\n\t"          \
    "v_add3_u32 v59, v59, v60, v61\n\t"                     \
    "v_lshl_add_u64 v[62:63], %[X], 0, v[62:63]\n\t"        \
    "v_lshl_add_u64 %[xo], v[62:63], 0, v[58:59]\n\t"       \
    "v_not_b32 v60, v58\n\t"                                \
    "v_not_b32 v61, v59\n\t"                                \
    "v_lshl_add_u64 v[62:63], v[62:63], 0, %[q2p1]\n\t"     \
    "v_lshl_add_u64 %[yo], v[62:63], 0, v[60:61]"
#define CKC_GS_BODY                                         \
    "v_lshl_add_u64 v[62:63], %[X], 0, %[Y]\n\t"            \
    "v_not_b32 v60, %[y0]\n\t"                              \
    "v_not_b32 v61, %[y1]\n\t"                              \
    "v_cmp_ge_u64_e64 %[m], v[62:63], %[q2]\n\t"            \
    "v_lshl_add_u64 v[58:59], %[X], 0, %[q2p1]\n\t"         \
    "v_lshl_add_u64 v[58:59], v[58:59], 0, v[60:61]\n\t"    \
    "v_mul_hi_u32 v56, v58, %[p0]\n\t"                      \
    "v_mov_b32 v57, 0\n\t"                                  \
    "v_mad_u64_u32 v[56:57], %[j], v59, %[p0], v[56:57]\n\t" \
    "v_cndmask_b32_e64 v60, 0, %[nq2lo], %[m]\n\t"          \
    "v_mad_u64_u32 v[56:57], %[k], v58, %[p1], v[56:57]\n\t" \
    "v_cndmask_b32_e64 v61, 0, %[nq2hi], %[m]\n\t"          \
    "v_lshl_add_u64 %[xo], v[62:63], 0, v[60:61]\n\t"       \
    "v_mov_b32 v56, v57\n\t"                                \
    "v_addc_co_u32_e64 v57, %[j], 0, 0, %[k]\n\t"           \
    "v_mad_u64_u32 v[56:57], %[j], v59, %[p1], v[56:57]\n\t" \
    "v_mul_lo_u32 v60, v58, %[w1]\n\t"                      \
    "v_mul_lo_u32 v61, v59, %[w0]\n\t"                      \
    "v_mul_lo_u32 v62, v56, %[qn1]\n\t"                     \
    "v_mul_lo_u32 v63, v57, %[qn0]\n\t"                     \
    "v_add3_u32 v61, v60, v61, v62\n\t"                     \
    "v_add_u32 v61, v61, v63\n\t"                           \
    "v_mov_b32 v60, 0\n\t"                                  \
    "v_mad_u64_u32 %[yo], %[j], v58, %[w0], v[60:61]\n\t"   \
    "v_mad_u64_u32 %[yo], %[j], v56, %[qn0], %[yo]"
template <bool UT>
__device__ __forceinline__ void ct_bfly(uint64_t &X, uint64_t &Y, uint64_t w, uint64_t wp, uint64_t q, uint64_t q2) {
    const uint64_t qn = 0 - q, nq2 = 0 - q2, q2p1 = q2 + 1;
    uint64_t xo, yo, m, k, j;
    if constexpr (UT)
        asm(CKC_CT_BODY
            : [xo] "=v"(xo), [yo] "=v"(yo), [m] "=&s"(m), [k] "=&s"(k), [j] "=&s"(j)
            : [X] "v"(X), [q2] "s"(q2), [y0] "v"(uint32_t(Y)), [y1] "v"(uint32_t(Y >> 32)), [w0] "s"(uint32_t(w)),
              [w1] "s"(uint32_t(w >> 32)), [p0] "s"(uint32_t(wp)), [p1] "s"(uint32_t(wp >> 32)),
              [qn0] "s"(uint32_t(qn)), [qn1] "s"(uint32_t(qn >> 32)), [nq2lo] "v"(uint32_t(nq2)),
              [nq2hi] "v"(uint32_t(nq2 >> 32)), [q2p1] "s"(q2p1)
            : CKC_BFLY_CLOBBERS);
    else
        asm(CKC_CT_BODY
            : [xo] "=v"(xo), [yo] "=v"(yo), [m] "=&s"(m), [k] "=&s"(k), [j] "=&s"(j)
            : [X] "v"(X), [q2] "s"(q2), [y0] "v"(uint32_t(Y)), [y1] "v"(uint32_t(Y >> 32)), [w0] "v"(uint32_t(w)),
              [w1] "v"(uint32_t(w >> 32)), [p0] "v"(uint32_t(wp)), [p1] "v"(uint32_t(wp >> 32)),
              [qn0] "s"(uint32_t(qn)), [qn1] "s"(uint32_t(qn >> 32)), [nq2lo] "v"(uint32_t(nq2)),
              [nq2hi] "v"(uint32_t(nq2 >> 32)), [q2p1] "s"(q2p1)
            : CKC_BFLY_CLOBBERS);
    X = xo;
    Y = yo;
}
template <bool UT>
__device__ __forceinline__ void gs_bfly(uint64_t &X, uint64_t &Y, uint64_t w, uint64_t wp, uint64_t q, uint64_t q2) {
    const uint64_t qn = 0 - q, nq2 = 0 - q2, q2p1 = q2 + 1;
    uint64_t xo, yo, m, k, j;
    if constexpr (UT)
        asm(CKC_GS_BODY
            : [xo] "=&v"(xo), [yo] "=&v"(yo), [m] "=&s"(m), [k] "=&s"(k), [j] "=&s"(j)
            : [X] "v"(X), [Y] "v"(Y), [q2] "s"(q2), [y0] "v"(uint32_t(Y)), [y1] "v"(uint32_t(Y >> 32)),
              [w0] "s"(uint32_t(w)), [w1] "s"(uint32_t(w >> 32)), [p0] "s"(uint32_t(wp)), [p1] "s"(uint32_t(wp >> 32)),
              [qn0] "s"(uint32_t(qn)), [qn1] "s"(uint32_t(qn >> 32)), [nq2lo] "v"(uint32_t(nq2)),
              [nq2hi] "v"(uint32_t(nq2 >> 32)), [q2p1] "s"(q2p1)
            : CKC_BFLY_CLOBBERS);
    else
        asm(CKC_GS_BODY
            : [xo] "=&v"(xo), [yo] "=&v"(yo), [m] "=&s"(m), [k] "=&s"(k), [j] "=&s"(j)
            : [X] "v"(X), [Y] "v"(Y), [q2] "s"(q2), [y0] "v"(uint32_t(Y)), [y1] "v"(uint32_t(Y >> 32)),
              [w0] "v"(uint32_t(w)), [w1] "v"(uint32_t(w >> 32)), [p0] "v"(uint32_t(wp)), [p1] "v"(uint32_t(wp >> 32)),
              [qn0] "s"(uint32_t(qn)), [qn1] "s"(uint32_t(qn >> 32)), [nq2lo] "v"(uint32_t(nq2)),
              [nq2hi] "v"(uint32_t(nq2 >> 32)), [q2p1] "s"(q2p1)
            : CKC_BFLY_CLOBBERS);
    X = xo;
    Y = yo;
}
// stage s pairs j, j + (8 >> s) inside groups g of 2 (8 >> s); twiddle index idx(s, g)
template <bool UT = false, class F>
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
            for (int k = 0; k < d; ++k) ct_bfly<UT>(x[g * 2 * d + k], x[g * 2 * d + k + d], w, wp, q, q2);
        }
    }
}
// stage s pairs j, j + (1 << s) inside groups g of 2 (1 << s)
template <bool UT = false, class F>
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
            for (int k = 0; k < d; ++k) gs_bfly<UT>(x[g * 2 * d + k], x[g * 2 * d + k + d], w, wp, q, q2);
        }
    }
}
__device__ __forceinline__ uint64_t full_reduce4(uint64_t x, uint64_t q, uint64_t q2) {
    x = x >= q2 ? x - q2 : x;
    return x >= q ? x - q : x;
}
__device__ __forceinline__ int lds16(int row, int col) { return row * 16 + col + (row >> 4); }  // N1 = 256, padded
__device__ __forceinline__ int pad16(int e) { return e + (e >> 4); }

// columns pass, forward: the first log2(N1) stages (N1 = N / 256 rows of 256
// columns); rows r0 + RS*j (RS = N1/16) then, for N1 = 256, rows 16*r0' + j.
// Output lazy in [0, 4q).
template <class Ld, class St>
__device__ __forceinline__ void cols16_fwd(Ld ld, St st, uint64_t *s, const uint64_t *W, const uint64_t *Wp,
                                           uint64_t q, size_t N, int col_block) {
    const uint64_t q2 = 2 * q;
    const int N1 = int(N >> 8);
    const int RS = N1 >> 4;     // 1 or 16
    const int C = kElems / N1;  // 256 or 16 columns per workgroup
    const int col0 = col_block * C;
    const int tid = threadIdx.x;
    const int c = tid % C, r0 = tid / C;
    uint64_t x[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) x[j] = ld(size_t(r0 + RS * j) * kN2 + col0 + c);
    ct16<true>(x, W, Wp, [](int st, int g) { return size_t((1 << st) + g); }, q, q2);
    if (N1 == 256) {
#pragma unroll
        for (int j = 0; j < 16; ++j) s[lds16(r0 + 16 * j, c)] = x[j];
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 16; ++j) x[j] = s[lds16(16 * r0 + j, c)];
        ct16(x, W, Wp, [r0](int st, int g) { return size_t((16 << st) + (r0 << st) + g); }, q, q2);
#pragma unroll
        for (int j = 0; j < 16; ++j) st(size_t(16 * r0 + j) * kN2 + col0 + c, x[j]);
    } else {
#pragma unroll
        for (int j = 0; j < 16; ++j) st(size_t(j) * kN2 + col0 + c, x[j]);
    }
}

// columns pass, inverse (the last pass of an INTT), output times (sc, scp)
template <class Ld, class St>
__device__ __forceinline__ void cols16_inv(Ld ld, St st, uint64_t *s, const uint64_t *W, const uint64_t *Wp,
                                           uint64_t q, size_t N, int col_block, uint64_t sc, uint64_t scp) {
    const uint64_t q2 = 2 * q;
    const int N1 = int(N >> 8);
    const int RS = N1 >> 4;
    const int C = kElems / N1;
    const int col0 = col_block * C;
    const int tid = threadIdx.x;
    const int c = tid % C, r0 = tid / C;
    uint64_t x[16];
    if (N1 == 256) {
#pragma unroll
        for (int j = 0; j < 16; ++j) x[j] = ld(size_t(16 * r0 + j) * kN2 + col0 + c);
        gs16(x, W, Wp, [r0](int st, int g) { return size_t((128 >> st) + r0 * (8 >> st) + g); }, q, q2);
#pragma unroll
        for (int j = 0; j < 16; ++j) s[lds16(16 * r0 + j, c)] = x[j];
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 16; ++j) x[j] = s[lds16(r0 + 16 * j, c)];
    } else {
#pragma unroll
        for (int j = 0; j < 16; ++j) x[j] = ld(size_t(j) * kN2 + col0 + c);
    }
    gs16<true>(x, W, Wp, [](int st, int g) { return size_t((8 >> st) + g); }, q, q2);
#pragma unroll
    for (int j = 0; j < 16; ++j) st(size_t(r0 + RS * j) * kN2 + col0 + c, mul_shoup(x[j], sc, scp, q));
}

// rows pass, forward: the last 8 stages inside runs of 256 words.  mapping A:
// element 256 b + x0 + 16 j; mapping B: element 256 b + 16 x0 + j.  Output in
// [0, q), stored through st(tile index, value) from LDS in tile order.
template <class Ld, class St>
__device__ __forceinline__ void rows16_fwd(Ld ld, St st, uint64_t *s, const uint64_t *W, const uint64_t *Wp,
                                           uint64_t q, size_t N, int tile) {
    const uint64_t q2 = 2 * q;
    const int tid = threadIdx.x;
    const int x0 = tid & 15, b = tid >> 4;
    const size_t G = size_t(tile) * 16 + b;  // global 256-run index
    const size_t Gp = 16 * G + x0;           // global 16-group index (mapping B)
    uint64_t x[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) x[j] = ld(256 * b + x0 + 16 * j);
    const size_t m1 = N >> 8;
    ct16(x, W, Wp, [m1, G](int st, int g) { return (m1 << st) + (G << st) + g; }, q, q2);
#pragma unroll
    for (int j = 0; j < 16; ++j) s[pad16(256 * b + x0 + 16 * j)] = x[j];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 16; ++j) x[j] = s[pad16(256 * b + 16 * x0 + j)];
    const size_t m2 = N >> 4;
    ct16(x, W, Wp, [m2, Gp](int st, int g) { return (m2 << st) + (Gp << st) + g; }, q, q2);
#pragma unroll
    for (int j = 0; j < 16; ++j) s[pad16(256 * b + 16 * x0 + j)] = full_reduce4(x[j], q, q2);
    __syncthreads();
    for (int e = tid; e < kElems; e += kThreads) st(e, s[pad16(e)]);
}

// rows pass, inverse (the first pass of an INTT); output lazy in [0, 2q)
template <class Ld, class St>
__device__ __forceinline__ void rows16_inv(Ld ld, St st, uint64_t *s, const uint64_t *W, const uint64_t *Wp,
                                           uint64_t q, size_t N, int tile) {
    const uint64_t q2 = 2 * q;
    const int tid = threadIdx.x;
    const int x0 = tid & 15, b = tid >> 4;
    const size_t G = size_t(tile) * 16 + b;
    const size_t Gp = 16 * G + x0;
    uint64_t x[16];
    for (int e = tid; e < kElems; e += kThreads) s[pad16(e)] = ld(e);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 16; ++j) x[j] = s[pad16(256 * b + 16 * x0 + j)];
    const size_t h2 = N >> 1;
    gs16(x, W, Wp, [h2, Gp](int st, int g) { return (h2 >> st) + Gp * (8 >> st) + g; }, q, q2);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 16; ++j) s[pad16(256 * b + 16 * x0 + j)] = x[j];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 16; ++j) x[j] = s[pad16(256 * b + x0 + 16 * j)];
    const size_t h1 = N >> 5;
    gs16(x, W, Wp, [h1, G](int st, int g) { return (h1 >> st) + G * (8 >> st) + g; }, q, q2);
#pragma unroll
    for (int j = 0; j < 16; ++j) st(256 * b + x0 + 16 * j, x[j]);
}

__device__ __forceinline__ bool radix16(int logN) { return logN == 16 || logN == 12; }

// ---------------------------------------------------------------- kernels
// grid (N / 4096 tiles, limbs, batch); limbs in [skip_lo, skip_hi) untouched
__global__ __launch_bounds__(kThreads) void k_fwd_cols(uint64_t *__restrict__ data, size_t bs, LimbMap map,
                                                       const Prime *__restrict__ primes,
                                                       const uint64_t *__restrict__ tw,
                                                       const uint64_t *__restrict__ twp, int logN, int skip_lo,
                                                       int skip_hi) {
    __shared__ uint64_t s[kElems + kElems / 16];
    const int limb = blockIdx.y;
    if (limb >= skip_lo && limb < skip_hi) return;
    const int pi = map.prime(limb);
    const uint64_t q = primes[pi].q;
    const size_t N = size_t(1) << logN;
    uint64_t *a = data + size_t(blockIdx.z) * bs + size_t(limb) * N;
    const uint64_t *W = tw + size_t(pi) * N, *Wp = twp + size_t(pi) * N;
    auto ld = [a](size_t i) { return a[i]; };
    auto st = [a](size_t i, uint64_t v) { a[i] = v; };
    if (radix16(logN))
        cols16_fwd(ld, st, s, W, Wp, q, N, blockIdx.x);
    else
        cols_generic(ld, st, false, s, W, Wp, q, logN, blockIdx.x << (12 - (logN - kLogN2)), 0, 0);
}

// first forward pass fed by fast basis conversion: word i of output limb t is
//   sum_{k < ns} v_k * hat[t][k]  mod q_t,  v_k = y_k[i] taken in (-s_k/2, s_k/2]
// (centred source values: the conversion is then the centred lift plus u S
// with |u| < ns/2, an unbiased rounding for ModDown and a zero-mean digit for
// ModUp; a value above s_k/2 stands for value - s_k, so each subtracts
// S = s_k hat_k, counted and applied as one more product by -S.  The table
// holds hat and -S times 2^64 mod q_t, and the sum ends in one Montgomery
// reduction, which removes the factor)
// from the pre-scaled coefficient-form source limbs y_k (y = x (S/s_k)^-1 mod
// s_k); limbs in [copy_lo, copy_hi) are copied from `copy` instead (their NTT
// form is already known) and left alone by the second pass.  The number of
// sources NS is a template argument: with a run-time count the compiler
// executed every one of the kMaxBconv possible products under a mask.
// Body of the pass for output block `a0` (its limbs, stride N), with one
// batch entry's pointers resolved: src its first source limb, copy its
// NTT-form input (limb 0).  The per-entry pointers are resolved by the
// kernels from their arguments, never through a local copy of a pointer
// table (indexed at run time, such a copy lives in scratch memory: 608 bytes
// per lane, twice the pass's time).
template <int NS>
__device__ __forceinline__ void bconv_cols(uint64_t *a0, const uint64_t *src, const uint64_t *hat,
                                           const uint64_t *neg_s, const uint64_t *s_half, const uint64_t *copy,
                                           int copy_lo, int copy_hi, LimbMap map, const Prime *__restrict__ primes,
                                           const uint64_t *__restrict__ tw, const uint64_t *__restrict__ twp,
                                           int logN, uint64_t *s) {
    const int limb = blockIdx.y;
    const size_t N = size_t(1) << logN;
    uint64_t *a = a0 + size_t(limb) * N;
    if (limb >= copy_lo && limb < copy_hi) {
        // this workgroup's words of the limb, in the same (row, column) tiling
        const int logN1 = logN - kLogN2;
        const int logC = 12 - logN1;
        const int col0 = blockIdx.x << logC;
        const uint64_t *cp = copy + size_t(limb) * N;
        for (int e = threadIdx.x; e < kElems; e += kThreads) {
            const size_t i = size_t(e >> logC) * kN2 + col0 + (e & ((1 << logC) - 1));
            a[i] = cp[i];
        }
        return;
    }
    const int pi = map.prime(limb);
    const Prime P = primes[pi];
    const uint64_t *W = tw + size_t(pi) * N, *Wp = twp + size_t(pi) * N;
    uint64_t h[NS], half[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        h[k] = hat[size_t(limb) * NS + k];
        half[k] = s_half[k];
    }
    const uint64_t negS = neg_s[limb];
    auto ld = [src, h, half, negS, N, P](size_t i) {
        accc acc{0, 0, 0, 0, 0};
        uint64_t neg = 0;
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            const uint64_t v = src[size_t(k) * N + i];
            macc(acc, v, h[k]);
            neg += v > half[k] ? 1 : 0;
        }
        macc(acc, neg, negS);
        return redc_accc<NS + 1>(acc, P);
    };
    auto st = [a](size_t i, uint64_t v) { a[i] = v; };
    if (radix16(logN))
        cols16_fwd(ld, st, s, W, Wp, P.q, N, blockIdx.x);
    else
        cols_generic(ld, st, false, s, W, Wp, P.q, logN, blockIdx.x << (12 - (logN - kLogN2)), 0, 0);
}

template <int NS>
__global__ __launch_bounds__(kThreads) void k_fwd_cols_bconv(uint64_t *__restrict__ data, size_t bs, LimbMap map,
                                                             const Prime *__restrict__ primes,
                                                             const uint64_t *__restrict__ tw,
                                                             const uint64_t *__restrict__ twp, int logN,
                                                             BconvIn in) {
    __shared__ uint64_t s[kElems + kElems / 16];
    const int b = blockIdx.z;
    const uint64_t *cp = in.use_copyp ? in.copyp.p[b] + in.copy_off : in.copy + size_t(b) * in.copy_bs;
    bconv_cols<NS>(data + size_t(b) * bs, in.src + size_t(b) * in.src_bs, in.hat, in.neg_s, in.s_half, cp,
                   in.copy_lo, in.copy_hi, map, primes, tw, twp, logN, s);
}

// The same first pass for the ModUp of `ndig` digits of NS primes each in
// one launch: batch index z = b ndig + j is digit j of input b, written to
// data + b bs + j nt N (the digits' layout [b][dnum][nt][N]); digit j reads
// the pre-scaled coefficient-form limbs j NS .. j NS + NS - 1 of input b and
// copies its own limbs from the NTT-form input.
struct DigitsIn {
    const uint64_t *src;   // [batch][l+1][N], stride src_bs
    size_t src_bs;
    const uint64_t *copy;  // [batch][l+1][N] NTT form, stride copy_bs
    size_t copy_bs;
    int ndig, nt;
    const uint64_t *hat[kMaxDnum], *neg_s[kMaxDnum], *s_half[kMaxDnum];
    Ptrs copyp;  // with use_copyp, input b's NTT form at copyp.p[b] + copy_off
    size_t copy_off;
    int use_copyp;
};
template <int NS>
__global__ __launch_bounds__(kThreads) void k_fwd_cols_bconv_dig(uint64_t *__restrict__ data, size_t bs,
                                                                 LimbMap map, const Prime *__restrict__ primes,
                                                                 const uint64_t *__restrict__ tw,
                                                                 const uint64_t *__restrict__ twp, int logN,
                                                                 DigitsIn d) {
    __shared__ uint64_t s[kElems + kElems / 16];
    const int z = blockIdx.z, b = z / d.ndig, j = z - b * d.ndig, lo = j * NS;
    const size_t N = size_t(1) << logN;
    const uint64_t *cp = d.use_copyp ? d.copyp.p[b] + d.copy_off : d.copy + size_t(b) * d.copy_bs;
    bconv_cols<NS>(data + size_t(b) * bs + size_t(j) * d.nt * N, d.src + size_t(b) * d.src_bs + size_t(lo) * N,
                   d.hat[j], d.neg_s[j], d.s_half[j], cp, lo, lo + NS, map, primes, tw, twp, logN, s);
}

// Second forward pass.  Limbs in [skip_lo, skip_hi) are left alone; with
// dig_n > 0 the batch is the digits of a ModUp ([b][dig_n][nt][N], z = b
// dig_n + j) and digit j leaves its own limbs [j dig_alpha, min((j + 1)
// dig_alpha, dig_nl)) alone instead.
__global__ __launch_bounds__(kThreads) void k_fwd_rows(uint64_t *__restrict__ data, size_t bs, LimbMap map,
                                                       const Prime *__restrict__ primes,
                                                       const uint64_t *__restrict__ tw,
                                                       const uint64_t *__restrict__ twp, int logN, int skip_lo,
                                                       int skip_hi, int dig_n, int dig_alpha, int dig_nl) {
    __shared__ uint64_t s[kElems + kElems / 16];
    const int limb = blockIdx.y;
    if (dig_n > 0) {
        const int j = int(blockIdx.z) % dig_n;
        skip_lo = j * dig_alpha;
        skip_hi = min(skip_lo + dig_alpha, dig_nl);
    }
    if (limb >= skip_lo && limb < skip_hi) return;
    const int pi = map.prime(limb);
    const uint64_t q = primes[pi].q;
    const size_t N = size_t(1) << logN;
    const size_t base = size_t(blockIdx.x) * kElems;
    uint64_t *a = data + size_t(blockIdx.z) * bs + size_t(limb) * N + base;
    const uint64_t *W = tw + size_t(pi) * N, *Wp = twp + size_t(pi) * N;
    auto ld = [a](int e) { return a[e]; };
    auto st = [a](int e, uint64_t v) { a[e] = v; };
    if (radix16(logN))
        rows16_fwd(ld, st, s, W, Wp, q, N, blockIdx.x);
    else
        rows_generic(ld, st, false, s, W, Wp, q, N, base);
}

// last forward pass finishing ModDown: batch index z = 2 b + p, and
//   out_p[b][i][k] = (acc[z][i][k] - x[k]) P^-1 + add_p[b][i][perm?(k)]
__global__ __launch_bounds__(kThreads) void k_fwd_rows_combine(const uint64_t *__restrict__ data, size_t bs,
                                                               const Prime *__restrict__ primes,
                                                               const uint64_t *__restrict__ tw,
                                                               const uint64_t *__restrict__ twp, int logN,
                                                               CombineOut co) {
    __shared__ uint64_t s[kElems + kElems / 16];
    const int limb = blockIdx.y;
    const int b = blockIdx.z >> 1, p = blockIdx.z & 1;
    const uint64_t q = primes[limb].q;
    const size_t N = size_t(1) << logN;
    const size_t base = size_t(blockIdx.x) * kElems;
    const uint64_t *a = data + size_t(blockIdx.z) * bs + size_t(limb) * N + base;
    const uint64_t *W = tw + size_t(limb) * N, *Wp = twp + size_t(limb) * N;
    const uint64_t *x = co.acc + size_t(blockIdx.z) * co.acc_bs + size_t(limb) * N + base;
    const uint64_t pv = co.pinv[2 * limb], pvp = co.pinv[2 * limb + 1];
    const bool has = p == 0 ? co.has_add0 : co.has_add1;
    const uint64_t *ad = has ? (p == 0 ? co.add0.p[b] : co.add1.p[b]) + size_t(limb) * N : nullptr;
    const uint32_t *pm = p == 0 ? co.perm0 : nullptr;
    uint64_t *o = (p == 0 ? co.out0.p[b] : co.out1.p[b]) + size_t(limb) * N;
    auto ld = [a](int e) { return a[e]; };
    auto st = [=](int e, uint64_t v) {
        const size_t k = base + e;
        uint64_t r = mul_shoup(sub_mod(x[e], v, q), pv, pvp, q);
        if (ad) r = add_mod(r, ad[pm ? pm[k] : k], q);
        o[k] = r;
    };
    if (radix16(logN))
        rows16_fwd(ld, st, s, W, Wp, q, N, blockIdx.x);
    else
        rows_generic(ld, st, false, s, W, Wp, q, N, base);
}

// first inverse pass, reading from src (may equal data: in place), or with
// use_srcp from srcp.p[z] + src_off
__global__ __launch_bounds__(kThreads) void k_inv_rows(uint64_t *__restrict__ data, size_t bs,
                                                       const uint64_t *src, size_t src_bs, LimbMap map,
                                                       const Prime *__restrict__ primes,
                                                       const uint64_t *__restrict__ itw,
                                                       const uint64_t *__restrict__ itwp, int logN, Ptrs srcp,
                                                       size_t src_off, int use_srcp) {
    __shared__ uint64_t s[kElems + kElems / 16];
    const int limb = blockIdx.y;
    const int pi = map.prime(limb);
    const uint64_t q = primes[pi].q;
    const size_t N = size_t(1) << logN;
    const size_t base = size_t(blockIdx.x) * kElems;
    uint64_t *a = data + size_t(blockIdx.z) * bs + size_t(limb) * N + base;
    const uint64_t *in =
        (use_srcp ? srcp.p[blockIdx.z] + src_off : src + size_t(blockIdx.z) * src_bs) + size_t(limb) * N + base;
    const uint64_t *W = itw + size_t(pi) * N, *Wp = itwp + size_t(pi) * N;
    auto ld = [in](int e) { return in[e]; };
    auto st = [a](int e, uint64_t v) { a[e] = v; };
    if (radix16(logN))
        rows16_inv(ld, st, s, W, Wp, q, N, blockIdx.x);
    else
        rows_generic(ld, st, true, s, W, Wp, q, N, base);
}

// last inverse pass; output times N^-1, or times scale2[limb] (a pair value,
// Shoup companion that already contains N^-1)
__global__ __launch_bounds__(kThreads) void k_inv_cols(uint64_t *__restrict__ data, size_t bs, LimbMap map,
                                                       const Prime *__restrict__ primes,
                                                       const uint64_t *__restrict__ itw,
                                                       const uint64_t *__restrict__ itwp,
                                                       const uint64_t *__restrict__ ninv,
                                                       const uint64_t *__restrict__ scale2, int logN) {
    __shared__ uint64_t s[kElems + kElems / 16];
    const int limb = blockIdx.y;
    const int pi = map.prime(limb);
    const uint64_t q = primes[pi].q;
    const size_t N = size_t(1) << logN;
    uint64_t *a = data + size_t(blockIdx.z) * bs + size_t(limb) * N;
    const uint64_t *W = itw + size_t(pi) * N, *Wp = itwp + size_t(pi) * N;
    const uint64_t sc = scale2 ? scale2[2 * limb] : ninv[2 * pi];
    const uint64_t scp = scale2 ? scale2[2 * limb + 1] : ninv[2 * pi + 1];
    auto ld = [a](size_t i) { return a[i]; };
    auto st = [a](size_t i, uint64_t v) { a[i] = v; };
    if (radix16(logN))
        cols16_inv(ld, st, s, W, Wp, q, N, blockIdx.x, sc, scp);
    else
        cols_generic(ld, st, true, s, W, Wp, q, logN, blockIdx.x << (12 - (logN - kLogN2)), sc, scp);
}

}  // namespace

int ntt_forward_ex(const ckc_ctx *c, uint64_t *d, int nlimbs, LimbMap map, int nbatch, size_t bs, hipStream_t s,
                   int skip_lo, int skip_hi, const BconvIn *bin, const CombineOut *cout) {
    if (nlimbs <= 0 || nbatch <= 0) return CKC_OK;
    CKC_REQUIRE(c->logN >= 12 && c->logN <= 16, CKC_EUNSUPPORTED, "NTT supports 2^12 <= N <= 2^16");
    CKC_REQUIRE(!bin || (bin->ns >= 1 && bin->ns <= kMaxBconv), CKC_EUNSUPPORTED, "too many basis-conversion sources");
    const dim3 grid(unsigned(c->N / kElems), unsigned(nlimbs), unsigned(nbatch));
    const int lo = bin ? bin->copy_lo : skip_lo, hi = bin ? bin->copy_hi : skip_hi;
    const int active = nlimbs - ((lo >= 0 && hi > lo) ? (hi - lo) : 0);
    {
        // algorithmic bytes: the source limbs once (basis conversion) or the
        // limb, the limb written, and the combine's operands
        const double W = 8.0 * double(c->N) * nbatch;
        const double src = bin ? double(bin->ns) + 2.0 * (nlimbs - active) : double(active);
        const double epi = cout ? 2.5 * active : 1.0 * active;
        CKC_PROF(PK_NTT_FWD, s, W * (src + epi), 0.5 * double(c->N) * c->logN * active * nbatch);
        if (bin) {
            using BconvFn = void (*)(uint64_t *, size_t, LimbMap, const Prime *, const uint64_t *, const uint64_t *,
                                     int, BconvIn);
            static constexpr BconvFn fns[kMaxBconv] = {k_fwd_cols_bconv<1>, k_fwd_cols_bconv<2>, k_fwd_cols_bconv<3>,
                                                       k_fwd_cols_bconv<4>, k_fwd_cols_bconv<5>, k_fwd_cols_bconv<6>,
                                                       k_fwd_cols_bconv<7>, k_fwd_cols_bconv<8>};
            hipLaunchKernelGGL(fns[bin->ns - 1], grid, dim3(kThreads), 0, s, d, bs, map, c->dprimes(), c->tw.u64(),
                               c->twp.u64(), c->logN, *bin);
        }
        else
            hipLaunchKernelGGL(k_fwd_cols, grid, dim3(kThreads), 0, s, d, bs, map, c->dprimes(), c->tw.u64(),
                               c->twp.u64(), c->logN, skip_lo, skip_hi);
        if (cout)
            hipLaunchKernelGGL(k_fwd_rows_combine, grid, dim3(kThreads), 0, s, d, bs, c->dprimes(), c->tw.u64(),
                               c->twp.u64(), c->logN, *cout);
        else
            hipLaunchKernelGGL(k_fwd_rows, grid, dim3(kThreads), 0, s, d, bs, map, c->dprimes(), c->tw.u64(),
                               c->twp.u64(), c->logN, lo, hi, 0, 0, 0);
    }
    CKC_HIP(hipGetLastError());
    return CKC_OK;
}

int ntt_modup(const ckc_ctx *c, uint64_t *digits, int level, int nb, const uint64_t *coeff, size_t coeff_bs,
              const uint64_t *x, size_t xs, const BconvTable *const *tabs, hipStream_t s, const Ptrs *xp,
              size_t x_off) {
    if (nb <= 0) return CKC_OK;
    CKC_REQUIRE(c->logN >= 12 && c->logN <= 16, CKC_EUNSUPPORTED, "NTT supports 2^12 <= N <= 2^16");
    const int nl = level + 1, nt = nl + c->np, alpha = c->alpha, dnum = c->dnum_at(level);
    CKC_REQUIRE(dnum <= kMaxDnum && alpha <= kMaxBconv, CKC_EUNSUPPORTED, "too many key-switching digits");
    const size_t N = c->N, dig_bs = size_t(dnum) * nt * N;
    const int nfull = nl / alpha, last = nl - nfull * alpha;  // a partial last digit of `last` primes
    const LimbMap ext{nl, c->nq};
    {
        // algorithmic bytes, per digit: its source limbs read, its own limbs
        // read and written (copied), every other limb written once
        const double W = 8.0 * double(N) * nb;
        const double active = double(dnum) * nt - nl;  // limbs transformed (a digit's own limbs are copied)
        CKC_PROF(PK_NTT_FWD, s, W * (2.0 * nl + double(dnum) * nt), 0.5 * double(N) * c->logN * active * nb);
        if (nfull > 0) {
            DigitsIn d{coeff, coeff_bs, x, xs, nfull, nt, {}, {}, {}, xp ? *xp : Ptrs{}, x_off, xp ? 1 : 0};
            for (int j = 0; j < nfull; ++j) {
                d.hat[j] = tabs[j]->hat.u64();
                d.neg_s[j] = tabs[j]->neg_s.u64();
                d.s_half[j] = tabs[j]->s_half.u64();
            }
            using DigFn = void (*)(uint64_t *, size_t, LimbMap, const Prime *, const uint64_t *, const uint64_t *,
                                   int, DigitsIn);
            static constexpr DigFn fns[kMaxBconv] = {
                k_fwd_cols_bconv_dig<1>, k_fwd_cols_bconv_dig<2>, k_fwd_cols_bconv_dig<3>, k_fwd_cols_bconv_dig<4>,
                k_fwd_cols_bconv_dig<5>, k_fwd_cols_bconv_dig<6>, k_fwd_cols_bconv_dig<7>, k_fwd_cols_bconv_dig<8>};
            hipLaunchKernelGGL(fns[alpha - 1], dim3(unsigned(N / kElems), unsigned(nt), unsigned(nb * nfull)),
                               dim3(kThreads), 0, s, digits, dig_bs, ext, c->dprimes(), c->tw.u64(), c->twp.u64(),
                               c->logN, d);
        }
        if (last > 0) {
            const int j = nfull, lo = j * alpha;
            const BconvIn in{coeff + size_t(lo) * N, coeff_bs, last, tabs[j]->hat.u64(), tabs[j]->neg_s.u64(),
                             tabs[j]->s_half.u64(), x, xs, lo, lo + last, xp ? *xp : Ptrs{}, x_off, xp ? 1 : 0};
            using BconvFn = void (*)(uint64_t *, size_t, LimbMap, const Prime *, const uint64_t *, const uint64_t *,
                                     int, BconvIn);
            static constexpr BconvFn fns[kMaxBconv] = {k_fwd_cols_bconv<1>, k_fwd_cols_bconv<2>, k_fwd_cols_bconv<3>,
                                                       k_fwd_cols_bconv<4>, k_fwd_cols_bconv<5>, k_fwd_cols_bconv<6>,
                                                       k_fwd_cols_bconv<7>, k_fwd_cols_bconv<8>};
            hipLaunchKernelGGL(fns[last - 1], dim3(unsigned(N / kElems), unsigned(nt), unsigned(nb)), dim3(kThreads),
                               0, s, digits + size_t(j) * nt * N, dig_bs, ext, c->dprimes(), c->tw.u64(),
                               c->twp.u64(), c->logN, in);
        }
        // the second pass of every digit of every input in one launch
        hipLaunchKernelGGL(k_fwd_rows, dim3(unsigned(N / kElems), unsigned(nt), unsigned(nb * dnum)),
                           dim3(kThreads), 0, s, digits, size_t(nt) * N, ext, c->dprimes(), c->tw.u64(),
                           c->twp.u64(), c->logN, -1, -1, dnum, alpha, nl);
    }
    CKC_HIP(hipGetLastError());
    return CKC_OK;
}

int ntt_forward(const ckc_ctx *c, uint64_t *d, int nlimbs, LimbMap map, int nbatch, size_t batch_stride,
                hipStream_t s, int skip_lo, int skip_hi) {
    return ntt_forward_ex(c, d, nlimbs, map, nbatch, batch_stride, s, skip_lo, skip_hi, nullptr, nullptr);
}

int ntt_inverse(const ckc_ctx *c, uint64_t *d, int nlimbs, LimbMap map, int nbatch, size_t batch_stride,
                hipStream_t s, const uint64_t *scale2, const uint64_t *src, size_t src_bs) {
    if (nlimbs <= 0 || nbatch <= 0) return CKC_OK;
    CKC_REQUIRE(c->logN >= 12 && c->logN <= 16, CKC_EUNSUPPORTED, "NTT supports 2^12 <= N <= 2^16");
    const dim3 grid(unsigned(c->N / kElems), unsigned(nlimbs), unsigned(nbatch));
    CKC_PROF(PK_NTT_INV, s, 16.0 * double(c->N) * nlimbs * nbatch, 0.5 * double(c->N) * c->logN * nlimbs * nbatch);
    hipLaunchKernelGGL(k_inv_rows, grid, dim3(kThreads), 0, s, d, batch_stride, src ? src : d,
                       src ? src_bs : batch_stride, map, c->dprimes(), c->itw.u64(), c->itwp.u64(), c->logN, Ptrs{},
                       size_t(0), 0);
    hipLaunchKernelGGL(k_inv_cols, grid, dim3(kThreads), 0, s, d, batch_stride, map, c->dprimes(), c->itw.u64(),
                       c->itwp.u64(), c->ninv.u64(), scale2, c->logN);
    CKC_HIP(hipGetLastError());
    return CKC_OK;
}

int ntt_inverse_ptrs(const ckc_ctx *c, uint64_t *d, int nlimbs, LimbMap map, int nbatch, size_t batch_stride,
                     hipStream_t s, const uint64_t *scale2, const Ptrs &src, size_t src_off) {
    if (nlimbs <= 0 || nbatch <= 0) return CKC_OK;
    CKC_REQUIRE(c->logN >= 12 && c->logN <= 16, CKC_EUNSUPPORTED, "NTT supports 2^12 <= N <= 2^16");
    CKC_REQUIRE(nbatch <= kMaxBatch, CKC_EINVAL, "ntt_inverse_ptrs: at most 64 inputs");
    const dim3 grid(unsigned(c->N / kElems), unsigned(nlimbs), unsigned(nbatch));
    CKC_PROF(PK_NTT_INV, s, 16.0 * double(c->N) * nlimbs * nbatch, 0.5 * double(c->N) * c->logN * nlimbs * nbatch);
    hipLaunchKernelGGL(k_inv_rows, grid, dim3(kThreads), 0, s, d, batch_stride, d, batch_stride, map, c->dprimes(),
                       c->itw.u64(), c->itwp.u64(), c->logN, src, src_off, 1);
    hipLaunchKernelGGL(k_inv_cols, grid, dim3(kThreads), 0, s, d, batch_stride, map, c->dprimes(), c->itw.u64(),
                       c->itwp.u64(), c->ninv.u64(), scale2, c->logN);
    CKC_HIP(hipGetLastError());
    return CKC_OK;
}
