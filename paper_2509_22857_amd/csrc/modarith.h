// Exact modular arithmetic on 64-bit RNS words for gfx950.
//
// Every prime q satisfies q < 2^62, so sums of two residues never wrap and
// Shoup products land in [0, 2q).  All reductions are integer VALU work; no
// floating point touches a residue.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define CKC_HD __host__ __device__ __forceinline__

struct u128v {
    uint64_t lo, hi;
};

CKC_HD uint64_t mulhi64(uint64_t a, uint64_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __umul64hi(a, b);
#else
    return (uint64_t)(((unsigned __int128)a * b) >> 64);
#endif
}

CKC_HD u128v mul64x64(uint64_t a, uint64_t b) {
    u128v r;
    r.lo = a * b;
    r.hi = mulhi64(a, b);
    return r;
}

CKC_HD u128v add128(u128v x, u128v y) {
    u128v r;
    r.lo = x.lo + y.lo;
    r.hi = x.hi + y.hi + (r.lo < x.lo ? 1ull : 0ull);
    return r;
}

// Carry-counted accumulator of products of residues < 2^62 (device only):
//   value = l + cl 2^64 + (m + cm 2^64) 2^32 + h 2^64.
// A product a b with a = a1 2^32 + a0, b = b1 2^32 + b0 (a1, b1 < 2^30) adds
// a0 b0 into l, a0 b1 and a1 b0 into m and a1 b1 into h, each with one
// 32x32+64 multiply-add; the carry out of every multiply-add into l or m is
// added to cl or cm (the multiply-add's own carry output feeds an add-with-
// carry), so one product costs four multiply-adds and three adds.  With
// k-bit residues every product is below 2^(2k), so up to prod_cap(k)
// products plus one reduced residue keep the value below 2^128.
// The seven instructions form one block: the four multiply-adds come first,
// each with its own carry register pair, and every add-with-carry reads its
// carry at least two instructions after it was written, the distance gfx950
// requires between a vector write of a scalar register and a vector read of
// it as carry-in; no instruction depends on the one right before it (measured:
// 5.1 T products/s from registers, 5 % above the order with the two
// multiply-adds into m back to back).  Nothing the block writes to a scalar register outlives it,
// so the compiler has no hazard to pad around it.
struct accc {
    uint64_t h, m, l;
    uint32_t cm, cl;
};
__device__ __forceinline__ void macc(accc &acc, uint64_t a, uint64_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
    const uint32_t a0 = uint32_t(a), a1 = uint32_t(a >> 32), b0 = uint32_t(b), b1 = uint32_t(b >> 32);
    uint64_t c1, c2, c3, j;
    asm("v_mad_u64_u32 %0, %5, %9, %11, %0\n\t"
        "v_mad_u64_u32 %1, %6, %9, %12, %1\n\t"
        "v_mad_u64_u32 %2, %8, %10, %12, %2\n\t"
        "v_mad_u64_u32 %1, %7, %10, %11, %1\n\t"
        "v_addc_co_u32_e64 %4, %8, %4, 0, %6\n\t"
        "v_addc_co_u32_e64 %3, %8, %3, 0, %5\n\t"
        "v_addc_co_u32_e64 %4, %8, %4, 0, %7"
        : "+v"(acc.l), "+v"(acc.m), "+v"(acc.h), "+v"(acc.cl), "+v"(acc.cm), "=&s"(c1), "=&s"(c2), "=&s"(c3),
          "=&s"(j)
        : "v"(a0), "v"(a1), "v"(b0), "v"(b1));
#endif
}
CKC_HD u128v accc_value(const accc &a) {
    const uint64_t ml = a.m << 32;
    u128v r;
    r.lo = a.l + ml;
    r.hi = a.h + a.cl + (a.m >> 32) + (uint64_t(a.cm) << 32) + (r.lo < ml ? 1ull : 0ull);
    return r;
}

// largest number of products (plus one reduced residue) an accumulator may
// take for a k-bit modulus
CKC_HD int prod_cap(int k) { return k >= 61 ? (1 << (128 - 2 * k)) - 1 : 64; }

// Only h can overflow: l and m count their carries.  Since the value is only
// needed mod q, a fold replaces the value V = V_hi 2^64 + V_lo by V_lo +
// V_hi (2^64 mod q): l = V_lo and one more product, V_hi times r = 2^64 mod q,
// into an otherwise cleared accumulator, which leaves h below 2^62.  Every
// product adds less than 2^(2k - 64) to h, so fold_cap(k) products may
// follow a fold while h stays below 2^64 - 2^53, which leaves room in
// accc_value for carry counts up to 2^20 (k <= 62, the largest modulus size
// the library takes: at least 3).  A fold costs about two products, against
// about eight for a full reduction; with every field but l restarting from
// zero, the compiler can keep the accumulators in as few registers as with a
// reduction.
CKC_HD int fold_cap(int k) {
    if (k <= 32) return 1 << 20;
    const uint64_t room = ~uint64_t(0) - (uint64_t(1) << 53) - (uint64_t(1) << 62);
    const uint64_t n = room >> (2 * k - 64);
    return n > (1u << 20) ? 1 << 20 : int(n);
}
__device__ __forceinline__ accc macc_folded(const accc &acc, uint64_t r64) {
    const u128v v = accc_value(acc);
    accc f{0, 0, v.lo, 0, 0};
    macc(f, v.hi, r64);
    return f;
}

// Per-prime constants.
struct Prime {
    uint64_t q;
    uint64_t mu;    // floor(2^(2k) / q), k = bit length of q (Barrett)
    uint64_t r2;    // 2^64 mod q
    uint64_t r2p;   // floor(r2 * 2^64 / q)   (Shoup companion of r2)
    uint64_t onep;  // floor(2^64 / q)        (Shoup companion of 1)
    uint64_t qinv;  // -q^-1 mod 2^64         (Montgomery reduction)
    int32_t k;      // bit length of q
    int32_t pad;
};

CKC_HD uint64_t add_mod(uint64_t a, uint64_t b, uint64_t q) {
    uint64_t s = a + b;
    return s >= q ? s - q : s;
}
CKC_HD uint64_t sub_mod(uint64_t a, uint64_t b, uint64_t q) {
    return a >= b ? a - b : a + q - b;
}
CKC_HD uint64_t neg_mod(uint64_t a, uint64_t q) { return a ? q - a : 0; }

// Barrett reduction of x < 2^(2k) (k = bit length of q <= 62) into [0, q).
CKC_HD uint64_t barrett128(u128v x, const Prime &P) {
    const int k = P.k;
    // x >> (k-1): < 2^(k+1)
    uint64_t x1 = (x.lo >> (k - 1)) | (x.hi << (65 - k));
    u128v t = mul64x64(x1, P.mu);
    // >> (k+1)
    uint64_t qh = (t.lo >> (k + 1)) | (t.hi << (63 - k));
    uint64_t r = x.lo - qh * P.q;
    if (r >= P.q) r -= P.q;
    if (r >= P.q) r -= P.q;
    return r;
}

CKC_HD uint64_t mul_mod(uint64_t a, uint64_t b, const Prime &P) {
    return barrett128(mul64x64(a, b), P);
}


// Shoup multiplication by a constant w (w < q) with w' = floor(w 2^64 / q).
// a may be any 64-bit word; result in [0, q).
CKC_HD uint64_t mul_shoup(uint64_t a, uint64_t w, uint64_t wp, uint64_t q) {
    uint64_t qh = mulhi64(a, wp);
    uint64_t r = a * w - qh * q;
    return r >= q ? r - q : r;
}
// Lazy variant: result in [0, 2q).
CKC_HD uint64_t mul_shoup_lazy(uint64_t a, uint64_t w, uint64_t wp, uint64_t q) {
    uint64_t qh = mulhi64(a, wp);
    return a * w - qh * q;
}

// Reduce any 128-bit value: hi*2^64 + lo = hi*(2^64 mod q) + lo  (mod q).
CKC_HD uint64_t reduce128(u128v x, const Prime &P) {
    uint64_t a = mul_shoup(x.hi, P.r2, P.r2p, P.q);
    uint64_t b = mul_shoup(x.lo, 1, P.onep, P.q);
    return add_mod(a, b, P.q);
}

// Montgomery reduction of a carry-counted sum: the representative in [0, q)
// of value * 2^-64 mod q, for a sum of at most NPROD products of residues
// (each below q^2 < q 2^62).  With m = lo * qinv mod 2^64, value + m q is a
// multiple of 2^64 whose quotient is hi + mulhi(m, q) + [lo != 0].  That
// quotient can exceed 2^64 (hi < NPROD q / 4 and mulhi(m, q) < q: for q near
// 2^62 and NPROD >= 12 the plain sum wraps), so hi is first brought below q
// by ceil(NPROD / 4) - 1 conditional subtractions (hi < (NPROD / 4) q); the
// quotient is then below 2q and one more subtraction finishes it.  Used where
// the sum's operands carry a factor 2^64 (evaluation keys are stored times
// 2^64 mod q).
template <int NPROD>
CKC_HD uint64_t redc_hi_lo(uint64_t hi, uint64_t lo, const Prime &P) {
#pragma unroll
    for (int i = 0; i < (NPROD + 3) / 4 - 1; ++i) hi = hi >= P.q ? hi - P.q : hi;
    const uint64_t m = lo * P.qinv;
    const uint64_t t = hi + mulhi64(m, P.q) + (lo != 0 ? 1ull : 0ull);
    return t >= P.q ? t - P.q : t;
}
template <int NPROD>
__device__ __forceinline__ uint64_t redc_accc(const accc &a, const Prime &P) {
    const u128v v = accc_value(a);
    return redc_hi_lo<NPROD>(v.hi, v.lo, P);
}

// Reduce an arbitrary 64-bit word into [0, q) (Shoup multiplication by 1).
CKC_HD uint64_t reduce64(uint64_t a, const Prime &P) { return mul_shoup(a, 1, P.onep, P.q); }
