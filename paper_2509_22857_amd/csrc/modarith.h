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

// acc += a * b for residues a, b < 2^62.  With 32-bit halves a = a1 2^32 + a0
// (a1, b1 < 2^30) the middle sum a0 b1 + a1 b0 + (a0 b0 >> 32) < 2^63 cannot
// overflow, so the 128-bit product takes four 32x32->64 multiply-adds and no
// carry handling; one carry chain adds it to the accumulator.
CKC_HD void mac62(u128v &acc, uint64_t a, uint64_t b) {
    const uint32_t a0 = uint32_t(a), a1 = uint32_t(a >> 32), b0 = uint32_t(b), b1 = uint32_t(b >> 32);
    const uint64_t p00 = uint64_t(a0) * b0;
    uint64_t mid = uint64_t(a0) * b1 + (p00 >> 32);
    mid = uint64_t(a1) * b0 + mid;
    const uint64_t hi = uint64_t(a1) * b1 + (mid >> 32);
    const uint64_t lo = (mid << 32) | (p00 & 0xffffffffull);
    acc.lo += lo;
    acc.hi += hi + (acc.lo < lo ? 1ull : 0ull);
}

// Carry-free accumulator of products of residues < 2^62: value =
// h 2^64 + m 2^32 + l, where l and m collect 32-bit halves (no overflow for
// 2^32 terms) and h the high words (< 2^(2k-64) + 2^32 each for k-bit
// residues, so up to prod_cap(k) terms fit).  One carry chain at the end.
struct acc3 {
    uint64_t h, m, l;
};
CKC_HD void mac3(acc3 &acc, uint64_t a, uint64_t b) {
    const uint32_t a0 = uint32_t(a), a1 = uint32_t(a >> 32), b0 = uint32_t(b), b1 = uint32_t(b >> 32);
    const uint64_t p00 = uint64_t(a0) * b0;
    uint64_t mid = uint64_t(a0) * b1 + (p00 >> 32);
    mid = uint64_t(a1) * b0 + mid;
    acc.h = uint64_t(a1) * b1 + acc.h + (mid >> 32);
    acc.m += mid & 0xffffffffull;
    acc.l += p00 & 0xffffffffull;
}
CKC_HD u128v acc3_value(const acc3 &a) {
    // l + m 2^32 + h 2^64
    u128v r;
    const uint64_t ml = a.m << 32, mh = a.m >> 32;
    r.lo = a.l + ml;
    r.hi = a.h + mh + (r.lo < ml ? 1ull : 0ull);
    return r;
}
// largest number of products (plus one reduced residue) an accumulator may
// take for a k-bit modulus
CKC_HD int prod_cap(int k) { return k >= 61 ? (1 << (128 - 2 * k)) - 1 : 64; }

// Per-prime constants.
struct Prime {
    uint64_t q;
    uint64_t mu;    // floor(2^(2k) / q), k = bit length of q (Barrett)
    uint64_t r2;    // 2^64 mod q
    uint64_t r2p;   // floor(r2 * 2^64 / q)   (Shoup companion of r2)
    uint64_t onep;  // floor(2^64 / q)        (Shoup companion of 1)
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

// Reduce an arbitrary 64-bit word into [0, q) (Shoup multiplication by 1).
CKC_HD uint64_t reduce64(uint64_t a, const Prime &P) { return mul_shoup(a, 1, P.onep, P.q); }
