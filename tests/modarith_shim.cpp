// Host build of the library's Montgomery reduction (modarith.h), so the
// bounds tests run the same code the kernels inline.
#include "../paper_2509_22857_amd/csrc/modarith.h"

template <int N>
static uint64_t red(uint64_t hi, uint64_t lo, const Prime &P) {
    return redc_hi_lo<N>(hi, lo, P);
}

extern "C" uint64_t shim_redc(int nprod, uint64_t hi, uint64_t lo, uint64_t q, uint64_t qinv) {
    Prime P{};
    P.q = q;
    P.qinv = qinv;
    switch (nprod) {
        case 1: return red<1>(hi, lo, P);
        case 2: return red<2>(hi, lo, P);
        case 3: return red<3>(hi, lo, P);
        case 4: return red<4>(hi, lo, P);
        case 5: return red<5>(hi, lo, P);
        case 6: return red<6>(hi, lo, P);
        case 7: return red<7>(hi, lo, P);
        case 8: return red<8>(hi, lo, P);
        case 9: return red<9>(hi, lo, P);
        case 10: return red<10>(hi, lo, P);
        case 11: return red<11>(hi, lo, P);
        case 12: return red<12>(hi, lo, P);
        case 13: return red<13>(hi, lo, P);
        case 14: return red<14>(hi, lo, P);
        case 15: return red<15>(hi, lo, P);
        case 16: return red<16>(hi, lo, P);
        case 17: return red<17>(hi, lo, P);
        case 64: return red<64>(hi, lo, P);
        case 65: return red<65>(hi, lo, P);
        default: return ~0ull;
    }
}

extern "C" int shim_fold_cap(int k) { return fold_cap(k); }

// the 128-bit value of a carry-counted accumulator
extern "C" void shim_accc_value(uint64_t h, uint64_t m, uint64_t l, uint32_t cm, uint32_t cl, uint64_t *hi,
                                uint64_t *lo) {
    const u128v v = accc_value(accc{h, m, l, cm, cl});
    *hi = v.hi;
    *lo = v.lo;
}
