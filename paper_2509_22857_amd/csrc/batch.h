// Batched building blocks: kernel-argument pointer tables and batched key
// switching shared by the layer kernels.
#pragma once
#include "ckc_internal.h"

// Up to kMaxBatch device pointers passed by value as a kernel argument (no
// host->device copy of pointer tables).
constexpr int kMaxBatch = 64;
struct Ptrs {
    uint64_t *p[kMaxBatch];
};

int copy_limbs(const uint64_t *src, size_t src_ps, uint64_t *dst, size_t dst_ps, size_t words, int npoly,
               hipStream_t s);

// Fast basis conversion computing the input of a forward NTT (see
// ntt_forward_ex): output limb t, word i = sum_k src[b][k][i] hat[t ns + k]
// mod q_t, with src pre-scaled by (S/s_k)^-1 in coefficient form.
constexpr int kMaxBconv = 8;
constexpr int kMaxDnum = 16;  // key-switching digits
struct BconvIn {
    const uint64_t *src;   // [batch][ns][N]
    size_t src_bs;
    int ns;
    const uint64_t *hat;   // [limbs][ns]
    const uint64_t *neg_s; // [limbs] (-S) 2^64 mod t: centring correction
    const uint64_t *s_half;  // [ns] s_k >> 1
    const uint64_t *copy;  // limbs [copy_lo, copy_hi) come from here (NTT form), untransformed
    size_t copy_bs;
    int copy_lo, copy_hi;
    // with use_copyp, batch b's copied limbs come from copyp.p[b] + copy_off instead
    Ptrs copyp;
    size_t copy_off;
    int use_copyp;
};
// ModDown epilogue of a forward NTT over [2 nb][nl][N] (batch z = 2 b + p):
//   out_p.p[b][i][k] = (acc[z][i][k] - ntt[z][i][k]) P^-1 + add_p.p[b][i][perm0?(k)]
struct CombineOut {
    const uint64_t *acc;   // [z][nl][N] with batch stride acc_bs
    size_t acc_bs;
    const uint64_t *pinv;  // [nl][2]
    Ptrs add0, add1, out0, out1;
    int has_add0, has_add1;
    const uint32_t *perm0;  // applied to add0 only (may be null)
};
// Forward NTT of nbatch blocks of nlimbs limbs whose first pass may read a
// basis conversion (bin) and whose last pass may finish ModDown (cout)
// instead of storing the transform.
int ntt_forward_ex(const ckc_ctx *c, uint64_t *d, int nlimbs, LimbMap map, int nbatch, size_t bs, hipStream_t s,
                   int skip_lo, int skip_hi, const BconvIn *bin, const CombineOut *cout);

// ModUp's forward transforms of every digit of nb inputs: digits [b][dnum][nt][N]
// (nt = level + 1 + n_P), digit j converted from the pre-scaled coefficient-
// form limbs coeff[b][j alpha ..] (stride coeff_bs) by table tabs[j], its own
// limbs copied from the NTT-form input x[b] (stride xs).  One first-pass launch
// covers all full digits (a partial last digit has one of its own) and one
// second-pass launch covers every digit.
struct BconvTable;
int ntt_modup(const ckc_ctx *c, uint64_t *digits, int level, int nb, const uint64_t *coeff, size_t coeff_bs,
              const uint64_t *x, size_t xs, const BconvTable *const *tabs, hipStream_t s,
              const Ptrs *xp = nullptr, size_t x_off = 0);
// the inverse transform reading batch b's input from src.p[b] + src_off
int ntt_inverse_ptrs(const ckc_ctx *c, uint64_t *d, int nlimbs, LimbMap map, int nbatch, size_t batch_stride,
                     hipStream_t s, const uint64_t *scale2, const Ptrs &src, size_t src_off);

// dst (contiguous, stride dst_bs words) <- src.p[b] + src_off for b < nb, `words` words each.
int gather(const Ptrs &src, size_t src_off, uint64_t *dst, size_t dst_bs, size_t words, int nb, hipStream_t s);

// Batched ModUp of nb polynomials x[b] = x + b*xs (NTT form, level+1 limbs)
// into digits[b] = digits + b*dnum*nt*N, layout [dnum][nt][N] (NTT form).
int ks_modup_b(ckc_ctx *c, const uint64_t *x, size_t xs, int nb, int level, uint64_t *digits, hipStream_t s);
// the same with input b at xp.p[b] + x_off (no gathered copy)
int ks_modup_p(ckc_ctx *c, const Ptrs &xp, size_t x_off, int nb, int level, uint64_t *digits, hipStream_t s);

// Batched key inner product + ModDown.  For b < nb:
//   u = ModDown(sum_j sigma_g(digit_j[b]) * key_j)
//   out0.p[b] = u_0 + (add0 ? add0.p[b][perm(k)] : 0), out1.p[b] = u_1 + (add1 ? add1.p[b] : 0)
// perm is the NTT-domain permutation of g (g = 1: none); `perm_add0` applies
// the permutation to add0 as well (rotations add sigma_g(c0)).
int ks_apply_b(ckc_ctx *c, const uint64_t *digits, int nb, int level, const uint64_t *key, uint64_t g,
               const Ptrs *add0, const Ptrs *add1, bool perm_add0, const Ptrs &out0, const Ptrs &out1,
               hipStream_t s);

// Batched rescale: out.p[b] <- rescale(in.p[b]) (npoly polys at `level`); out must not alias in.
int rescale_b(ckc_ctx *c, const Ptrs &in, const Ptrs &out, int nb, int npoly, int level, hipStream_t s);

// Batched limb-wise op over whole ciphertexts: out.p[b] = a.p[b] op b.p[b] (npoly polys, nl limbs)
int ew_b(ckc_ctx *c, EwOp op, const Ptrs &out, const Ptrs &a, const Ptrs *b, int nb, int npoly, int nl,
         hipStream_t s);

// Hoisted rotations of nb 2-polynomial ciphertexts in.p[b] (NTT form, `level`):
// one ModUp per input shared by every step, then one batched key inner
// product + ModDown per nonzero step (the Galois key is read once for the
// batch).  dst[i].p[b] receives Rot_{steps[i]}(in.p[b]); step 0 is a copy.
int hoisted_group(ckc_ctx *c, const ckc_evk *evk, const Ptrs &in, int nb, int level, const std::vector<int32_t> &steps,
                  const std::vector<Ptrs> &dst, hipStream_t s);

// Double hoisting (convolutions): rotations kept in the extended basis Q u P.
// For every nonzero step i and input b, dst[i].p[b] ([2][l+1+n_P][N]) gets
//   (P sigma_g(c0) + u0, u1),  u = sum_j sigma_g(ModUp_j(c1)) * key_j,
// and for step 0 (P c0, P c1) on the Q limbs and zeros on the P limbs; one
// ModUp per input serves every step.
int hoisted_group_ext(ckc_ctx *c, const ckc_evk *evk, const Ptrs &in, int nb, int level,
                      const std::vector<int32_t> &steps, const std::vector<Ptrs> &dst, hipStream_t s);

// ModDown of n extended-basis ciphertexts y ([n][2][l+1+n_P][N], contiguous)
// into out0.p[b] / out1.p[b] (Q limbs), adding add0.p[b] (Q limbs, NTT form)
// to polynomial 0 when add0 is given; n <= kMaxBatch.
int moddown_b(ckc_ctx *c, const uint64_t *y, int n, int level, const Ptrs *add0, const Ptrs &out0, const Ptrs &out1,
              hipStream_t s);
