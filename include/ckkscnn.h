/*
 * ckkscnn.h -- C-ABI of the gfx950 leveled RNS-CKKS evaluator for private CNN
 * inference with quadratic activations (arXiv 2509.22857).
 *
 * The problem statement (paper Section 2.1, Threat Model): a client holds an
 * input image and the CKKS secret key, encrypts the image and sends only the
 * ciphertext; the server holds a CNN with plaintext parameters, evaluates it
 * under leveled FHE without bootstrapping, and returns encrypted logits that
 * only the client decrypts.  The scheme is RNS-CKKS (Section 2.2): ring
 * Z_Q[X]/(X^N+1), Q = q_0 ... q_L as 64-bit RNS words, a special modulus P for
 * hybrid key switching, scale Delta, rescaling that drops one modulus.
 *
 * Conventions for every function below:
 *  - Return value: CKC_OK (0) or a negative error code.  On error the outputs
 *    are unspecified, the inputs are untouched, and ckc_last_error() returns a
 *    message (per thread).  Nothing throws across the ABI.
 *  - Ciphertext and plaintext buffers (ckc_ct.d, ckc_pt.d) are DEVICE memory
 *    owned by the caller, sized with ckc_ct_words / ckc_pt_words.  Layout is
 *    limb-major: [npoly][level+1][N] uint64, limb l reduced modulo q_l, every
 *    limb in NTT form (the library's evaluation order; use ckc_ntt with
 *    inverse=1 to obtain coefficient form).
 *  - Host arrays passed in are read before the call returns.
 *  - `stream` is a hipStream_t (may be NULL for the default stream).  All
 *    work is enqueued asynchronously on it unless a function says otherwise.
 *  - Handles (ckc_ctx, ckc_sk, ckc_evk, ckc_layer) are owned by the library
 *    and freed by their *_destroy function.  ctx, evk and layers are
 *    read-only after creation, so calls on different streams may share them.
 */
#ifndef CKKSCNN_H
#define CKKSCNN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    CKC_OK = 0,
    CKC_EINVAL = -1,      /* bad argument */
    CKC_ELEVEL = -2,      /* level too low, or levels that cannot be aligned */
    CKC_ESCALE = -3,      /* operand scales differ by more than 2^-30 relative */
    CKC_ENOKEY = -4,      /* missing relinearisation or Galois key */
    CKC_ENOMEM = -5,      /* device allocation failed */
    CKC_EDEVICE = -6,     /* HIP runtime error */
    CKC_ESHAPE = -7,      /* shape / layout mismatch */
    CKC_EUNSUPPORTED = -8 /* parameters outside what the kernels support */
};

typedef struct ckc_ctx ckc_ctx;     /* parameters and device tables */
typedef struct ckc_sk ckc_sk;       /* client secret key (ternary, host + device copy) */
typedef struct ckc_evk ckc_evk;     /* device-resident relinearisation + Galois keys */
typedef struct ckc_layer ckc_layer; /* device-resident conv / dense layer */
typedef struct ckc_plan ckc_plan;   /* a network's layer program (native runner) */

/* Ciphertext: d = device [npoly][level+1][N]; scale is the CKKS scale. */
typedef struct {
    uint64_t *d;
    int32_t level;
    int32_t npoly;
    double scale;
} ckc_ct;

/* Plaintext: d = device [level+1][N] (NTT form). */
typedef struct {
    uint64_t *d;
    int32_t level;
    double scale;
} ckc_pt;

const char *ckc_last_error(void);

/* ------------------------------------------------------------------ context
 * Section 2.2 and Appendix D: N = 2^log_n, moduli q_0..q_{n_q-1} (q_0 holds
 * the output, q_{n_q-1} is dropped first), special primes p_0..p_{n_p-1}.
 * Every modulus must be a prime < 2^62 with q = 1 mod 2N, all distinct.
 * alpha = primes per key-switching digit (dnum = ceil(n_q / alpha)); the
 * product of the special primes should exceed every digit's product for
 * small key-switching noise.  log_n in [12, 16].  Sums of products of
 * residues are accumulated without reduction, so dnum + 1, alpha and n_p must
 * each stay within what the largest modulus allows (2^(128 - 2k) - 1 products
 * for k-bit moduli of 61 bits or more, 64 below), and dnum <= 16: otherwise
 * CKC_EUNSUPPORTED.  Errors: CKC_EINVAL, CKC_EUNSUPPORTED, CKC_ENOMEM,
 * CKC_EDEVICE.
 */
int ckc_ctx_create(int log_n, const uint64_t *q, int n_q, const uint64_t *p, int n_p, int alpha,
                   ckc_ctx **out);
int ckc_ctx_destroy(ckc_ctx *ctx);
/* words (uint64) of a ciphertext at `level` with `npoly` polynomials */
size_t ckc_ct_words(const ckc_ctx *ctx, int level, int npoly);
size_t ckc_pt_words(const ckc_ctx *ctx, int level);
/* the same ciphertext size in bytes (8 ckc_ct_words) */
size_t ckc_ct_bytes(const ckc_ctx *ctx, int level, int npoly);
/* the primitive 2N-th root of unity the library uses for prime index t
 * (Q primes first, then P), and its NTT order: output index k of a forward
 * transform holds a(psi^(2*bitrev(k)+1)). */
uint64_t ckc_ctx_root(const ckc_ctx *ctx, int t);

/* ------------------------------------------------------------------ NTT
 * Negacyclic NTT over Z_q[X]/(X^N+1) (Section 2.2, NTT-based polynomial
 * arithmetic), in place.  d holds n_blocks blocks of n_limbs limbs (each N
 * words, contiguous); limb l of every block is taken modulo q_l.
 * inverse = 0: coefficient -> NTT form; inverse = 1: NTT -> coefficient form.
 */
int ckc_ntt(const ckc_ctx *ctx, uint64_t *d, int n_blocks, int n_limbs, int inverse, void *stream);

/* ------------------------------------------------------------------ keys
 * Client key generation (Section 2.1: the client holds the secret key).
 * Secret: ternary s from a counter-based SplitMix64 stream of `seed`.
 * Evaluation keys (server side, device resident): one relinearisation key
 * (s^2 -> s) and one Galois key per rotation step (left rotation of the
 * N/2 slots by steps[i], Section 2.2), hybrid key switching with the
 * special modulus P.  Step 0 and duplicate Galois elements are ignored.
 * Errors: CKC_EINVAL, CKC_ENOMEM, CKC_EDEVICE.
 */
int ckc_keygen(ckc_ctx *ctx, uint64_t seed, const int32_t *steps, int n_steps, ckc_sk **sk_out,
               ckc_evk **evk_out, void *stream);
/* add Galois keys for more rotation steps to an existing key set */
int ckc_evk_add_rotations(ckc_ctx *ctx, const ckc_sk *sk, ckc_evk *evk, const int32_t *steps, int n_steps,
                          void *stream);
int ckc_sk_destroy(ckc_sk *sk);
int ckc_evk_destroy(ckc_evk *evk);
size_t ckc_evk_bytes(const ckc_evk *evk);
/* A key group: the key set of every image of a batched layer call, so that
 * one call (ckc_eval_conv, _quad_act, _dense, _avgpool2) evaluates images of
 * different clients together -- the serving loop's continuous batching across
 * clients of one network.  keys: n_keys key sets of one context (the caller
 * keeps them alive while the group is used); key_of_img[i] (in [0, n_keys))
 * is the key set of image i of the call, which must then have exactly n_img
 * images (for pooling, n_img equal groups of ciphertexts).  The calls split
 * their key-switching batches where the key set changes and share every
 * other launch (the contraction over the layer's codebook); each image's
 * ciphertexts are the same as with its own key set alone.  Destroy with
 * ckc_evk_destroy (the member key sets are untouched); ckc_evk_bytes of a
 * group is 0.  The single-ciphertext and *_many entry points refuse groups.
 * Errors: CKC_EINVAL for null arguments, a key index out of range, a member
 * that is itself a group or key sets of different shapes. */
int ckc_evk_group_create(const ckc_evk *const *keys, int n_keys, const int32_t *key_of_img, int n_img,
                         ckc_evk **group);

/* ------------------------------------------------------------------ client
 * Encoding (Section 2.2): n <= N/2 real slot values (host array), scaled by
 * `scale`, rounded to integers, reduced modulo q_0..q_level, NTT form.
 * The remaining slots are zero.  out->d must hold ckc_pt_words(level).
 */
int ckc_encode(ckc_ctx *ctx, const double *slots, size_t n, int level, double scale, ckc_pt *out,
               void *stream);
/* Symmetric RLWE encryption (Section 2.2): ct = (-a s + m + e, a) over
 * q_0..q_{pt.level}; stream_id selects the PRNG streams of a and e and must
 * be unique per ciphertext under one key. */
int ckc_encrypt(ckc_ctx *ctx, const ckc_sk *sk, const ckc_pt *pt, uint64_t stream_id, ckc_ct *out,
                void *stream);
/* Client-side HW-layout packing and encryption of one image (Sections 5.1
 * and 5.3): chw is [C][H][W] (host, FP64); channel c becomes the ciphertext
 * out[c] at `level` and `scale`, with member mm's copy of the image in the
 * slot block [mm block, (mm + 1) block) and pixel (r, x) at slot
 * mm block + r row_stride + x (all ensemble members share the input
 * ciphertexts); every other slot is zero.  Channel c uses PRNG stream
 * stream_id + c.  The same as ckc_encode then ckc_encrypt per channel.
 * out[c].d must each hold ckc_ct_words(level, 2).
 * Errors: CKC_EINVAL if (H - 1) row_stride + W > block, row_stride < W or
 * members block > N/2; CKC_ELEVEL for a level out of range. */
int ckc_encode_encrypt_image(ckc_ctx *ctx, const ckc_sk *sk, const double *chw, int C, int H, int W, int members,
                             int block, int row_stride, int level, double scale, uint64_t stream_id, ckc_ct *out,
                             void *stream);
/* m = c0 + c1 s (+ c2 s^2 for 3-polynomial ciphertexts) at the ciphertext's level. */
int ckc_decrypt(ckc_ctx *ctx, const ckc_sk *sk, const ckc_ct *ct, ckc_pt *out, void *stream);
/* Decoding: limb q_0 of pt, centred, mapped to n real slot values divided by
 * pt->scale, written to the host array `slots`.  Synchronises `stream`. */
int ckc_decode(ckc_ctx *ctx, const ckc_pt *pt, double *slots, size_t n, void *stream);

/* ------------------------------------------------------------------ arithmetic
 * Section 2.2: slot-wise addition and multiplication, rotation, rescale.
 * Binary operations need equal levels and scales within 2^-30 (CKC_ELEVEL /
 * CKC_ESCALE).  `out` may alias an input unless stated otherwise.
 */
int ckc_add(ckc_ctx *ctx, const ckc_ct *a, const ckc_ct *b, ckc_ct *out, void *stream);
int ckc_sub(ckc_ctx *ctx, const ckc_ct *a, const ckc_ct *b, ckc_ct *out, void *stream);
/* add a plaintext (its level >= the ciphertext's; extra limbs ignored) */
int ckc_add_plain(ckc_ctx *ctx, const ckc_ct *a, const ckc_pt *p, ckc_ct *out, void *stream);
/* add round(value * a.scale) to every slot */
int ckc_add_const(ckc_ctx *ctx, const ckc_ct *a, double value, ckc_ct *out, void *stream);
/* multiply by a plaintext; result scale = a.scale * p.scale (no rescale) */
int ckc_mul_plain(ckc_ctx *ctx, const ckc_ct *a, const ckc_pt *p, ckc_ct *out, void *stream);
/* tensor product of two 2-polynomial ciphertexts -> 3 polynomials; out must not alias */
int ckc_tensor(ckc_ctx *ctx, const ckc_ct *a, const ckc_ct *b, ckc_ct *out, void *stream);
/* relinearise a 3-polynomial ciphertext (s^2 -> s) into a 2-polynomial one */
int ckc_relin(ckc_ctx *ctx, const ckc_evk *evk, const ckc_ct *in, ckc_ct *out, void *stream);

/* ckc_relin without any device allocation, for callers that cannot allocate
 * (code under HIP graph capture, serving loops that must not call hipMalloc).
 * Same arguments, kernels and results as ckc_relin (bit for bit).  Its scratch
 * is one static device array of ckc_noalloc_capacity() bytes (256 MiB), which
 * every GPU the library runs on holds until the process ends (its address is
 * looked up at the first call on each device, which allocates nothing);
 * ckc_relin_noalloc_bytes(ctx, level) gives the scratch a ciphertext at
 * `level` needs (8N[dnum (l+1+n_P) + 4(l+1) + 2 n_P]
 * bytes, each buffer rounded up to 256).  Nothing in the scratch needs to
 * start at zero.  Every call on one GPU shares that GPU's array: calls that
 * overlap on one GPU (other streams, other threads) race and must be
 * serialised by the caller.
 * Errors: as ckc_relin; CKC_ENOMEM if the level needs more scratch than the
 * array holds (nothing is launched). */
int ckc_relin_noalloc(ckc_ctx *ctx, const ckc_evk *evk, const ckc_ct *in, ckc_ct *out, void *stream);
size_t ckc_relin_noalloc_bytes(const ckc_ctx *ctx, int level);
size_t ckc_noalloc_capacity(void);

/* Hoisted rotations: one ModUp of in->c1 shared by every step; out[i] is the
 * left rotation of the slots by steps[i] (0 = copy).  The Galois
 * automorphism is applied after ModUp.  out[i] must not alias in. */
int ckc_rotate(ckc_ctx *ctx, const ckc_evk *evk, const ckc_ct *in, const int32_t *steps, int n_steps,
               ckc_ct *out, void *stream);
/* Rescale (Section 2.2): divide by q_level with rounding, drop that limb;
 * scale /= q_level.  out->d must not alias in->d. */
int ckc_rescale(ckc_ctx *ctx, const ckc_ct *in, ckc_ct *out, void *stream);
/* keep limbs q_0..q_to_level (value and scale unchanged) */
int ckc_mod_drop(ckc_ctx *ctx, const ckc_ct *in, int to_level, ckc_ct *out, void *stream);


/* ------------------------------------------------------------------ batches
 * Batched forms of rescale and addition (one launch per 64 ciphertexts).
 * ckc_rescale_many: out[i] = rescale(in[i]); out[i].d must not alias in[j].d.
 * ckc_add_many: out[i] = a[i] + b[i] (equal levels, scales within 2^-30;
 * out may alias a or b). */
int ckc_rescale_many(ckc_ctx *ctx, const ckc_ct *in, int n, ckc_ct *out, void *stream);
int ckc_add_many(ckc_ctx *ctx, const ckc_ct *a, const ckc_ct *b, int n, ckc_ct *out, void *stream);
/* Hoisted rotations of a batch (Section 2.2 rotation; the hoisting shares one
 * ModUp of c1 per input across every step):
 * out[i * n_steps + j] = left rotation of in[i] by steps[j] (0 = copy).
 * Inputs: 2-polynomial ciphertexts at one level with equal scales.  Every
 * Galois key is read once per 64 inputs.  out must not alias any input.
 * Errors: CKC_EINVAL, CKC_ELEVEL, CKC_ESHAPE, CKC_ESCALE, CKC_ENOKEY,
 * CKC_ENOMEM, CKC_EDEVICE. */
int ckc_rotate_many(ckc_ctx *ctx, const ckc_evk *evk, const ckc_ct *in, int n, const int32_t *steps, int n_steps,
                    ckc_ct *out, void *stream);
/* Ciphertext multiplication with relinearisation (Section 2.2; with a == b
 * the squaring of the quadratic activation, Section 2.3):
 * out[i] = Relin(a[i] (x) b[i]), scale a.scale * b.scale, level unchanged.
 * a and b: 2-polynomial ciphertexts at one level (scales may differ
 * between pairs); out[i] may alias a[i] or b[i].  CKC_ENOKEY without a
 * relinearisation key. */
int ckc_mul_relin_many(ckc_ctx *ctx, const ckc_evk *evk, const ckc_ct *a, const ckc_ct *b, int n, ckc_ct *out,
                       void *stream);
/* Plaintext multiply-accumulate (the ct x pt MAC of packed convolution and
 * dense layers, Section 5.1):
 * out[o] = sum_{t < n_terms} in[o * n_terms + t] * pt[t],  o < n_out,
 * 1 <= n_terms <= 64; inputs 2-polynomial at one level with equal scales,
 * plaintexts at that level or above (extra limbs ignored) with equal scales;
 * result scale = in.scale * pt.scale.  out must not alias any input. */
int ckc_mac_plain_many(ckc_ctx *ctx, const ckc_ct *in, const ckc_pt *pt, int n_terms, int n_out, ckc_ct *out,
                       void *stream);

/* ------------------------------------------------------------------ layers
 * HW layout (Section 5.1, Data Layout): every channel is its own
 * ciphertext.  Ensemble member m (Section 5.3) owns the slot block
 * [m*block, (m+1)*block); logical pixel (r, c) of a channel with valid grid
 * height x width sits at slot m*block + gap*(r*row_stride + c).  Convolution
 * and pooling leave gaps instead of re-packing (lazy mapping): the output of a
 * stride-s layer has gap*s.  Slots outside the valid grid hold values that
 * no consumer reads (every mask is zero there).
 *
 * flags & CKC_LAYOUT_SLICE_SHARED: the slice-shared layout (Section 5.2: the
 * weights of one kernel column across a layer's filters share an encoding).
 * Every member block keeps zero rows below its image -- at least gap*(height
 * + 1) rows of row_stride slots per block, so the row after the image and
 * the row before it (the previous block's last) read as zeros -- and a 3x3
 * weight's plaintext then masks only the columns: one plaintext per (kernel
 * column, centroid), shared by the column's three taps.  The spare rows stay
 * zero through the network because every layer writes only its grid there
 * (the activation places its constant term on the grid only).
 */
#define CKC_LAYOUT_SLICE_SHARED 1
typedef struct {
    int32_t block;      /* slots per ensemble member (power of two) */
    int32_t row_stride; /* slot distance of vertically adjacent pixels at gap 1 */
    int32_t gap;        /* current gap */
    int32_t height;     /* valid grid height */
    int32_t width;      /* valid grid width */
    int32_t members;    /* ensemble members packed side by side */
    int32_t flags;      /* CKC_LAYOUT_SLICE_SHARED or 0 */
} ckc_layout;

/*
 * Convolution layer, ksize in {1, 3}, 'same' zero padding, stride in {1, 2},
 * with clustered weights (Section 5.2, slice clustering; slice ensemble
 * clustering in Section 5.3).  codebook: [ksize][n_centroids][members] -- one codebook per kernel
 * column (a slice), each centroid a vector over the ensemble members; idx:
 * [out_ch][in_ch][ksize][ksize] centroid indices into the codebook of the
 * tap's column.  bias: [members][out_ch] or NULL.
 * Every (tap, centroid) pair is encoded once into a plaintext codebook at
 * `level` and scale pt_scale: the centroid's member values on the slots of
 * the output grid whose input pixel for that tap lies inside the image.  In
 * the slice-shared layout (in->flags & CKC_LAYOUT_SLICE_SHARED, 3x3 layers)
 * every (kernel column, centroid) pair is encoded once instead, on the
 * output slots whose input column lies inside the image, and the column's
 * three taps share it (a third of the plaintexts).
 * The bias plaintext is encoded at bias_scale on the output grid.
 * The layer copies every host array.  Errors: CKC_EINVAL, CKC_ESHAPE,
 * CKC_ENOMEM, CKC_EDEVICE.
 */
int ckc_layer_create_conv(ckc_ctx *ctx, const ckc_layout *in, int out_ch, int in_ch, int ksize, int stride,
                          int n_centroids, const double *codebook, const uint16_t *idx, const double *bias,
                          int level, double pt_scale, double bias_scale, ckc_layer **out, void *stream);

/*
 * Key-switching form of a layer's rotations (Section 2.2 hybrid key
 * switching behind the Section 5.1 rotations of a convolution).  Both share
 * one decomposition (ModUp) per input ciphertext; they differ in where the
 * ModDown happens, so their ciphertexts differ in the low bits while
 * decrypting to the same values within the key-switching noise:
 *   CKC_HOIST_DOUBLE: every rotated input stays in Q_l u P and the products
 *     with the codebook (encoded over Q_l u P) are summed there; one ModDown
 *     per output polynomial.  Fewer ModDowns; the contraction runs over
 *     l + 1 + n_P limbs.
 *   CKC_HOIST_SINGLE: every rotated input is brought back to Q_l (one ModDown
 *     per input and tap), then summed over l + 1 limbs.  Cheaper where the
 *     P limbs are a large share of the limbs (low levels).
 * 1x1 layers have no rotations and ignore the choice.
 */
enum { CKC_HOIST_SINGLE = 1, CKC_HOIST_DOUBLE = 2 };

/*
 * ckc_layer_create_conv with the key-switching form chosen explicitly
 * (ckc_layer_create_conv is this with CKC_HOIST_DOUBLE).  Errors as
 * ckc_layer_create_conv, and CKC_EINVAL for another hoisting value.
 */
int ckc_layer_create_conv_ex(ckc_ctx *ctx, const ckc_layout *in, int out_ch, int in_ch, int ksize, int stride,
                             int n_centroids, const double *codebook, const uint16_t *idx, const double *bias,
                             int level, double pt_scale, double bias_scale, int hoisting, ckc_layer **out,
                             void *stream);
/*
 * out[img][o] = sum_t sum_c PT[t][c] * (sum_{i : idx[o][i][t] = c} Rot_{step(t)}(in[img][i])) + bias_o
 * with step(t) = gap*(dh*row_stride + dw) for tap t = (dh, dw); one hoisted
 * rotation group per input ciphertext.  in: [n_img][in_ch] 2-poly
 * ciphertexts at the layer's level with equal scales; out: [n_img][out_ch]
 * caller buffers of ckc_ct_words(level, 2).  Result scale = in scale *
 * pt_scale, level unchanged (no rescale).  CKC_ENOKEY if a tap's Galois key
 * is missing.
 */
int ckc_eval_conv(ckc_ctx *ctx, const ckc_evk *evk, const ckc_layer *layer, const ckc_ct *in, int n_img,
                  ckc_ct *out, void *stream);

/*
 * Quadratic activation (Section 2.3; weight redistribution, Section 4.2,
 * makes it monic): y = x^2 + b x + c per (channel, member),
 * evaluated as t = x + b, y = Relin(x * t) + c.  b and c: [members][channels];
 * for members == 1 they are added as constant polynomials, otherwise as
 * block-constant plaintexts; in the slice-shared layout c is placed on the
 * layout's grid slots only (the spare rows stay zero).  The leading coefficient a_absorb is absorbed
 * into the scale: result scale = in_scale^2 / a_absorb (1.0 when the
 * coefficient was redistributed into the next layer).  Consumes no level.
 */
int ckc_layer_create_act(ckc_ctx *ctx, const ckc_layout *layout, int channels, const double *b, const double *c,
                         double a_absorb, int level, double in_scale, ckc_layer **out, void *stream);
int ckc_eval_quad_act(ckc_ctx *ctx, const ckc_evk *evk, const ckc_layer *layer, const ckc_ct *in, int n_img,
                      ckc_ct *out, void *stream);

/*
 * Dense layer after a global average pooling whose divisor is folded into
 * w (Section 4.2): for every input channel S_c = rotation-sum of in[c] over
 * the valid grid (steps gap*2^j, then gap*row_stride*2^j, ascending), then
 * out[k] = sum_c PT[k][c] * S_c + bias_k, where PT[k][c] holds w[m][k][c] in
 * slot m*block of member m.  w: [members][classes][in_ch]; bias:
 * [members][classes] or NULL.  Member m's logit for class k is slot m*block
 * of out[img][k].  Result scale = in scale * pt_scale.  With one member
 * only slot 0 is read, so PT[k][c] is the encoding of the constant vector
 * w[0][k][c] (the constant polynomial round(w * pt_scale)) and the bias the
 * constant round(bias * bias_scale); nothing per (class, channel) is stored
 * but those residues.
 */
int ckc_layer_create_dense(ckc_ctx *ctx, const ckc_layout *in, int classes, int in_ch, const double *w,
                           const double *bias, int level, double pt_scale, double bias_scale, ckc_layer **out,
                           void *stream);
/*
 * Dense layer over the flattened feature map (every grid position its own
 * weight; Section 5.1's lazy mapping leaves the map on the layout's grid):
 * out[k] = SUM over the valid grid (the same rotation steps as above) of
 * (sum_c PT[k][c] * in[c] + B[k]), where PT[k][c] holds w[m][k][c][r][col]
 * in slot m*block + gap*(r*row_stride + col) and B[k] holds bias[m][k] in
 * slot m*block, so member m's logit for class k is slot m*block of out[k].
 * w: [members][classes][in_ch][height][width] (the layout's grid); bias:
 * [members][classes] or NULL.  Result scale = in scale * pt_scale.  K x C
 * plaintexts and K bias plaintexts are stored; ckc_eval_dense evaluates it
 * (the products first, then K rotation sums instead of C).
 * Errors: as ckc_layer_create_dense.
 */
int ckc_layer_create_dense_spatial(ckc_ctx *ctx, const ckc_layout *in, int classes, int in_ch, const double *w,
                                   const double *bias, int level, double pt_scale, double bias_scale,
                                   ckc_layer **out, void *stream);
int ckc_eval_dense(ckc_ctx *ctx, const ckc_evk *evk, const ckc_layer *layer, const ckc_ct *in, int n_img,
                   ckc_ct *out, void *stream);

/* 2x2 sum pooling (average pooling with the divisor folded into the next
 * layer, Section 4.2): y = x + Rot_g x + Rot_{g*row_stride} x +
 * Rot_{g*(row_stride+1)} x; the output layout has gap 2g. */
int ckc_eval_avgpool2(ckc_ctx *ctx, const ckc_evk *evk, const ckc_layout *layout, const ckc_ct *in, int n,
                      ckc_ct *out, void *stream);

/* rotation steps a layer needs Galois keys for (returns the count; writes at
 * most max of them), and the layout of its output */
int ckc_layer_steps(const ckc_layer *layer, int32_t *steps, int max);
int ckc_layer_out_layout(const ckc_layer *layer, ckc_layout *out);
size_t ckc_layer_bytes(const ckc_layer *layer);
int ckc_layer_destroy(ckc_layer *layer);

/* ------------------------------------------------------------------ profiling
 * Opt-in launch timing for measurement: while enabled, the library records a
 * HIP event pair around every launch of the named kernel classes ("ntt_fwd",
 * "ntt_inv", "kip", "conv_contract", "act_tensor", "rescale", "dense_mac",
 * "ew", "mac_plain", "tensor", "copy"; "bconv" and "moddown" run inside the
 * forward NTT and record nothing of their own) on the stream the kernel runs
 * on, together with the algorithmic bytes (each word read or written once)
 * and work (butterflies for the NTT, 64-bit products for the key inner
 * product and the multiply-accumulates) of the launch.
 * ckc_prof_enable clears the records; ckc_prof_query waits for the recorded
 * events and sums them for one class. */
int ckc_prof_enable(int on);
int ckc_prof_query(const char *kernel, int64_t *launches, double *total_ms, double *bytes, double *work);

/* Opt-in count of launches per kernel instantiation, so that a test can check
 * which variant of a kernel a call ran.  Names are the kernel's base name with
 * its template arguments and launch options, e.g. "conv_mac<8,4>+dbuf+fused"
 * (contraction, 8 outputs per wave, 4 images per workgroup, double-buffered
 * codebook tiles, all output groups in one launch), "conv_contract" (grouped
 * form), "kip_ext_rot<7>" (extended key inner product of a rotation group,
 * 7 digits; <0> is the generic digit count), "kip_ext<d>", "kip_b<d>".
 * ckc_variant_enable(on) clears the counts and turns counting on or off;
 * ckc_variant_count gives the launches counted for one name (0 if none);
 * ckc_variant_list writes "name=count" lines into buf.
 * Errors: CKC_EINVAL for null arguments or a list longer than cap bytes. */
int ckc_variant_enable(int on);
int ckc_variant_count(const char *name, int64_t *launches);
int ckc_variant_list(char *buf, size_t cap);

/* ------------------------------------------------------------------ tuning
 * Launch choices picked by an autotuner (process-wide; every choice gives
 * bit-identical results, only the speed differs):
 *   "conv_outs"  outputs per wave of the convolution contraction: 8 or 16
 *   "conv_imgs"  most images per contraction workgroup: 1, 2 or 4
 *   "ks_batch"   rotated inputs per key-switching launch in a convolution,
 *                8 .. 64
 *   "conv_fuse"  1: one contraction launch covers every output group of a 3x3
 *                layer (the groups of one coefficient tile share an XCD's
 *                L2); 0: one launch per output group
 *   "conv_rows"  polynomials per contraction wave: 1, or 2 (each codebook
 *                word read from LDS serves both polynomials' products)
 * Errors: CKC_EINVAL for an unknown knob or a value it does not allow. */
int ckc_tune_set(const char *knob, int value);
int ckc_tune_get(const char *knob, int *value);

/* ------------------------------------------------------------------ runner
 * Native execution of a whole network.  ckc_batch_plan parses the network's
 * layer program (JSON) once, over the layer handles it names by index:
 *   {"input": {"name": "x", "count": C, "level": L},
 *    "output": "<tensor>",
 *    "steps": [{"op": "conv" | "act" | "dense" | "pool", "in": "<tensor>",
 *               "out": "<new tensor>", "count": <ciphertexts per image>,
 *               "level": <level the layer runs at>, "layer": <index>,
 *               "rescale": 0 | 1,
 *               "short": {"layer": <1x1 conv index>, "in": "<tensor>",
 *                         "level": <its level>},          (conv, optional)
 *               "layout": {"block", "row_stride", "gap", "height", "width",
 *                          "members"}},                   (pool)
 *              ...]}
 * A step evaluates its layer on every image (ckc_eval_conv / _quad_act /
 * _dense / _avgpool2); a shortcut's input is mod-dropped to its level, taken
 * through its 1x1 convolution and added to the step's output (residual,
 * Section 4.3); "rescale" rescales the result once.  Tensors are written once
 * and freed after their last reader.  The plan keeps the layer handles (the
 * caller keeps them alive) and the ctx.
 * ckc_batch_run evaluates the plan for n_requests images: inputs[r] holds
 * request r's `count` input ciphertexts at the input level, outputs[r] the
 * caller's buffers for the output tensor (ckc_batch_plan_info gives its count
 * and level); consecutive requests with the same key set run as one batched
 * pass.  Intermediate ciphertexts are allocated on `stream`.
 * Errors: CKC_EINVAL for a malformed program or null arguments; CKC_ELEVEL
 * for inconsistent levels; any error of the layer calls, after which the
 * outputs are unspecified. */
int ckc_batch_plan(ckc_ctx *ctx, const char *network_json, ckc_layer *const *layers, int n_layers,
                   ckc_plan **plan_out);
int ckc_batch_plan_info(const ckc_plan *plan, int *in_count, int *in_level, int *out_count, int *out_level);
int ckc_batch_plan_destroy(ckc_plan *plan);
int ckc_batch_run(ckc_plan *plan, const ckc_evk *const *evks, ckc_ct *const *inputs, int n_requests,
                  ckc_ct *const *outputs, void *stream);

/* ------------------------------------------------------------------ memory
 * Scratch memory (rotated inputs, digits, key-switching buffers) comes from
 * one growable arena per (device, stream) that keeps its largest size so that
 * steady-state calls allocate nothing.  ckc_stream_release frees the arena of
 * `stream` (a hipStream_t; NULL = the default stream) on the current device
 * after waiting for the work queued on it, and returns what the device's
 * default memory pool caches (overflow buffers) to the device; the next call
 * on the stream grows a new arena.  For callers that bound device memory per stream, such as a
 * serving loop releasing a finished batch's stream.  ckc_stream_reserve
 * grows the stream's arena to at least `bytes` now (one allocation), so that
 * the calls of a batch whose scratch peak the caller knows allocate nothing
 * while it runs.  Neither is to be called while another thread has a call
 * running on the same stream.
 * Errors: CKC_EINVAL if a call on the stream still holds scratch;
 * CKC_ENOMEM if the reservation cannot be allocated; CKC_EDEVICE on a HIP
 * error. */
int ckc_stream_release(void *stream);
int ckc_stream_reserve(void *stream, size_t bytes);

/* ------------------------------------------------------------------ testing
 * Test-only fault injection, for callers' failure handling (a serving loop
 * that must retire a failed batch and go on): the call_index-th following
 * call of a layer evaluation entry point (ckc_eval_conv, ckc_eval_quad_act,
 * ckc_eval_dense, ckc_eval_avgpool2; counted process-wide from 1) returns
 * `code` (a negative CKC_ error) at once, before touching any buffer or
 * launching anything; once.  call_index 0 disarms.
 * Errors: CKC_EINVAL for a negative index or a non-negative code. */
int ckc_set_test_fault(int call_index, int code);

#ifdef __cplusplus
}
#endif
#endif /* CKKSCNN_H */
