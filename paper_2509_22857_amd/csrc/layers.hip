// CNN layers over the HW layout: clustered convolution, quadratic
// activation, dense layer with rotation sums, 2x2 sum pooling.
//
// Convolution (Sections 5.1-5.3): for every input channel one hoisted group
// of rotations yields R[i][t] = Rot_{step(t)}(x_i) for the taps t of the
// kernel.  Weights are clustered per kernel column, so the layer stores one
// plaintext per (tap, centroid) -- the centroid's per-member values on the
// output slots whose input pixel is inside the image.  The contraction
//   y_o = sum_t sum_c PT[t][c] * (sum_{i : idx[o][i][t] = c} R[i][t]) + bias_o
// adds the rotated inputs that share a centroid before the single plaintext
// product, which is exact ring arithmetic (the same residues as multiplying
// every weight separately).
#include <math.h>
#include <stdlib.h>

#include <algorithm>
#include <vector>

#include "batch.h"
#include "prof.h"
#include "tune.h"

int encode_impl(ckc_ctx *c, const double *slots_h, size_t nslots, int level, double scale, uint64_t *m,
                hipStream_t s, bool ext = false);
uint64_t galois_element(const ckc_ctx *c, int64_t step);

enum LayerKind { LK_CONV = 0, LK_ACT = 1, LK_DENSE = 2 };

struct ckc_layer {
    int kind = 0;
    ckc_layout lin{}, lout{};
    int level = 0;
    // conv
    int O = 0, I = 0, ksz = 0, stride = 1, ntap = 0, kcent = 0;
    double pt_scale = 1.0, bias_scale = 1.0;
    bool has_bias = false;
    std::vector<int32_t> tap_step;
    DevMem pts;                        // conv: [npt][kcent][nl][N]; dense: [K][C][nl][N]
    int npt = 0;                       // conv plaintext sets: one per tap, or one per kernel column
    bool pt_shared = false;            // slice-shared layout: tap t uses the set of its column t % 3
    DevMem bias;                       // conv: [O][nl][N]; dense: [K][nl][N]
    DevMem og_off, g_c, g_moff, m_i;   // conv group lists (grouped form, any codebook size)
    DevMem ioff;                       // conv: [ntap][Opad/4][I] codebook row byte offsets, 16 bits each (direct form)
    bool ext = false;                  // conv with rotations: codebook over Q_l u P, one ModDown per output
    int Opad = 0;
    // act
    int C = 0;
    double a_absorb = 1.0, in_scale = 1.0;
    DevMem bpt, cpt;                   // [C][nl][N] NTT-form plaintexts (constants or block-constant vectors)
    // dense
    int K = 0;
    bool spatial = false;              // weights per grid position: products first, slot sums of the K outputs
    std::vector<int32_t> sum_steps;
    DevMem dconst, bconst;             // dense with one member: [K][C][nl] and [K][nl] constant residues
    size_t bytes = 0;
};

namespace {

hipStream_t S(void *s) { return (hipStream_t)s; }
unsigned tiles(size_t N) { return unsigned(std::min<size_t>(N / 256, 64)); }

bool is_pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }

int check_layout(const ckc_ctx *c, const ckc_layout *L) {
    CKC_REQUIRE(L, CKC_EINVAL, "null layout");
    CKC_REQUIRE(is_pow2(L->block) && L->members >= 1 && size_t(L->block) * L->members <= c->N / 2, CKC_ESHAPE,
                "layout: block must be a power of two with members*block <= N/2");
    CKC_REQUIRE(L->gap >= 1 && L->height >= 1 && L->width >= 1 && L->row_stride >= L->width, CKC_ESHAPE,
                "layout: bad grid");
    const int64_t last = int64_t(L->gap) * (int64_t(L->row_stride) * (L->height - 1) + (L->width - 1));
    CKC_REQUIRE(last < L->block, CKC_ESHAPE, "layout: grid does not fit in a block");
    CKC_REQUIRE((L->flags & ~CKC_LAYOUT_SLICE_SHARED) == 0, CKC_EINVAL, "layout: unknown flags");
    if (L->flags & CKC_LAYOUT_SLICE_SHARED) {
        // the row below the image and the row above it (the previous block's
        // last) must be spare rows, which hold zeros
        CKC_REQUIRE(L->block % L->row_stride == 0 &&
                        int64_t(L->block / L->row_stride) >= int64_t(L->gap) * (L->height + 1),
                    CKC_ESHAPE, "layout: the slice-shared layout needs gap*(height+1) rows per block");
    }
    return CKC_OK;
}

size_t slot_of(const ckc_layout &L, int m, int r, int col) {
    return size_t(m) * L.block + size_t(L.gap) * (size_t(r) * L.row_stride + col);
}

// constant polynomial value*scale (rounded) in NTT form: the same residue at every point
void const_residues(const ckc_ctx *c, double value, double scale, int nl, std::vector<uint64_t> &out) {
    const double v = round(value * scale);
    out.resize(nl);
    for (int t = 0; t < nl; ++t) {
        const uint64_t q = c->mods[t];
        const double av = fabs(v);
        uint64_t r;
        if (av < 9.2e18) {
            r = uint64_t(av) % q;
        } else {
            int e;
            const double mant = frexp(av, &e);
            const uint64_t M = uint64_t(ldexp(mant, 53));
            uint64_t pw = 1, base = 2 % q;
            unsigned ex = unsigned(e - 53);
            while (ex) {
                if (ex & 1) pw = (uint64_t)(((unsigned __int128)pw * base) % q);
                base = (uint64_t)(((unsigned __int128)base * base) % q);
                ex >>= 1;
            }
            r = (uint64_t)(((unsigned __int128)(M % q) * pw) % q);
        }
        out[t] = (v < 0 && r) ? q - r : r;
    }
}

__global__ void k_fill_limbs(uint64_t *__restrict__ d, const uint64_t *__restrict__ vals, int nl, int logN) {
    const int t = blockIdx.y;
    const size_t N = size_t(1) << logN;
    const uint64_t v = vals[t];
    for (size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x; k < N; k += size_t(gridDim.x) * blockDim.x)
        d[size_t(t) * N + k] = v;
}

int fill_const_pt(ckc_ctx *c, uint64_t *d, double value, double scale, int nl, hipStream_t s) {
    std::vector<uint64_t> r;
    const_residues(c, value, scale, nl, r);
    DevBuf rb;
    CKC_TRY(rb.alloc(8 * nl, s));
    CKC_HIP(hipMemcpyAsync(rb.p, r.data(), 8 * nl, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_fill_limbs, dim3(tiles(c->N), unsigned(nl)), dim3(256), 0, s, d, rb.u64(), nl, c->logN);
    CKC_HIP(hipGetLastError());
    CKC_HIP(hipStreamSynchronize(s));
    return CKC_OK;
}

__global__ void k_scatter(const uint64_t *__restrict__ src, size_t src_bs, Ptrs dst, size_t words) {
    const int b = blockIdx.y;
    const uint64_t *sp = src + b * src_bs;
    uint64_t *d = dst.p[b];
    for (size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x; k < words; k += size_t(gridDim.x) * blockDim.x)
        d[k] = sp[k];
}

// ----------------------------------------------------------------------- conv
constexpr int kTile = 64;        // coefficients per workgroup
constexpr int kGrpOut = 8;       // outputs per wave of the grouped form
constexpr int kOutPerWg = 4 * kGrpOut;

// One workgroup: 64 coefficients of one limb of one polynomial, 32 outputs.
// R_img: [I][ntap][2][nl][N]; pts: [npt][kcent][nl][N] (tap t reads set t, or
// set t % 3 of its kernel column when pt_shared); bias: [O][nl][N].
__global__ __launch_bounds__(256) void k_conv_contract(
    const uint64_t *__restrict__ R, int I, int ntap, int pt_shared, int nl, LimbMap map,
    const uint64_t *__restrict__ pts, int kcent,
    const int32_t *__restrict__ og_off, const int32_t *__restrict__ g_c, const int32_t *__restrict__ g_moff,
    const int32_t *__restrict__ m_i, const uint64_t *__restrict__ bias, Ptrs outs, int o_base, int o_count,
    const Prime *__restrict__ primes, int logN) {
    extern __shared__ uint64_t sR[];  // [I][kTile]
    const size_t N = size_t(1) << logN;
    const int limb = blockIdx.y;
    const int poly = blockIdx.z & 1, ogrp = blockIdx.z >> 1;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const size_t k = size_t(blockIdx.x) * kTile + lane;
    const Prime P = primes[map.prime(limb)];
    // a sum of n residues stays below 2^64 while (n + 1) q <= 2^64; a sum of
    // products (each < q^2) plus one residue stays below 2^128 for
    // prod_cap <= 2^(128 - 2k) - 1 (k = bit length of q)
    const uint64_t add_cap = P.onep - 1;
    const int prod_cap = P.k >= 61 ? (1 << (128 - 2 * P.k)) - 1 : 64;
    u128v acc[kGrpOut];
    int cnt[kGrpOut];
#pragma unroll
    for (int j = 0; j < kGrpOut; ++j) {
        acc[j] = u128v{0, 0};
        cnt[j] = 0;
    }
    for (int t = 0; t < ntap; ++t) {
        __syncthreads();
        for (int e = threadIdx.x; e < I * kTile; e += 256) {
            const int i = e / kTile, l = e - i * kTile;
            sR[e] = R[((size_t(i) * ntap + t) * 2 + poly) * nl * N + size_t(limb) * N + size_t(blockIdx.x) * kTile + l];
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kGrpOut; ++j) {
            const int ol = ogrp * kOutPerWg + wave + 4 * j;  // local output index
            if (ol >= o_count) continue;
            const int o = o_base + ol;
            const int g0 = og_off[o * ntap + t], g1 = og_off[o * ntap + t + 1];
            for (int g = g0; g < g1; ++g) {
                const int cc = g_c[g];
                const int m0 = g_moff[g], m1 = g_moff[g + 1];
                uint64_t s = 0;
                uint64_t nadd = 0;
                for (int m = m0; m < m1; ++m) {
                    s += sR[m_i[m] * kTile + lane];
                    if (++nadd == add_cap) {
                        s = reduce64(s, P);
                        nadd = 0;
                    }
                }
                s = reduce64(s, P);
                const uint64_t pv = pts[((size_t(pt_shared ? t % 3 : t) * kcent + cc) * nl + limb) * N + k];
                acc[j] = add128(acc[j], mul64x64(s, pv));
                if (++cnt[j] == prod_cap) {
                    acc[j] = u128v{reduce128(acc[j], P), 0};
                    cnt[j] = 0;
                }
            }
        }
    }
#pragma unroll
    for (int j = 0; j < kGrpOut; ++j) {
        const int ol = ogrp * kOutPerWg + wave + 4 * j;
        if (ol >= o_count) continue;
        const int o = o_base + ol;
        uint64_t y = reduce128(acc[j], P);
        if (poly == 0 && bias) y = add_mod(y, bias[(size_t(o) * nl + limb) * N + k], P.q);
        outs.p[ol][(size_t(poly) * nl + limb) * N + k] = y;
    }
}

// Direct form of the same contraction, batched over images, for codebooks of
// at most kMaxCentLds centroids:
//   y[m][o] = sum_t sum_i PT[t][idx[o][i][t]] * R[m][i][t] + bias_o
// for up to IMGS images m and OUTS consecutive outputs o.  One
// workgroup = one 64-coefficient column tile of one limb; with ROWS = 1 wave w
// handles image w >> 1 and polynomial w & 1, with ROWS = 2 image w and both
// polynomials (each codebook word read from LDS then serves two products,
// for twice the accumulator registers); a wave keeps one accumulator per
// output and polynomial.  Per tap
// the tap's whole codebook tile (kcent x 64 words) is staged in LDS once and
// read by every wave, so the codebook crosses HBM once per group of images and
// outputs rather than once per image and polynomial.  The centroid choices
// are wave-uniform: each is stored as the byte offset of its codebook row in
// the LDS tile (c * 512, 16 bits), four per 64-bit word, so a product's LDS
// address costs one scalar field extraction and one vector add; the words of
// consecutive inputs are contiguous so one scalar load brings several; R is read straight
// from HBM, each element by exactly one wave, for all its outputs, two blocks
// of kUnroll inputs ahead of their use (across tap boundaries).  With dbuf the next
// tap's codebook tile travels from HBM straight into a second LDS buffer
// (direct-to-LDS loads, two 512-byte rows per wave instruction) while the
// current tap computes.
// ioff: [ntap][ngrp][I] words, bits 16 j .. 16 j + 15 of word (t, g, i) =
// 512 * idx[4 g + j][i][t].
constexpr int kMaxCentLds = 128;
constexpr int kImgPerWg = 4;
constexpr int kUnroll = 4;
// With ybase set, one launch covers every group of OUTS outputs: block id ->
// (output group, column tile, limb) with the tile-limb pair's low 3 bits equal
// to id mod 8, so all output groups of one tile of one limb run on the same
// XCD (workgroups go round-robin over the 8 XCDs) within 8 ngroups
// consecutive ids and read the tile's rotated inputs from that XCD's L2 after
// the first; outputs at ybase + img * y_img + o * 2 nl N.  Otherwise blockIdx
// = (tile, limb) and the outputs of the o_count outputs from o_base are at
// outs.p[img * OUTS + j].
struct ConvOut {
    uint64_t *ybase;
    size_t y_img;
    int ngroups;
    int O;
};
template <int OUTS, int IMGS, int ROWS>
__global__ __launch_bounds__(128 / ROWS * IMGS) void k_conv_mac(const uint64_t *__restrict__ R, size_t r_img_words,
                                                           int n_img, int ni, int I, int i_base, int ntap, int nl,
                                                           LimbMap map, const uint64_t *__restrict__ pts, int kcent,
                                                           const uint64_t *__restrict__ ioff, int ngrp,
                                                           const uint64_t *__restrict__ bias, Ptrs outs, int o_base,
                                                           int o_count, int accumulate,
                                                           const Prime *__restrict__ primes, int logN, int dbuf,
                                                           int skip_tap, int pt_shared, uint64_t seq_all,
                                                           uint64_t seq_skip, ConvOut yo) {
    static_assert(OUTS % 4 == 0, "outputs per wave come in packed words of 4 offsets");
    static_assert(ROWS == 1 || ROWS == 2, "one or both polynomials per wave");
    constexpr int NW = OUTS / 4;
    constexpr int NWAVE = 2 / ROWS * IMGS;
    extern __shared__ uint64_t sP[];  // [dbuf ? 2 : 1][kcent][kTile]
    const size_t N = size_t(1) << logN;
    int limb, tile;
    if (yo.ybase) {
        const unsigned id = blockIdx.x, ng = unsigned(yo.ngroups);
        const unsigned tl = (id / (8u * ng)) * 8u + (id & 7u), ntiles = unsigned(N / kTile);
        tile = int(tl % ntiles);
        limb = int(tl / ntiles);
        o_base = int((id >> 3) % ng) * OUTS;
        o_count = min(OUTS, yo.O - o_base);
    } else {
        tile = blockIdx.x;
        limb = blockIdx.y;
    }
    const int lane = threadIdx.x & 63;
    // wave index as a wave-uniform (scalar) value, so per-wave control flow and
    // index loads stay scalar
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int img = ROWS == 2 ? wave : wave >> 1, poly = ROWS == 2 ? 0 : wave & 1;
    const bool active = img < n_img;
    const size_t col0 = size_t(tile) * kTile;
    const size_t pw = size_t(nl) * N, ctw = 2 * pw;
    const Prime P = primes[map.prime(limb)];
    const int pcap = fold_cap(P.k);
    const uint64_t r64 = P.r2;  // 2^64 mod q
    const size_t rstride = size_t(ntap) * ctw;  // R words between consecutive inputs
    const uint64_t *Rb = R + size_t(active ? img : 0) * r_img_words + size_t(poly) * pw + size_t(limb) * N + col0 + lane;
    const int g0 = o_base / 4;
    // acc[r][j]: output o_base + j, polynomial poly + r
    accc acc[ROWS][OUTS];
#pragma unroll
    for (int r = 0; r < ROWS; ++r)
#pragma unroll
        for (int j = 0; j < OUTS; ++j) acc[r][j] = accc{0, 0, 0, 0, 0};
    int cnt = 0;
    // codebook rows 2 pr and 2 pr + 1 of plaintext set ps: lane l brings words
    // 2 (l & 31) and 2 (l & 31) + 1 of row 2 pr + (l >> 5) to LDS address 16 l
    // past the pair (an odd last row leaves the upper half-wave idle)
    auto stage = [&](int ps, uint64_t *buf) {
        for (int pr = wave; 2 * pr < kcent; pr += NWAVE) {
            const int c = 2 * pr + (lane >> 5);
            if (c < kcent)
                __builtin_amdgcn_global_load_lds(
                    (const void *)(pts + ((size_t(ps) * kcent + c) * nl + limb) * N + col0 + 2 * (lane & 31)),
                    (__attribute__((address_space(3))) void *)(buf + size_t(2 * pr) * kTile), 16, 0, 0);
        }
    };
    // taps are visited in the order of a packed sequence (4 bits per visit):
    // column by column when the taps of a kernel column share their
    // plaintexts (one codebook tile serves the column's three taps), and
    // without the identity tap on the P limbs, where its rotated inputs P x
    // are zero (visit v -> stored tap phys(v))
    const bool skip = skip_tap >= 0 && limb >= map.nlow;
    const int ntl = skip ? ntap - 1 : ntap;
    const uint64_t seq = skip ? seq_skip : seq_all;
    auto phys = [&](int v) { return int((seq >> (4 * v)) & 15u); };
    auto ptix = [&](int t) { return pt_shared ? t % 3 : t; };
    // visit v starts a new plaintext set (a new codebook tile)
    auto newset = [&](int v) { return v == 0 || ptix(phys(v)) != ptix(phys(v - 1)); };
    uint64_t *const buf0 = sP, *const buf1 = dbuf ? sP + size_t(kcent) * kTile : sP;
    if (dbuf) stage(ptix(phys(0)), buf0);
    int nset = 0;          // plaintext sets begun so far
    uint64_t *cur = buf0;  // the current set's codebook tile
    const uint64_t *ixw0 = ioff + size_t(g0) * I + i_base;
    // The flat stream of blocks of kUnroll inputs, tap by tap.  Coefficients
    // travel two blocks ahead of their use in a ring of three register
    // buffers that swap roles in straight-line code (a register copy would wait
    // for its load); indices past the end are clamped to the last valid input
    // and tap, so every load is unconditional.  Positions are kept as
    // wave-uniform counters (no division).
    int tc = 0, ic = 0;  // block being computed
    // next block whose coefficients to fetch: (tp, ip), word offset roff of
    // its first input from Rb; past the last block the offset stays on the
    // last valid one
    int tp = 0, ip = 0;
    size_t roff = size_t(phys(0)) * ctw;
    auto load_block = [&](uint64_t(&buf)[ROWS][kUnroll]) {
        const uint64_t *rp = Rb + roff;
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            // opaque to the optimiser: a past-the-end offset of 0 must stay a
            // load of its own (merged with input 0 it becomes a register copy,
            // and a copy waits for its load)
            size_t off = ip + u < ni ? size_t(u) * rstride : 0;
            asm("" : "+s"(off));
#pragma unroll
            for (int r = 0; r < ROWS; ++r) buf[r][u] = rp[off + size_t(r) * pw];
        }
        if (ip + kUnroll < ni) {
            ip += kUnroll;
            roff += size_t(kUnroll) * rstride;
        } else if (tp + 1 < ntl) {
            ip = 0;
            ++tp;
            roff = size_t(phys(tp)) * ctw;
        }
    };
    // the offset words of a block, one contiguous scalar load per group of 4
    // outputs (a row's ragged end reads into the next row, the last row into
    // kUnroll words of zero padding)
    int tk = 0, ik = 0;
    size_t koff = size_t(phys(0)) * ngrp * I;
    auto load_index = [&](uint64_t(&kw)[NW][kUnroll]) {
        const uint64_t *ixw = ixw0 + koff;
#pragma unroll
        for (int w = 0; w < NW; ++w)
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) kw[w][u] = ixw[size_t(w) * I + u];
        if (ik + kUnroll < ni) {
            ik += kUnroll;
            koff += kUnroll;
        } else if (tk + 1 < ntl) {
            ik = 0;
            ++tk;
            koff = size_t(phys(tk)) * ngrp * I;
        }
    };
    // the products of the block at (tc, ic): coefficients cr, index words kw,
    // codebook tile cb
    auto block = [&](const uint64_t(&cr)[ROWS][kUnroll], const uint64_t(&kw)[NW][kUnroll], const uint64_t *cb) {
        const int i = ic;
        if (cnt + kUnroll > pcap) {
#pragma unroll
            for (int r = 0; r < ROWS; ++r)
#pragma unroll
                for (int j = 0; j < OUTS; ++j) {
                    // macc_folded written out: through the call (or with the
                    // fold's products as one asm block) the compiler gives
                    // this kernel 14 more registers (occupancy 3, not 4)
                    const u128v v = accc_value(acc[r][j]);
                    acc[r][j] = accc{0, 0, v.lo, 0, 0};
                    macc(acc[r][j], v.hi, r64);
                }
            cnt = 0;
        }
        // codebook words of the next input are read while this input's
        // products run
        const char *cbl = (const char *)(cb + lane);
        auto word = [&](uint64_t k, int j) {
            return *(const uint64_t *)(cbl + uint32_t(k >> (16 * j)) % 65536u);
        };
        uint64_t cv[OUTS];
#pragma unroll
        for (int w = 0; w < NW; ++w)
#pragma unroll
            for (int j = 0; j < 4; ++j) cv[4 * w + j] = word(kw[w][0], j);
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            if (i + u >= ni) break;
            uint64_t cn[OUTS];
            if (u + 1 < kUnroll) {
#pragma unroll
                for (int w = 0; w < NW; ++w)
#pragma unroll
                    for (int j = 0; j < 4; ++j) cn[4 * w + j] = word(kw[w][u + 1 < kUnroll ? u + 1 : u], j);
            }
#pragma unroll
            for (int j = 0; j < OUTS; ++j)
#pragma unroll
                for (int r = 0; r < ROWS; ++r) macc(acc[r][j], cr[r][u], cv[j]);
            if (u + 1 < kUnroll) {
#pragma unroll
                for (int j = 0; j < OUTS; ++j) cv[j] = cn[j];
            }
        }
        cnt += kUnroll;
    };
    // one block: a tap's first block first synchronises on its codebook tile
    // (and starts the next tap's transfer); the coefficients two blocks ahead
    // are fetched before the products, the next block's index words after
    // them (a wait on a scalar load also waits for every LDS read in flight)
    auto step = [&](const uint64_t(&cr)[ROWS][kUnroll], uint64_t(&nx)[ROWS][kUnroll],
                    const uint64_t(&kc)[NW][kUnroll], uint64_t(&kn)[NW][kUnroll]) {
        if (tc >= ntl) return;
        if (ic == 0 && newset(tc)) {
            cur = (nset & 1) ? buf1 : buf0;
            if (!dbuf) {
                __syncthreads();
                stage(ptix(phys(tc)), cur);
            }
            __syncthreads();
            if (dbuf) {
                // the next set's tile goes into the other buffer, whose last
                // readers (the previous set) are past the barrier
                int v2 = tc + 1;
                while (v2 < ntl && !newset(v2)) ++v2;
                if (v2 < ntl) stage(ptix(phys(v2)), (nset & 1) ? buf0 : buf1);
            }
            ++nset;
        }
        if (active) {
            load_block(nx);
            block(cr, kc, cur);
            load_index(kn);
        }
        ic += kUnroll;
        if (ic >= ni) {
            ic = 0;
            ++tc;
        }
    };
    uint64_t ra[ROWS][kUnroll], rb[ROWS][kUnroll], rc[ROWS][kUnroll];
    uint64_t ka[NW][kUnroll], kb[NW][kUnroll];
    if (active) {
        load_block(ra);
        load_block(rb);
        load_index(ka);
    }
    // three blocks per iteration: coefficients rotate through three buffers,
    // index words through two
    while (tc < ntl) {
        step(ra, rc, ka, kb);
        step(rb, ra, kb, ka);
        step(rc, rb, ka, kb);
        step(ra, rc, kb, ka);
        step(rb, ra, ka, kb);
        step(rc, rb, kb, ka);
    }
    if (!active) return;
#pragma unroll
    for (int r = 0; r < ROWS; ++r)
#pragma unroll
        for (int j = 0; j < OUTS; ++j) {
            if (j >= o_count) continue;
            const int o = o_base + j, pl = poly + r;
            uint64_t y = reduce128(accc_value(acc[r][j]), P);
            uint64_t *dst = (yo.ybase ? yo.ybase + size_t(img) * yo.y_img + size_t(o) * ctw : outs.p[img * OUTS + j]) +
                            size_t(pl) * pw + size_t(limb) * N + col0 + lane;
            if (accumulate) y = add_mod(y, *dst, P.q);
            else if (pl == 0 && bias) y = add_mod(y, bias[(size_t(o) * nl + limb) * N + col0 + lane], P.q);
            *dst = y;
        }
}

using ConvFn = void (*)(const uint64_t *, size_t, int, int, int, int, int, int, LimbMap, const uint64_t *, int,
                        const uint64_t *, int, const uint64_t *, Ptrs, int, int, int, const Prime *, int, int, int,
                        int, uint64_t, uint64_t, ConvOut);

// visiting order of a layer's taps for the direct-form contraction, 4 bits
// per visit: column by column when the taps of a column share their
// plaintexts, else in stored order; without tap `skip` (when >= 0)
uint64_t tap_sequence(const ckc_layer *L, int skip) {
    uint64_t seq = 0;
    int v = 0;
    for (int j = 0; j < L->ntap; ++j) {
        const int t = L->pt_shared ? (j % L->ksz) * L->ksz + j / L->ksz : j;
        if (t == skip) continue;
        seq |= uint64_t(t) << (4 * v++);
    }
    return seq;
}
// kernel for a group of gi images: the smallest workgroup (1, 2 or 4 images)
// that holds them; outs = outputs per wave (8 or 16), a tuning choice between
// accumulator registers (occupancy) and codebook re-reads per output group;
// rows = polynomials per wave (1 or 2), between registers and LDS reads
static ConvFn conv_kernel(int outs, int rows, int gi, int *imgs) {
    *imgs = gi <= 1 ? 1 : gi <= 2 ? 2 : 4;
    if (rows == 2) {
        if (outs == 16)
            return *imgs == 1 ? k_conv_mac<16, 1, 2> : *imgs == 2 ? k_conv_mac<16, 2, 2> : k_conv_mac<16, 4, 2>;
        return *imgs == 1 ? k_conv_mac<8, 1, 2> : *imgs == 2 ? k_conv_mac<8, 2, 2> : k_conv_mac<8, 4, 2>;
    }
    if (outs == 16)
        return *imgs == 1 ? k_conv_mac<16, 1, 1> : *imgs == 2 ? k_conv_mac<16, 2, 1> : k_conv_mac<16, 4, 1>;
    return *imgs == 1 ? k_conv_mac<8, 1, 1> : *imgs == 2 ? k_conv_mac<8, 2, 1> : k_conv_mac<8, 4, 1>;
}

int check_inputs(const ckc_ct *in, int n, int level, const char *what) {
    for (int i = 0; i < n; ++i) {
        CKC_REQUIRE(in[i].d, CKC_EINVAL, std::string(what) + ": null input");
        CKC_REQUIRE(in[i].level == level, CKC_ELEVEL, std::string(what) + ": input level differs from the layer's");
        CKC_REQUIRE(in[i].npoly == 2, CKC_ESHAPE, std::string(what) + ": inputs must be 2-poly ciphertexts");
        CKC_REQUIRE(fabs(in[i].scale / in[0].scale - 1.0) <= ldexp(1.0, -30), CKC_ESCALE,
                    std::string(what) + ": input scales differ");
    }
    return CKC_OK;
}

}  // namespace

// ============================================================= layer creation
extern "C" int ckc_layer_create_conv_ex(ckc_ctx *c, const ckc_layout *in, int out_ch, int in_ch, int ksize,
                                        int stride, int n_centroids, const double *codebook, const uint16_t *idx,
                                        const double *bias, int level, double pt_scale, double bias_scale,
                                        int hoisting, ckc_layer **out, void *stream) {
    CKC_REQUIRE(c && out && codebook && idx, CKC_EINVAL, "null argument");
    CKC_REQUIRE(hoisting == CKC_HOIST_DOUBLE || hoisting == CKC_HOIST_SINGLE, CKC_EINVAL, "bad hoisting mode");
    CKC_TRY(check_layout(c, in));
    CKC_REQUIRE(ksize == 1 || ksize == 3, CKC_EUNSUPPORTED, "kernel size must be 1 or 3");
    CKC_REQUIRE(stride == 1 || stride == 2, CKC_EUNSUPPORTED, "stride must be 1 or 2");
    CKC_REQUIRE(out_ch >= 1 && in_ch >= 1, CKC_EINVAL, "channel counts must be positive");
    CKC_REQUIRE(n_centroids <= kMaxCentLds || in_ch <= kMaxBatch, CKC_EUNSUPPORTED,
                "codebooks above 128 centroids need in_ch <= 64");
    CKC_REQUIRE(n_centroids >= 1 && n_centroids <= 65535, CKC_EINVAL, "bad centroid count");
    CKC_REQUIRE(level >= 0 && level < c->nq, CKC_ELEVEL, "level out of range");
    CKC_REQUIRE(in->height % stride == 0 && in->width % stride == 0, CKC_ESHAPE, "grid not divisible by stride");
    hipStream_t s = S(stream);
    auto L = std::make_unique<ckc_layer>();
    L->kind = LK_CONV;
    L->lin = *in;
    L->lout = *in;
    L->lout.gap = in->gap * stride;
    L->lout.height = in->height / stride;
    L->lout.width = in->width / stride;
    L->level = level;
    L->O = out_ch;
    L->I = in_ch;
    L->ksz = ksize;
    L->stride = stride;
    L->ntap = ksize * ksize;
    L->kcent = n_centroids;
    L->pt_scale = pt_scale;
    L->bias_scale = bias_scale;
    const int nl = level + 1, M = in->members, half = ksize / 2;
    const size_t N = c->N, n = N / 2, pw = size_t(nl) * N;
    for (int t = 0; t < L->ntap; ++t) {
        const int dh = t / ksize - half, dw = t % ksize - half;
        L->tap_step.push_back(in->gap * (dh * in->row_stride + dw));
    }
    // codebook plaintexts: PT[t][c] = centroid c of column(t), per member, on
    // the tap's mask.  A layer with rotations sums its products in Q_l u P
    // (one ModDown per output) unless it is single-hoisted (one ModDown per
    // rotated input), so its plaintexts carry the P limbs too.
    L->ext = ksize > 1 && hoisting == CKC_HOIST_DOUBLE;
    // slice-shared layout: the taps of one kernel column share its plaintexts
    // (the zero rows stand in for the vertical mask), which are those of the
    // column's middle tap
    L->pt_shared = (in->flags & CKC_LAYOUT_SLICE_SHARED) && ksize == 3;
    L->npt = L->pt_shared ? ksize : L->ntap;
    const size_t ppw = L->ext ? size_t(nl + c->np) * N : pw;  // words per codebook plaintext
    CKC_TRY(L->pts.alloc(8 * ppw * L->npt * n_centroids));
    std::vector<double> v(n);
    const ckc_layout &Lo = L->lout;
    for (int ps = 0; ps < L->npt; ++ps) {
        const int t = L->pt_shared ? half * ksize + ps : ps;
        const int dh = t / ksize - half, dw = t % ksize - half, col = t % ksize;
        for (int cc = 0; cc < n_centroids; ++cc) {
            std::fill(v.begin(), v.end(), 0.0);
            for (int m = 0; m < M; ++m) {
                const double w = codebook[(size_t(col) * n_centroids + cc) * M + m];
                for (int r = 0; r < Lo.height; ++r) {
                    const int ri = stride * r + dh;
                    if (ri < 0 || ri >= in->height) continue;
                    for (int q = 0; q < Lo.width; ++q) {
                        const int ci = stride * q + dw;
                        if (ci < 0 || ci >= in->width) continue;
                        v[slot_of(Lo, m, r, q)] = w;
                    }
                }
            }
            CKC_TRY(encode_impl(c, v.data(), n, level, pt_scale, L->pts.u64() + (size_t(ps) * n_centroids + cc) * ppw,
                                s, L->ext));
        }
    }
    if (bias) {
        L->has_bias = true;
        CKC_TRY(L->bias.alloc(8 * pw * out_ch));
        for (int o = 0; o < out_ch; ++o) {
            std::fill(v.begin(), v.end(), 0.0);
            for (int m = 0; m < M; ++m)
                for (int r = 0; r < Lo.height; ++r)
                    for (int q = 0; q < Lo.width; ++q) v[slot_of(Lo, m, r, q)] = bias[size_t(m) * out_ch + o];
            CKC_TRY(encode_impl(c, v.data(), n, level, bias_scale, L->bias.u64() + size_t(o) * pw, s));
        }
    }
    // group lists: for each (o, t) the centroids used and the inputs per centroid
    std::vector<int32_t> og_off{0}, g_c, g_moff{0}, m_i;
    std::vector<std::vector<int32_t>> members(n_centroids);
    for (int o = 0; o < out_ch; ++o)
        for (int t = 0; t < L->ntap; ++t) {
            for (auto &mv : members) mv.clear();
            for (int i = 0; i < in_ch; ++i) {
                const int ci = idx[(size_t(o) * in_ch + i) * L->ntap + t];
                CKC_REQUIRE(ci < n_centroids, CKC_EINVAL, "centroid index out of range");
                members[ci].push_back(i);
            }
            for (int cc = 0; cc < n_centroids; ++cc) {
                if (members[cc].empty()) continue;
                g_c.push_back(cc);
                for (int i : members[cc]) m_i.push_back(i);
                g_moff.push_back(int32_t(m_i.size()));
            }
            og_off.push_back(int32_t(g_c.size()));
        }
    // codebook row byte offsets for the direct form, [tap][output group of
    // 4][input], outputs padded to a multiple of 32
    if (n_centroids <= kMaxCentLds) {
        L->Opad = (out_ch + kOutPerWg - 1) / kOutPerWg * kOutPerWg;
        const int ngrp = L->Opad / 4;
        // kUnroll zero words past the end: the kernel reads whole blocks
        std::vector<uint64_t> ix(size_t(L->ntap) * ngrp * in_ch + kUnroll, 0);
        for (int o = 0; o < out_ch; ++o)
            for (int i = 0; i < in_ch; ++i)
                for (int t = 0; t < L->ntap; ++t)
                    ix[(size_t(t) * ngrp + o / 4) * in_ch + i] |=
                        uint64_t(uint32_t(idx[(size_t(o) * in_ch + i) * L->ntap + t]) * kTile * 8) << (16 * (o % 4));
        CKC_TRY(L->ioff.upload(ix.data(), 8 * ix.size()));
    }
    if (g_c.empty()) g_c.push_back(0);
    if (m_i.empty()) m_i.push_back(0);
    CKC_TRY(L->og_off.upload(og_off.data(), 4 * og_off.size()));
    CKC_TRY(L->g_c.upload(g_c.data(), 4 * g_c.size()));
    CKC_TRY(L->g_moff.upload(g_moff.data(), 4 * g_moff.size()));
    CKC_TRY(L->m_i.upload(m_i.data(), 4 * m_i.size()));
    L->bytes = L->pts.bytes + L->bias.bytes + 4 * (og_off.size() + g_c.size() + g_moff.size() + m_i.size());
    CKC_HIP(hipStreamSynchronize(s));
    *out = L.release();
    return CKC_OK;
}

extern "C" int ckc_layer_create_conv(ckc_ctx *c, const ckc_layout *in, int out_ch, int in_ch, int ksize, int stride,
                                     int n_centroids, const double *codebook, const uint16_t *idx, const double *bias,
                                     int level, double pt_scale, double bias_scale, ckc_layer **out, void *stream) {
    return ckc_layer_create_conv_ex(c, in, out_ch, in_ch, ksize, stride, n_centroids, codebook, idx, bias, level,
                                    pt_scale, bias_scale, CKC_HOIST_DOUBLE, out, stream);
}

extern "C" int ckc_layer_create_act(ckc_ctx *c, const ckc_layout *layout, int channels, const double *b,
                                    const double *cc, double a_absorb, int level, double in_scale, ckc_layer **out,
                                    void *stream) {
    CKC_REQUIRE(c && out && b && cc, CKC_EINVAL, "null argument");
    CKC_TRY(check_layout(c, layout));
    CKC_REQUIRE(channels >= 1, CKC_EINVAL, "bad channel count");
    CKC_REQUIRE(level >= 0 && level < c->nq, CKC_ELEVEL, "level out of range");
    CKC_REQUIRE(a_absorb != 0.0 && isfinite(a_absorb) && in_scale > 0, CKC_EINVAL, "bad scale arguments");
    hipStream_t s = S(stream);
    auto L = std::make_unique<ckc_layer>();
    L->kind = LK_ACT;
    L->lin = L->lout = *layout;
    L->level = level;
    L->C = channels;
    L->a_absorb = a_absorb;
    L->in_scale = in_scale;
    const int nl = level + 1, M = layout->members;
    const size_t N = c->N, n = N / 2, pw = size_t(nl) * N;
    const double s2 = in_scale * in_scale;
    CKC_TRY(L->bpt.alloc(8 * pw * channels));
    CKC_TRY(L->cpt.alloc(8 * pw * channels));
    std::vector<double> v(n);
    // slice-shared layout: the spare rows stay zero, so the constant term goes
    // on the grid's slots only (b multiplies x, which is zero there)
    const bool grid_c = layout->flags & CKC_LAYOUT_SLICE_SHARED;
    for (int ch = 0; ch < channels; ++ch) {
        if (grid_c) {
            std::fill(v.begin(), v.end(), 0.0);
            for (int m = 0; m < M; ++m)
                for (int r = 0; r < layout->height; ++r)
                    for (int q = 0; q < layout->width; ++q) v[slot_of(*layout, m, r, q)] = cc[size_t(m) * channels + ch];
            CKC_TRY(encode_impl(c, v.data(), n, level, s2, L->cpt.u64() + size_t(ch) * pw, s));
        }
        if (M == 1) {
            CKC_TRY(fill_const_pt(c, L->bpt.u64() + size_t(ch) * pw, b[ch], in_scale, nl, s));
            if (!grid_c) CKC_TRY(fill_const_pt(c, L->cpt.u64() + size_t(ch) * pw, cc[ch], s2, nl, s));
        } else {
            for (int which = 0; which < (grid_c ? 1 : 2); ++which) {
                const double *src = which == 0 ? b : cc;
                std::fill(v.begin(), v.end(), 0.0);
                for (int m = 0; m < M; ++m)
                    for (int j = 0; j < layout->block; ++j) v[size_t(m) * layout->block + j] = src[size_t(m) * channels + ch];
                uint64_t *dst = (which == 0 ? L->bpt.u64() : L->cpt.u64()) + size_t(ch) * pw;
                CKC_TRY(encode_impl(c, v.data(), n, level, which == 0 ? in_scale : s2, dst, s));
            }
        }
    }
    L->bytes = L->bpt.bytes + L->cpt.bytes;
    *out = L.release();
    return CKC_OK;
}

namespace {
// the fields both dense forms share: sizes, scales, output layout (one grid
// point), and the rotation steps of the slot sums over the grid
int dense_common(ckc_ctx *c, const ckc_layout *in, int classes, int in_ch, int level, double pt_scale,
                 double bias_scale, std::unique_ptr<ckc_layer> &L) {
    CKC_TRY(check_layout(c, in));
    CKC_REQUIRE(is_pow2(in->height) && is_pow2(in->width), CKC_EUNSUPPORTED, "dense: grid sides must be powers of two");
    CKC_REQUIRE(classes >= 1 && in_ch >= 1, CKC_EINVAL, "bad sizes");
    CKC_REQUIRE(level >= 0 && level < c->nq, CKC_ELEVEL, "level out of range");
    L = std::make_unique<ckc_layer>();
    L->kind = LK_DENSE;
    L->lin = *in;
    L->lout = *in;
    L->lout.height = L->lout.width = 1;
    L->level = level;
    L->K = classes;
    L->C = in_ch;
    L->pt_scale = pt_scale;
    L->bias_scale = bias_scale;
    for (int j = 1; j < in->width; j <<= 1) L->sum_steps.push_back(in->gap * j);
    for (int j = 1; j < in->height; j <<= 1) L->sum_steps.push_back(in->gap * in->row_stride * j);
    return CKC_OK;
}
}  // namespace

extern "C" int ckc_layer_create_dense(ckc_ctx *c, const ckc_layout *in, int classes, int in_ch, const double *w,
                                      const double *bias, int level, double pt_scale, double bias_scale,
                                      ckc_layer **out, void *stream) {
    CKC_REQUIRE(c && out && w, CKC_EINVAL, "null argument");
    hipStream_t s = S(stream);
    std::unique_ptr<ckc_layer> L;
    CKC_TRY(dense_common(c, in, classes, in_ch, level, pt_scale, bias_scale, L));
    const int nl = level + 1, M = in->members;
    const size_t N = c->N, n = N / 2, pw = size_t(nl) * N;
    if (M == 1) {
        // one member: only slot 0 is read, so every weight is a constant
        // multiplier (the encoding of the constant slot vector) and the bias a
        // constant addend
        std::vector<uint64_t> all(size_t(classes) * in_ch * nl), r;
        for (int k = 0; k < classes; ++k)
            for (int ch = 0; ch < in_ch; ++ch) {
                const_residues(c, w[size_t(k) * in_ch + ch], pt_scale, nl, r);
                std::copy(r.begin(), r.end(), all.begin() + (size_t(k) * in_ch + ch) * nl);
            }
        CKC_TRY(L->dconst.upload(all.data(), 8 * all.size()));
        if (bias) {
            L->has_bias = true;
            std::vector<uint64_t> bc(size_t(classes) * nl);
            for (int k = 0; k < classes; ++k) {
                const_residues(c, bias[k], bias_scale, nl, r);
                std::copy(r.begin(), r.end(), bc.begin() + size_t(k) * nl);
            }
            CKC_TRY(L->bconst.upload(bc.data(), 8 * bc.size()));
        }
    } else {
        CKC_TRY(L->pts.alloc(8 * pw * classes * in_ch));
        std::vector<double> v(n, 0.0);
        for (int k = 0; k < classes; ++k)
            for (int ch = 0; ch < in_ch; ++ch) {
                for (int m = 0; m < M; ++m) v[size_t(m) * in->block] = w[(size_t(m) * classes + k) * in_ch + ch];
                CKC_TRY(encode_impl(c, v.data(), n, level, pt_scale, L->pts.u64() + (size_t(k) * in_ch + ch) * pw, s));
            }
        if (bias) {
            L->has_bias = true;
            CKC_TRY(L->bias.alloc(8 * pw * classes));
            for (int k = 0; k < classes; ++k) {
                for (int m = 0; m < M; ++m) v[size_t(m) * in->block] = bias[size_t(m) * classes + k];
                CKC_TRY(encode_impl(c, v.data(), n, level, bias_scale, L->bias.u64() + size_t(k) * pw, s));
            }
        }
    }
    L->bytes = L->pts.bytes + L->bias.bytes + L->dconst.bytes + L->bconst.bytes;
    *out = L.release();
    return CKC_OK;
}

extern "C" int ckc_layer_create_dense_spatial(ckc_ctx *c, const ckc_layout *in, int classes, int in_ch,
                                              const double *w, const double *bias, int level, double pt_scale,
                                              double bias_scale, ckc_layer **out, void *stream) {
    CKC_REQUIRE(c && out && w, CKC_EINVAL, "null argument");
    hipStream_t s = S(stream);
    std::unique_ptr<ckc_layer> L;
    CKC_TRY(dense_common(c, in, classes, in_ch, level, pt_scale, bias_scale, L));
    L->spatial = true;
    const int nl = level + 1, M = in->members, H = in->height, W = in->width;
    const size_t N = c->N, n = N / 2, pw = size_t(nl) * N;
    CKC_TRY(L->pts.alloc(8 * pw * classes * in_ch));
    std::vector<double> v(n, 0.0);
    for (int k = 0; k < classes; ++k)
        for (int ch = 0; ch < in_ch; ++ch) {
            // w[m][k][ch][r][col] at member m's grid point (r, col)
            for (int m = 0; m < M; ++m)
                for (int r = 0; r < H; ++r)
                    for (int col = 0; col < W; ++col)
                        v[size_t(m) * in->block + size_t(in->gap) * (size_t(r) * in->row_stride + col)] =
                            w[(((size_t(m) * classes + k) * in_ch + ch) * H + r) * W + col];
            CKC_TRY(encode_impl(c, v.data(), n, level, pt_scale, L->pts.u64() + (size_t(k) * in_ch + ch) * pw, s));
        }
    if (bias) {
        L->has_bias = true;
        std::fill(v.begin(), v.end(), 0.0);
        CKC_TRY(L->bias.alloc(8 * pw * classes));
        for (int k = 0; k < classes; ++k) {
            for (int m = 0; m < M; ++m) v[size_t(m) * in->block] = bias[size_t(m) * classes + k];
            CKC_TRY(encode_impl(c, v.data(), n, level, bias_scale, L->bias.u64() + size_t(k) * pw, s));
        }
    }
    L->bytes = L->pts.bytes + L->bias.bytes;
    *out = L.release();
    return CKC_OK;
}

extern "C" int ckc_layer_steps(const ckc_layer *L, int32_t *steps, int max) {
    if (!L) return 0;
    std::vector<int32_t> st;
    if (L->kind == LK_CONV)
        for (int32_t x : L->tap_step)
            if (x != 0) st.push_back(x);
    if (L->kind == LK_DENSE) st = L->sum_steps;
    for (int i = 0; i < int(st.size()) && i < max; ++i) steps[i] = st[i];
    return int(st.size());
}

extern "C" int ckc_layer_out_layout(const ckc_layer *L, ckc_layout *out) {
    CKC_REQUIRE(L && out, CKC_EINVAL, "null argument");
    *out = L->lout;
    return CKC_OK;
}

extern "C" size_t ckc_layer_bytes(const ckc_layer *L) { return L ? L->bytes : 0; }

extern "C" int ckc_layer_destroy(ckc_layer *L) {
    delete L;
    return CKC_OK;
}

// ============================================================= evaluation
extern "C" int ckc_eval_conv(ckc_ctx *c, const ckc_evk *evk, const ckc_layer *L, const ckc_ct *in, int n_img,
                             ckc_ct *out, void *stream) {
    CKC_FAULT_POINT();
    CKC_REQUIRE(c && evk && L && in && out && n_img >= 0, CKC_EINVAL, "null argument");
    CKC_REQUIRE(L->kind == LK_CONV, CKC_EINVAL, "not a convolution layer");
    CKC_TRY(check_evk_images(evk, n_img, "eval_conv"));
    if (n_img == 0) return CKC_OK;
    CKC_TRY(check_inputs(in, n_img * L->I, L->level, "eval_conv"));
    for (int i = 0; i < n_img * L->O; ++i) CKC_REQUIRE(out[i].d, CKC_EINVAL, "eval_conv: null output");
    const double out_scale = in[0].scale * L->pt_scale;
    if (L->has_bias)
        CKC_REQUIRE(fabs(out_scale / L->bias_scale - 1.0) <= ldexp(1.0, -30), CKC_ESCALE,
                    "eval_conv: bias scale does not match in.scale * pt_scale");
    hipStream_t s = S(stream);
    const size_t N = c->N;
    const int nl = L->level + 1, I = L->I, ntap = L->ntap, O = L->O;
    const size_t pw = size_t(nl) * N;
    // A layer with rotations (ext) keeps every rotated input in Q_l u P and
    // sums the products there; one ModDown per output polynomial returns to
    // Q_l and adds the bias.  A 1x1 layer multiplies its inputs directly.
    const int nlim = L->ext ? nl + c->np : nl;  // limbs of R and of the sums
    const LimbMap map = L->ext ? LimbMap{nl, c->nq} : qmap();
    const size_t lpw = size_t(nlim) * N, lctw = 2 * lpw;
    // Input channels in chunks of at most kMaxBatch (one key-switching batch
    // per image); the contraction accumulates the chunks' partial sums (exact
    // modular sums, so the result does not depend on the chunking).  Images
    // per pass: at least one contraction group, and enough to fill a
    // key-switching batch when the layer has few inputs.
    const int ichunk = std::min(I, kMaxBatch);
    const int chunk = std::max(kImgPerWg, kMaxBatch / ichunk);
    const int nchunk = std::min(chunk, n_img);
    const size_t r_img = size_t(ichunk) * ntap * lctw;  // R words per image
    DevBuf R, Y;
    CKC_TRY(R.alloc(8 * r_img * nchunk, s));
    if (L->ext) CKC_TRY(Y.alloc(8 * lctw * O * nchunk, s));
    const size_t lds = size_t(I) * kTile * 8;
    // with the products in Q_l u P, the identity tap's rotated inputs (P x)
    // are zero on the P limbs, which the contraction then skips
    int skip_tap = -1;
    if (L->ext)
        for (int t = 0; t < ntap; ++t)
            if (L->tap_step[t] == 0) skip_tap = t;
    const double skipped = skip_tap >= 0 ? double(c->np) : 0.0;  // P limbs without the identity tap
    const uint64_t seq_all = tap_sequence(L, -1), seq_skip = tap_sequence(L, skip_tap);
    // codebook rows the skip saves: the identity tap's own set, unless its
    // column's other taps read that set too
    const double skipped_pt = L->pt_shared ? 0.0 : double(L->kcent);
    for (int img0 = 0; img0 < n_img; img0 += chunk) {
        const int ni_img = std::min(chunk, n_img - img0);
        if (!L->ioff.p)
            CKC_REQUIRE(ichunk == I, CKC_EUNSUPPORTED, "grouped contraction needs in_ch <= 64");
        // destination of output o of image m of the chunk: its extended-basis
        // sum (ext) or the caller's ciphertext
        auto dest = [&](int m, int o) -> uint64_t * {
            return L->ext ? Y.u64() + (size_t(m) * O + o) * lctw : out[size_t(img0 + m) * O + o].d;
        };
        const uint64_t *bias_k = L->ext ? nullptr : (L->has_bias ? L->bias.u64() : nullptr);
        for (int ic0 = 0; ic0 < I; ic0 += ichunk) {
            const int nic = std::min(ichunk, I - ic0);
            // rotations, in KS batches: (image in chunk, input channel of the
            // chunk); a batch shares one key set (a key group splits it)
            const int total = ni_img * nic;
            const int ksb = tune_value(TK_KS_BATCH);
            for (int b0 = 0, nb = 0; b0 < total; b0 += nb) {
                nb = std::min(ksb, total - b0);
                if (evk->is_group()) nb = key_run(evk, img0 * nic + b0, nb, nic);
                const ckc_evk *ek = evk_of(evk, img0 + b0 / nic);
                Ptrs ip;
                std::vector<Ptrs> dst(ntap);
                for (int b = 0; b < nb; ++b) {
                    const int flat = b0 + b, im = flat / nic, ii = flat - im * nic;
                    ip.p[b] = in[size_t(img0 + im) * I + ic0 + ii].d;
                    for (int t = 0; t < ntap; ++t)
                        dst[t].p[b] = R.u64() + size_t(im) * r_img + (size_t(ii) * ntap + t) * lctw;
                }
                if (L->ext)
                    CKC_TRY(hoisted_group_ext(c, ek, ip, nb, L->level, L->tap_step, dst, s));
                else
                    CKC_TRY(hoisted_group(c, ek, ip, nb, L->level, L->tap_step, dst, s));
            }
            if (L->ioff.p) {
                // contraction: groups of up to conv_imgs images x conv_outs outputs
                const int outs = tune_value(TK_CONV_OUTS), wg_max = tune_value(TK_CONV_IMGS),
                          rows = tune_value(TK_CONV_ROWS);
                for (int g0 = 0; g0 < ni_img; g0 += wg_max) {
                    const int gi = std::min(wg_max, ni_img - g0);
                    int wg_imgs = 1;
                    const ConvFn fn = conv_kernel(outs, rows, gi, &wg_imgs);
                    const unsigned threads = unsigned(128 / rows * wg_imgs);

                    // two codebook tiles (double buffered) when they fit in
                    // 64 KiB and the workgroup has four images' waves: with
                    // fewer waves per workgroup the doubled tile would cut the
                    // waves a CU can hold
                    const int dbuf = wg_imgs == kImgPerWg && 2 * size_t(L->kcent) * kTile * 8 <= 65536 ? 1 : 0;
                    const size_t lds_mac = size_t(1 + dbuf) * L->kcent * kTile * 8;
                    if (L->ext && tune_value(TK_CONV_FUSE)) {
                        // every output group in one launch (outputs in Y)
                        const int ngroups = (O + outs - 1) / outs;
                        const ConvOut yo{Y.u64() + size_t(g0) * O * lctw, size_t(O) * lctw, ngroups, O};
                        CKC_PROF(PK_CONV_CONTRACT, s,
                                 8.0 * N * (nlim * (2.0 * gi * nic * ntap + 2.0 * gi * O * (ic0 > 0 ? 2 : 1) +
                                                    double(L->npt) * L->kcent) -
                                            skipped * (2.0 * gi * nic + skipped_pt)),
                                 2.0 * N * double(gi) * O * nic * (double(nlim) * ntap - skipped));
                        count_variant("conv_mac", outs, wg_imgs,
                                      dbuf ? (rows == 2 ? "+dbuf+fused+rows2" : "+dbuf+fused")
                                           : (rows == 2 ? "+fused+rows2" : "+fused"));
                        hipLaunchKernelGGL(fn, dim3(unsigned(N / kTile) * unsigned(nlim) * unsigned(ngroups)),
                                           dim3(threads), lds_mac, s, R.u64() + size_t(g0) * r_img, r_img, gi,
                                           nic, I, ic0, ntap, nlim, map, L->pts.u64(), L->kcent, L->ioff.u64(),
                                           L->Opad / 4, bias_k, Ptrs{}, 0, 0, ic0 > 0 ? 1 : 0, c->dprimes(), c->logN,
                                           dbuf, skip_tap, L->pt_shared ? 1 : 0, seq_all, seq_skip, yo);
                        CKC_HIP(hipGetLastError());
                        continue;
                    }
                    for (int o0 = 0; o0 < O; o0 += outs) {
                        const int oc = std::min(outs, O - o0);
                        Ptrs op{};
                        for (int m = 0; m < gi; ++m)
                            for (int j = 0; j < oc; ++j) op.p[m * outs + j] = dest(g0 + m, o0 + j);
                        CKC_PROF(PK_CONV_CONTRACT, s,
                                 8.0 * N * (nlim * (2.0 * gi * nic * ntap + 2.0 * gi * oc * (ic0 > 0 ? 2 : 1) +
                                                    double(L->npt) * L->kcent) -
                                            skipped * (2.0 * gi * nic + skipped_pt)),
                                 2.0 * N * double(gi) * oc * nic * (double(nlim) * ntap - skipped));
                        count_variant("conv_mac", outs, wg_imgs,
                                      dbuf ? (rows == 2 ? "+dbuf+rows2" : "+dbuf") : (rows == 2 ? "+rows2" : ""));
                        hipLaunchKernelGGL(fn, dim3(unsigned(N / kTile), unsigned(nlim)), dim3(threads),
                                           lds_mac, s, R.u64() + size_t(g0) * r_img, r_img, gi, nic, I, ic0, ntap,
                                           nlim, map, L->pts.u64(), L->kcent, L->ioff.u64(), L->Opad / 4,
                                           bias_k, op, o0, oc, ic0 > 0 ? 1 : 0, c->dprimes(), c->logN, dbuf,
                                           skip_tap, L->pt_shared ? 1 : 0, seq_all, seq_skip,
                                           ConvOut{nullptr, 0, 0, 0});
                        CKC_HIP(hipGetLastError());
                    }
                }
            } else {
                // grouped form: per image, outputs in groups of kMaxBatch
                for (int ii = 0; ii < ni_img; ++ii) {
                    const uint64_t *Rimg = R.u64() + size_t(ii) * r_img;
                    for (int o0 = 0; o0 < O; o0 += kMaxBatch) {
                        const int oc = std::min(kMaxBatch, O - o0);
                        Ptrs op;
                        for (int j = 0; j < oc; ++j) op.p[j] = dest(ii, o0 + j);
                        const unsigned ogroups = unsigned((oc + kOutPerWg - 1) / kOutPerWg);
                        CKC_PROF(PK_CONV_CONTRACT, s,
                                 8.0 * N * nlim * (2.0 * I * ntap + 2.0 * oc + double(L->npt) * L->kcent),
                                 2.0 * N * nlim * double(oc) * I * ntap);
                        count_variant("conv_contract");
                        hipLaunchKernelGGL(k_conv_contract, dim3(unsigned(N / kTile), unsigned(nlim), 2 * ogroups),
                                           dim3(256), lds, s, Rimg, I, ntap, L->pt_shared ? 1 : 0, nlim, map,
                                           L->pts.u64(), L->kcent,
                                           (const int32_t *)L->og_off.p, (const int32_t *)L->g_c.p,
                                           (const int32_t *)L->g_moff.p, (const int32_t *)L->m_i.p, bias_k, op, o0,
                                           oc, c->dprimes(), c->logN);
                        CKC_HIP(hipGetLastError());
                    }
                }
            }
        }
        if (L->ext) {
            // one ModDown per output polynomial (bias added to polynomial 0)
            const int total = ni_img * O;
            for (int b0 = 0; b0 < total; b0 += kMaxBatch) {
                const int nb = std::min(kMaxBatch, total - b0);
                Ptrs o0{}, o1{}, bp{};
                for (int b = 0; b < nb; ++b) {
                    const int flat = b0 + b, m = flat / O, o = flat - m * O;
                    o0.p[b] = out[size_t(img0 + m) * O + o].d;
                    o1.p[b] = o0.p[b] + pw;
                    if (L->has_bias) bp.p[b] = L->bias.u64() + size_t(o) * pw;
                }
                CKC_TRY(moddown_b(c, Y.u64() + size_t(b0) * lctw, nb, L->level, L->has_bias ? &bp : nullptr, o0, o1,
                                  s));
            }
        }
    }
    for (int i = 0; i < n_img * L->O; ++i) {
        out[i].level = L->level;
        out[i].npoly = 2;
        out[i].scale = out_scale;
    }
    return CKC_OK;
}

namespace {
// D[b] = (x0 t0, x0 x1 + x1 t0, x1 x1) with t0 = x0 + bpt[b]  (NTT form)
__global__ __launch_bounds__(256) void k_act_tensor(Ptrs x, Ptrs bp, uint64_t *__restrict__ D, int nl,
                                                    const Prime *__restrict__ primes, int logN) {
    const int t = blockIdx.y, b = blockIdx.z;
    const size_t N = size_t(1) << logN, pw = size_t(nl) * N;
    const Prime P = primes[t];
    const uint64_t *x0 = x.p[b] + size_t(t) * N, *x1 = x.p[b] + pw + size_t(t) * N;
    const uint64_t *bb = bp.p[b] + size_t(t) * N;
    uint64_t *d = D + b * 3 * pw + size_t(t) * N;
    for (size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x; k < N; k += size_t(gridDim.x) * blockDim.x) {
        const uint64_t a0 = x0[k], a1 = x1[k];
        const uint64_t t0 = add_mod(a0, bb[k], P.q);
        d[k] = mul_mod(a0, t0, P);
        d[pw + k] = reduce128(add128(mul64x64(a0, a1), mul64x64(a1, t0)), P);
        d[2 * pw + k] = mul_mod(a1, a1, P);
    }
}
}  // namespace

extern "C" int ckc_eval_quad_act(ckc_ctx *c, const ckc_evk *evk, const ckc_layer *L, const ckc_ct *in, int n_img,
                                 ckc_ct *out, void *stream) {
    CKC_FAULT_POINT();
    CKC_REQUIRE(c && evk && L && in && out && n_img >= 0, CKC_EINVAL, "null argument");
    CKC_REQUIRE(L->kind == LK_ACT, CKC_EINVAL, "not an activation layer");
    CKC_TRY(check_evk_images(evk, n_img, "eval_quad_act"));
    for (int i = 0; i < (evk->is_group() ? n_img : 1); ++i)
        CKC_REQUIRE(evk_of(evk, i)->relin, CKC_ENOKEY, "no relinearisation key");
    if (n_img == 0) return CKC_OK;
    const int total = n_img * L->C;
    CKC_TRY(check_inputs(in, total, L->level, "eval_quad_act"));
    CKC_REQUIRE(fabs(in[0].scale / L->in_scale - 1.0) <= ldexp(1.0, -30), CKC_ESCALE,
                "eval_quad_act: input scale differs from the layer's");
    for (int i = 0; i < total; ++i) CKC_REQUIRE(out[i].d, CKC_EINVAL, "eval_quad_act: null output");
    hipStream_t s = S(stream);
    const size_t N = c->N;
    const int nl = L->level + 1, nt = nl + c->np, dnum = c->dnum_at(L->level);
    const size_t pw = size_t(nl) * N;
    const int nbmax = std::min(kMaxBatch, total);
    DevBuf D, digits;
    CKC_TRY(D.alloc(8 * 3 * pw * nbmax, s));
    CKC_TRY(digits.alloc(8 * N * nt * dnum * nbmax, s));
    for (int b0 = 0, nb = 0; b0 < total; b0 += nb) {
        // a batch shares one relinearisation key (a key group splits it)
        nb = key_run(evk, b0, std::min(kMaxBatch, total - b0), L->C);
        const ckc_evk *ek = evk_of(evk, b0 / L->C);
        Ptrs xp, bp, cp, a0, a1, o0, o1;
        for (int b = 0; b < nb; ++b) {
            const int ch = (b0 + b) % L->C;
            xp.p[b] = in[b0 + b].d;
            bp.p[b] = L->bpt.u64() + size_t(ch) * pw;
            cp.p[b] = L->cpt.u64() + size_t(ch) * pw;
            a0.p[b] = D.u64() + size_t(b) * 3 * pw;
            a1.p[b] = a0.p[b] + pw;
            o0.p[b] = out[b0 + b].d;
            o1.p[b] = out[b0 + b].d + pw;
        }
        {
            CKC_PROF(PK_ACT_TENSOR, s, 8.0 * N * nl * nb * 6.0, 0.0);
        hipLaunchKernelGGL(k_act_tensor, dim3(tiles(N), unsigned(nl), unsigned(nb)), dim3(256), 0, s, xp, bp, D.u64(),
                           nl, c->dprimes(), c->logN);
        }
        CKC_HIP(hipGetLastError());
        CKC_TRY(ks_modup_b(c, D.u64() + 2 * pw, 3 * pw, nb, L->level, digits.u64(), s));
        CKC_TRY(ks_apply_b(c, digits.u64(), nb, L->level, ek->relin->u64(), 1, &a0, &a1, false, o0, o1, s));
        CKC_TRY(ew_b(c, EW_ADD, o0, o0, &cp, nb, 1, nl, s));
    }
    const double sc = (in[0].scale * in[0].scale) / L->a_absorb;
    for (int i = 0; i < total; ++i) {
        out[i].level = L->level;
        out[i].npoly = 2;
        out[i].scale = sc;
    }
    return CKC_OK;
}

namespace {
// Z[img][k][p] = sum_c PT[k][c] * S[img][c][p] (+ bias[k] on p = 0); images of one launch: up to 8
constexpr int kDenseImg = 8;
// With one member the weights and biases are constants (consts [K][C][nl],
// bconsts [K][nl]): in NTT form a constant polynomial is the same value in
// every coefficient.
__global__ __launch_bounds__(256) void k_dense_mac(const uint64_t *__restrict__ Sb, int nimg, int C, int nl,
                                                   const uint64_t *__restrict__ pts, const uint64_t *__restrict__ bias,
                                                   const uint64_t *__restrict__ consts,
                                                   const uint64_t *__restrict__ bconsts, uint64_t *__restrict__ Z,
                                                   int K, const Prime *__restrict__ primes, int logN) {
    // one 256-coefficient chunk of one (limb, polynomial) per block, block id
    // -> (class kk, group) with the group's low 3 bits equal to id mod 8: the
    // K class blocks of a group are dispatched within 8 K consecutive ids to
    // the same XCD (workgroups go round-robin over the 8 XCDs), so all but
    // the first read the group's inputs S from that XCD's L2 (without this
    // every class re-read S from HBM)
    const unsigned id = blockIdx.x;
    const unsigned j = id >> 3, kk = j % unsigned(K), grp = (j / unsigned(K)) * 8u + (id & 7u);
    const unsigned nchunk = unsigned(size_t(1) << logN) / 256u;
    const int chunk = int(grp % nchunk), limb = int((grp / nchunk) % unsigned(nl)),
              poly = int(grp / (nchunk * unsigned(nl)));
    const size_t N = size_t(1) << logN, pw = size_t(nl) * N;
    const Prime P = primes[limb];
    const int pcap = fold_cap(P.k);
    const uint64_t r64 = P.r2;  // 2^64 mod q
    {
        const size_t k = size_t(chunk) * 256 + threadIdx.x;
        accc acc[kDenseImg];
        for (int i = 0; i < kDenseImg; ++i) acc[i] = accc{0, 0, 0, 0, 0};
        int cnt = 0;
        for (int ch = 0; ch < C; ++ch) {
            const uint64_t pv = consts ? consts[(size_t(kk) * C + ch) * nl + limb]
                                       : pts[(size_t(kk) * C + ch) * pw + size_t(limb) * N + k];
#pragma unroll
            for (int i = 0; i < kDenseImg; ++i)
                if (i < nimg) macc(acc[i], Sb[((size_t(i) * C + ch) * 2 + poly) * pw + size_t(limb) * N + k], pv);
            if (++cnt == pcap) {
#pragma unroll
                for (int i = 0; i < kDenseImg; ++i) {
                    const u128v v = accc_value(acc[i]);  // macc_folded, written out as in k_conv_mac
                    acc[i] = accc{0, 0, v.lo, 0, 0};
                    macc(acc[i], v.hi, r64);
                }
                cnt = 0;
            }
        }
#pragma unroll
        for (int i = 0; i < kDenseImg; ++i) {
            if (i >= nimg) continue;
            uint64_t y = reduce128(accc_value(acc[i]), P);
            if (poly == 0 && bias) y = add_mod(y, bias[size_t(kk) * pw + size_t(limb) * N + k], P.q);
            if (poly == 0 && bconsts) y = add_mod(y, bconsts[size_t(kk) * nl + limb], P.q);
            Z[((size_t(i) * K + kk) * 2 + poly) * pw + size_t(limb) * N + k] = y;
        }
    }
}
}  // namespace

extern "C" int ckc_eval_dense(ckc_ctx *c, const ckc_evk *evk, const ckc_layer *L, const ckc_ct *in, int n_img,
                              ckc_ct *out, void *stream) {
    CKC_FAULT_POINT();
    CKC_REQUIRE(c && evk && L && in && out && n_img >= 0, CKC_EINVAL, "null argument");
    CKC_REQUIRE(L->kind == LK_DENSE, CKC_EINVAL, "not a dense layer");
    CKC_TRY(check_evk_images(evk, n_img, "eval_dense"));
    if (n_img == 0) return CKC_OK;
    const int C = L->C, K = L->K;
    CKC_TRY(check_inputs(in, n_img * C, L->level, "eval_dense"));
    for (int i = 0; i < n_img * K; ++i) CKC_REQUIRE(out[i].d, CKC_EINVAL, "eval_dense: null output");
    const double out_scale = in[0].scale * L->pt_scale;
    if (L->has_bias)
        CKC_REQUIRE(fabs(out_scale / L->bias_scale - 1.0) <= ldexp(1.0, -30), CKC_ESCALE,
                    "eval_dense: bias scale does not match in.scale * pt_scale");
    hipStream_t s = S(stream);
    const size_t N = c->N;
    const int nl = L->level + 1;
    const size_t pw = size_t(nl) * N, ctw = 2 * pw;
    for (int img0 = 0; img0 < n_img; img0 += kDenseImg) {
        const int ni = std::min(kDenseImg, n_img - img0);
        const int total = ni * C;
        DevBuf Sb, Tb, Z;
        CKC_TRY(Sb.alloc(8 * ctw * total, s));
        // rotated copies of one batch of the summed ciphertexts (inputs, or
        // in the spatial form the K outputs of each image)
        CKC_TRY(Tb.alloc(8 * ctw * std::min(L->spatial ? ni * K : total, kMaxBatch), s));
        CKC_TRY(Z.alloc(8 * ctw * ni * K, s));
        // S = inputs
        for (int b0 = 0; b0 < total; b0 += kMaxBatch) {
            const int nb = std::min(kMaxBatch, total - b0);
            Ptrs ip;
            for (int b = 0; b < nb; ++b) ip.p[b] = in[size_t(img0) * C + b0 + b].d;
            CKC_TRY(gather(ip, 0, Sb.u64() + size_t(b0) * ctw, ctw, ctw, nb, s));
        }
        // rotation sums X <- X + Rot_step(X), steps in order, over the n
        // ciphertexts at X (per image, `per` of them)
        auto slot_sums = [&](uint64_t *X, int n, int per) -> int {
            for (int32_t st : L->sum_steps) {
                for (int b0 = 0, nb = 0; b0 < n; b0 += nb) {
                    // a batch shares one key set (a key group splits it)
                    nb = key_run(evk, img0 * per + b0, std::min(kMaxBatch, n - b0), per);
                    const ckc_evk *ek = evk_of(evk, img0 + b0 / per);
                    Ptrs sp, tp;
                    for (int b = 0; b < nb; ++b) {
                        sp.p[b] = X + size_t(b0 + b) * ctw;
                        tp.p[b] = Tb.u64() + size_t(b) * ctw;
                    }
                    std::vector<Ptrs> dst{tp};
                    CKC_TRY(hoisted_group(c, ek, sp, nb, L->level, std::vector<int32_t>{st}, dst, s));
                    CKC_TRY(ew_b(c, EW_ADD, sp, sp, &tp, nb, 2, nl, s));
                }
            }
            return CKC_OK;
        };
        // grid-average form: the channels' slot sums first; spatial form:
        // the products first, then the slot sums of the K outputs
        if (!L->spatial) CKC_TRY(slot_sums(Sb.u64(), total, C));
        {
            CKC_PROF(PK_DENSE_MAC, s, 8.0 * N * nl * (2.0 * ni * C + double(K) * C + 2.0 * ni * K),
                     2.0 * N * nl * double(ni) * K * C);
        // groups (chunk, limb, polynomial): N / 256 chunks, a multiple of 8 for N >= 2^11
        const size_t groups = (N / 256) * size_t(nl) * 2;
        hipLaunchKernelGGL(k_dense_mac, dim3(unsigned(groups * K)), dim3(256), 0, s, Sb.u64(), ni, C, nl,
                           L->pts.u64(), L->bias.u64(), L->dconst.u64(), L->bconst.u64(), Z.u64(), K, c->dprimes(),
                           c->logN);
        }
        CKC_HIP(hipGetLastError());
        if (L->spatial) CKC_TRY(slot_sums(Z.u64(), ni * K, K));
        for (int b0 = 0; b0 < ni * K; b0 += kMaxBatch) {
            const int nb = std::min(kMaxBatch, ni * K - b0);
            Ptrs op;
            for (int b = 0; b < nb; ++b) op.p[b] = out[size_t(img0) * K + b0 + b].d;
            hipLaunchKernelGGL(k_scatter, dim3(1024, unsigned(nb)), dim3(256), 0, s, Z.u64() + size_t(b0) * ctw, ctw, op,
                               ctw);
            CKC_HIP(hipGetLastError());
        }
    }
    for (int i = 0; i < n_img * K; ++i) {
        out[i].level = L->level;
        out[i].npoly = 2;
        out[i].scale = out_scale;
    }
    return CKC_OK;
}

extern "C" int ckc_eval_avgpool2(ckc_ctx *c, const ckc_evk *evk, const ckc_layout *layout, const ckc_ct *in, int n,
                                 ckc_ct *out, void *stream) {
    CKC_FAULT_POINT();
    CKC_REQUIRE(c && evk && layout && in && out && n >= 0, CKC_EINVAL, "null argument");
    CKC_TRY(check_layout(c, layout));
    CKC_REQUIRE(layout->height % 2 == 0 && layout->width % 2 == 0, CKC_ESHAPE, "pool: odd grid");
    // with a key group of G images, ciphertext i belongs to image i / (n / G)
    const int G = evk->is_group() ? int(evk->key_of_img.size()) : 1;
    CKC_REQUIRE(n % G == 0, CKC_EINVAL, "eval_avgpool2: ciphertexts not a multiple of the key group's images");
    const int per_img = n / G > 0 ? n / G : 1;
    if (n == 0) return CKC_OK;
    CKC_TRY(check_inputs(in, n, in[0].level, "eval_avgpool2"));
    hipStream_t s = S(stream);
    const int level = in[0].level, nl = level + 1;
    const size_t pw = size_t(nl) * c->N, ctw = 2 * pw;
    const int g = layout->gap, W0 = layout->row_stride;
    const std::vector<int32_t> steps{g, g * W0, g * (W0 + 1)};
    const int nbmax = std::min(kMaxBatch, n);
    DevBuf T;
    CKC_TRY(T.alloc(8 * ctw * 3 * nbmax, s));
    for (int b0 = 0, nb = 0; b0 < n; b0 += nb) {
        nb = key_run(evk, b0, std::min(kMaxBatch, n - b0), per_img);
        const ckc_evk *ek = evk_of(evk, b0 / per_img);
        Ptrs ip, op;
        std::vector<Ptrs> dst(3);
        for (int b = 0; b < nb; ++b) {
            ip.p[b] = in[b0 + b].d;
            op.p[b] = out[b0 + b].d;
            for (int j = 0; j < 3; ++j) dst[j].p[b] = T.u64() + (size_t(b) * 3 + j) * ctw;
        }
        CKC_TRY(hoisted_group(c, ek, ip, nb, level, steps, dst, s));
        CKC_TRY(ew_b(c, EW_ADD, op, ip, &dst[0], nb, 2, nl, s));
        CKC_TRY(ew_b(c, EW_ADD, op, op, &dst[1], nb, 2, nl, s));
        CKC_TRY(ew_b(c, EW_ADD, op, op, &dst[2], nb, 2, nl, s));
    }
    for (int i = 0; i < n; ++i) {
        out[i].level = level;
        out[i].npoly = 2;
        out[i].scale = in[i].scale;
    }
    return CKC_OK;
}

extern "C" int ckc_rescale_many(ckc_ctx *c, const ckc_ct *in, int n, ckc_ct *out, void *stream) {
    CKC_REQUIRE(c && in && out && n >= 0, CKC_EINVAL, "null argument");
    if (n == 0) return CKC_OK;
    const int level = in[0].level, npoly = in[0].npoly;
    CKC_REQUIRE(level >= 1, CKC_ELEVEL, "cannot rescale at level 0");
    for (int i = 0; i < n; ++i) {
        CKC_REQUIRE(in[i].d && out[i].d && in[i].level == level && in[i].npoly == npoly, CKC_ESHAPE,
                    "rescale_many: inputs must share level and npoly");
        for (int j = 0; j < n; ++j) CKC_REQUIRE(out[i].d != in[j].d, CKC_EINVAL, "rescale_many: output aliases an input");
    }
    hipStream_t s = S(stream);
    for (int b0 = 0; b0 < n; b0 += kMaxBatch) {
        const int nb = std::min(kMaxBatch, n - b0);
        Ptrs ip, op;
        for (int b = 0; b < nb; ++b) {
            ip.p[b] = in[b0 + b].d;
            op.p[b] = out[b0 + b].d;
        }
        CKC_TRY(rescale_b(c, ip, op, nb, npoly, level, s));
    }
    for (int i = 0; i < n; ++i) {
        out[i].scale = in[i].scale / double(c->mods[level]);
        out[i].level = level - 1;
        out[i].npoly = npoly;
    }
    return CKC_OK;
}

extern "C" int ckc_add_many(ckc_ctx *c, const ckc_ct *a, const ckc_ct *b, int n, ckc_ct *out, void *stream) {
    CKC_REQUIRE(c && a && b && out && n >= 0, CKC_EINVAL, "null argument");
    if (n == 0) return CKC_OK;
    const int level = a[0].level;
    for (int i = 0; i < n; ++i) {
        CKC_REQUIRE(a[i].d && b[i].d && out[i].d, CKC_EINVAL, "add_many: null buffer");
        CKC_REQUIRE(a[i].level == level && b[i].level == level, CKC_ELEVEL, "add_many: levels differ");
        CKC_REQUIRE(a[i].npoly == 2 && b[i].npoly == 2, CKC_ESHAPE, "add_many: 2-poly ciphertexts only");
        CKC_REQUIRE(fabs(a[i].scale / b[i].scale - 1.0) <= ldexp(1.0, -30), CKC_ESCALE, "add_many: scales differ");
    }
    hipStream_t s = S(stream);
    for (int b0 = 0; b0 < n; b0 += kMaxBatch) {
        const int nb = std::min(kMaxBatch, n - b0);
        Ptrs ap, bp, op;
        for (int j = 0; j < nb; ++j) {
            ap.p[j] = a[b0 + j].d;
            bp.p[j] = b[b0 + j].d;
            op.p[j] = out[b0 + j].d;
        }
        CKC_TRY(ew_b(c, EW_ADD, op, ap, &bp, nb, 2, level + 1, s));
    }
    for (int i = 0; i < n; ++i) {
        out[i].level = level;
        out[i].npoly = 2;
        out[i].scale = a[i].scale;
    }
    return CKC_OK;
}
