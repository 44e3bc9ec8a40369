// Internal declarations of the gfx950 RNS-CKKS library (not part of the C-ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/ckkscnn.h"
#include "modarith.h"

// ---------------------------------------------------------------- errors
void ckc_set_error(const std::string &msg);
// test-only fault injection (ckc_set_test_fault): nonzero = the code this
// call must return instead of running
int test_fault_take();
#define CKC_FAULT_POINT()                          \
    do {                                           \
        const int _f = test_fault_take();          \
        if (_f != 0) {                             \
            ckc_set_error("injected test fault");  \
            return _f;                             \
        }                                          \
    } while (0)

#define CKC_HIP(call)                                                        \
    do {                                                                     \
        hipError_t _e = (call);                                              \
        if (_e != hipSuccess) {                                              \
            ckc_set_error(std::string(#call) + ": " + hipGetErrorString(_e)); \
            return CKC_EDEVICE;                                              \
        }                                                                    \
    } while (0)

#define CKC_REQUIRE(cond, code, msg)  \
    do {                              \
        if (!(cond)) {                \
            ckc_set_error(msg);       \
            return (code);            \
        }                             \
    } while (0)

#define CKC_TRY(expr)              \
    do {                           \
        int _rc = (expr);          \
        if (_rc != CKC_OK) return _rc; \
    } while (0)

// ---------------------------------------------------------------- limb maps
// Limb i of an array maps to prime index (i < nlow ? i : pbase + i - nlow).
// A Q-only array uses nlow = INT32_MAX.  An extended basis at level l uses
// nlow = l + 1, pbase = number of Q primes.
struct LimbMap {
    int32_t nlow;
    int32_t pbase;
    CKC_HD int prime(int i) const { return i < nlow ? i : pbase + (i - nlow); }
};
static inline LimbMap qmap() { return LimbMap{0x7fffffff, 0}; }

// Per-stream scratch arena.  Every call takes its temporary buffers from the
// arena of the stream it runs on, stack-wise; the arena keeps one device
// buffer that grows to the most scratch any call has held at once and is
// reused by every later call on that stream (work on one stream runs in
// order, so a later call may reuse what an earlier one released while its
// kernels are still queued).  Steady-state calls therefore make no
// allocation API calls.  When a request does not fit while other buffers are
// live, it is served from the stream-ordered allocator and the arena grows to
// cover it the next time it is empty.
struct Arena;
int arena_alloc(hipStream_t s, size_t bytes, void **p, Arena **a, size_t *off);
void arena_release(Arena *a, size_t off, void *p, hipStream_t s);
// release the unused arenas of the current device (their streams idle)
void arena_trim();
// frees the arena of (current device, s) once the stream is idle
int arena_trim_stream(hipStream_t s);
// grows the (idle) arena of (current device, s) to at least `bytes`
int arena_reserve_stream(hipStream_t s, size_t bytes);

// A fixed device region that, while installed on the calling thread, serves
// every DevBuf of that thread stack-wise in place of the stream's arena: no
// allocation API call is made, and a request beyond its capacity fails with
// CKC_ENOMEM.  Used by the entry points that must not allocate.
struct FixedScratch {
    char *base = nullptr;
    size_t cap = 0, top = 0, high = 0;
};
extern thread_local FixedScratch *t_fixed_scratch;
int fixed_alloc(FixedScratch *f, size_t bytes, void **p, size_t *off);
void fixed_release(FixedScratch *f, size_t off, size_t bytes);

// RAII scratch buffer from the stream's arena (or the installed fixed region).
struct DevBuf {
    void *p = nullptr;
    hipStream_t s = nullptr;
    Arena *a = nullptr;
    FixedScratch *f = nullptr;
    size_t off = 0, bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() {
        if (p && f) fixed_release(f, off, bytes);
        else if (p) arena_release(a, off, p, s);
    }
    int alloc(size_t nbytes, hipStream_t st) {
        s = st;
        if (nbytes == 0) nbytes = 256;
        if (t_fixed_scratch) {
            f = t_fixed_scratch;
            bytes = (nbytes + 255) / 256 * 256;
            return fixed_alloc(f, bytes, &p, &off);
        }
        return arena_alloc(st, nbytes, &p, &a, &off);
    }
    uint64_t *u64() const { return (uint64_t *)p; }
};

// Persistent device allocation owned by a handle.
struct DevMem {
    void *p = nullptr;
    size_t bytes = 0;
    ~DevMem() {
        if (p) (void)hipFree(p);
    }
    int alloc(size_t b) {
        bytes = b;
        hipError_t e = hipMalloc(&p, b ? b : 256);
        if (e != hipSuccess) {
            p = nullptr;
            ckc_set_error(std::string("hipMalloc: ") + hipGetErrorString(e));
            (void)hipGetLastError();  // reported here, not by the next launch check
            return CKC_ENOMEM;
        }
        return CKC_OK;
    }
    int upload(const void *h, size_t b) {
        CKC_TRY(alloc(b));
        CKC_HIP(hipMemcpy(p, h, b, hipMemcpyHostToDevice));
        return CKC_OK;
    }
    uint64_t *u64() const { return (uint64_t *)p; }
};

// Fast basis conversion constants for a source set of primes S -> targets T:
//   y_i = [x_i * (S/s_i)^-1]_{s_i};   out_t = sum_i y_i * (S/s_i mod t)  (mod t)
struct BconvTable {
    int ns = 0, nt = 0;
    DevMem inv;     // [ns] (S/s_i)^-1 mod s_i
    DevMem invp;    // [ns] Shoup companions
    DevMem hat;     // [nt][ns] S/s_i mod t
    DevMem neg_s;   // [nt] (-S) 2^64 mod t: the centring correction of the conversion
    DevMem s_half;  // [ns] s_i >> 1: a source value above it stands for value - s_i
    std::vector<uint64_t> iscale_h;  // [ns][2] N^-1 (S/s_i)^-1 mod s_i and its Shoup companion
    DevMem iscale;  // device copy: the last multiply of an INTT that feeds the conversion
};

struct ckc_ctx {
    int logN = 0;
    size_t N = 0;
    int nq = 0, np = 0, alpha = 1;
    std::vector<uint64_t> mods;     // Q primes then P primes
    std::vector<Prime> primes_h;
    std::vector<uint64_t> psi_h;    // chosen 2N-th roots
    DevMem primes_d;                // Prime[nprimes]
    DevMem tw, twp, itw, itwp;      // [nprimes][N] bit-reversed psi powers (+Shoup)
    DevMem ninv;                    // [nprimes][2] N^-1 and its Shoup companion
    // encoding FFT tables (host-computed from a fixed series, uploaded)
    DevMem fft_w;                   // [n/2] double2 (cos, sin) of 2 pi e / n
    DevMem twist;                   // [n]   double2 (cos, sin) of pi k / N
    DevMem slot_idx;                // [n]   uint32  t_j = (5^j mod 2N - 1)/4
    // rescale: for level l, [i < l] (q_l^-1 mod q_i, Shoup)
    DevMem rescale_inv;             // [nq][nq][2]
    // ModDown P -> Q constants for every Q prime: P^-1 mod q_i (Shoup)
    DevMem pinv;                    // [nq][2]
    DevMem pmod;                    // [nq][2] P mod q_i (Shoup): lifting into Q u P as P x
    BconvTable p_to_q;              // P -> q_0..q_{nq-1}
    // ModUp tables per (level, digit)
    std::mutex mu;
    std::map<std::pair<int, int>, std::unique_ptr<BconvTable>> modup_tabs;
    std::map<uint64_t, std::unique_ptr<DevMem>> galois_perm;   // NTT-domain permutations
    std::map<int, std::unique_ptr<DevMem>> modup_scale;        // per level: [l+1][2] INTT scale of ModUp

    int nprimes() const { return nq + np; }
    const Prime *dprimes() const { return (const Prime *)primes_d.p; }
    int dnum_at(int level) const { return (level + 1 + alpha - 1) / alpha; }
};

struct ckc_sk {
    uint64_t seed = 0;
    std::vector<int8_t> s;          // ternary coefficients (host, client side)
    DevMem s_ntt;                   // [nprimes][N] s in NTT form, every prime
};

struct ckc_evk {
    int dnum = 0;
    size_t key_words = 0;           // words per key: dnum * 2 * nprimes * N
    std::unique_ptr<DevMem> relin;  // may be null
    std::map<uint64_t, std::unique_ptr<DevMem>> galois;  // Galois element -> key
    // a key group (ckc_evk_group_create): the key set of every image of a
    // batched layer call, by image index; the member key sets stay their
    // owners'
    std::vector<const ckc_evk *> members;
    std::vector<int32_t> key_of_img;
    bool is_group() const { return !members.empty(); }
};
// key set of image `img` of a layer call (a plain key set serves every image)
inline const ckc_evk *evk_of(const ckc_evk *e, int img) {
    return e->is_group() ? e->members[size_t(e->key_of_img[size_t(img)])] : e;
}
// items first .. first + n - 1 of a layer call, item i of image i / per_img:
// how many of them, from `first`, share one key set (at least 1)
inline int key_run(const ckc_evk *e, int first, int n, int per_img) {
    if (!e->is_group()) return n;
    const int32_t k = e->key_of_img[size_t(first / per_img)];
    int r = 1;
    while (r < n && e->key_of_img[size_t((first + r) / per_img)] == k) ++r;
    return r;
}
// a layer call on n_img images accepts a plain key set or a group of n_img images
int check_evk_images(const ckc_evk *e, int n_img, const char *what);

// ---------------------------------------------------------------- launchers
// (all asynchronous on the given stream; data pointers are device pointers)
int ntt_forward(const ckc_ctx *c, uint64_t *d, int nlimbs, LimbMap map, int nbatch, size_t batch_stride,
                hipStream_t s, int skip_lo = -1, int skip_hi = -1);
// inverse transform; scale2 (optional, [nlimbs][2] value + Shoup companion)
// replaces the final multiply by N^-1 per limb; src (optional) makes it
// out of place (src batch stride src_bs, same limb layout)
int ntt_inverse(const ckc_ctx *c, uint64_t *d, int nlimbs, LimbMap map, int nbatch, size_t batch_stride,
                hipStream_t s, const uint64_t *scale2 = nullptr, const uint64_t *src = nullptr, size_t src_bs = 0);

enum EwOp { EW_ADD = 0, EW_SUB = 1, EW_MUL = 2, EW_NEG = 3, EW_COPY = 4 };
// out[p][l] = a[p][l] op b[bp][l] over npoly polys of nlimbs limbs (prime l via map);
// b_poly_stride = 0 broadcasts one b polynomial to every poly of a.
int ew_binary(const ckc_ctx *c, EwOp op, uint64_t *out, const uint64_t *a, const uint64_t *b, int npoly,
              int nlimbs, size_t a_poly_stride, size_t b_poly_stride, size_t out_poly_stride, LimbMap map,
              hipStream_t s);

const BconvTable *modup_table(ckc_ctx *c, int level, int digit, int *rc);
// [level+1][2]: for limb i of digit j, N^-1 (D_j/q_i)^-1 mod q_i (+ Shoup)
const uint64_t *modup_scale(ckc_ctx *c, int level, int *rc);
const uint64_t *galois_table(ckc_ctx *c, uint64_t g, int *rc);
uint64_t galois_element(const ckc_ctx *c, int64_t step);

int rescale_impl(ckc_ctx *c, const uint64_t *in, int npoly, int level, uint64_t *out, hipStream_t s);
// relinearisation (argument checks included) on the calling thread's scratch
int relin_impl(ckc_ctx *c, const ckc_evk *evk, const ckc_ct *in, ckc_ct *out, void *stream);
// scratch bytes relin_impl holds at once for a ciphertext at `level`
size_t relin_scratch_bytes(const ckc_ctx *c, int level);
// device address of the no-allocation entry points' static scratch on the
// current device (looked up once per device)
int noalloc_scratch(void **ptr);

size_t words_ct(const ckc_ctx *c, int level, int npoly);
