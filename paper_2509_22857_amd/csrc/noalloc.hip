// Relinearisation that allocates nothing: for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops).  Its
// scratch (the ModUp digits, the key inner product's outputs and ModDown's
// conversion) lives in one file-scope device array instead of the stream's
// arena; the kernels are those of ckc_relin.
#include <mutex>

#include "ckc_internal.h"

constexpr size_t kScratchBytes = size_t(256) << 20;

// Each GPU that loads the library holds its own copy until the process ends.
// Host code never uses this name as an address: noalloc_scratch() looks up
// the device address once per device, at the first call of an entry point
// that uses it on that device (the lookup loads the library's code object,
// which a context's creation does not do: it runs before the caller's
// framework has set up the device).
static __device__ __align__(256) uint64_t scratch[kScratchBytes / 8];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};
}  // namespace

int noalloc_scratch(void **ptr) {
    int dev = 0;
    CKC_HIP(hipGetDevice(&dev));
    CKC_REQUIRE(dev >= 0 && dev < kMaxDevices, CKC_EDEVICE, "device index beyond the static scratch table");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            ckc_set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
            return CKC_EDEVICE;
        }
        g_ptr[dev] = p;
    }
    *ptr = g_ptr[dev];
    return CKC_OK;
}

namespace {
// installs a fixed region as the calling thread's scratch for one call
struct FixedGuard {
    FixedScratch fs;
    FixedScratch *prev;
    FixedGuard(void *base, size_t cap) : prev(t_fixed_scratch) {
        fs.base = (char *)base;
        fs.cap = cap;
        t_fixed_scratch = &fs;
    }
    ~FixedGuard() { t_fixed_scratch = prev; }
};
}  // namespace

extern "C" size_t ckc_relin_noalloc_bytes(const ckc_ctx *c, int level) {
    if (!c || level < 0 || level >= c->nq) return 0;
    return relin_scratch_bytes(c, level);
}

extern "C" size_t ckc_noalloc_capacity(void) { return kScratchBytes; }

extern "C" int ckc_relin_noalloc(ckc_ctx *c, const ckc_evk *evk, const ckc_ct *in, ckc_ct *out, void *stream) {
    CKC_REQUIRE(c && in, CKC_EINVAL, "null argument");
    CKC_REQUIRE(in->level >= 0 && in->level < c->nq, CKC_ELEVEL, "relin_noalloc: level out of range");
    const size_t need = relin_scratch_bytes(c, in->level);
    CKC_REQUIRE(need <= kScratchBytes, CKC_ENOMEM,
                "relin_noalloc: a ciphertext at level " + std::to_string(in->level) + " needs " +
                    std::to_string(need) + " bytes of scratch; the static scratch holds " +
                    std::to_string(kScratchBytes));
    void *base = nullptr;
    CKC_TRY(noalloc_scratch(&base));
    FixedGuard g(base, kScratchBytes);
    return relin_impl(c, evk, in, out, stream);
}
