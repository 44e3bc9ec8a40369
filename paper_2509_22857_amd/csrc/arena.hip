// Per-stream scratch arenas (see DevBuf): one growable device buffer per
// (device, stream), sub-allocated stack-wise by the calls on that stream.
#include <algorithm>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "ckc_internal.h"

struct Arena {
    std::mutex mu;
    int dev = 0;
    hipStream_t s = nullptr;
    char *base = nullptr;
    size_t cap = 0;
    size_t top = 0;
    size_t high = 0;          // most scratch (arena + overflow) live at once
    size_t overflow_live = 0; // bytes currently served outside the arena
    struct Slot {
        void *ptr;
        size_t off, bytes;  // off = SIZE_MAX: served outside the arena
        bool live;
    };
    std::vector<Slot> stack;
};

namespace {
constexpr size_t kAlign = 256;
std::mutex g_mu;
std::map<std::pair<int, hipStream_t>, Arena *> g_arenas;

Arena *arena_for(hipStream_t s, int *rc) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        ckc_set_error(std::string("hipGetDevice: ") + hipGetErrorString(e));
        *rc = CKC_EDEVICE;
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    Arena *&a = g_arenas[{dev, s}];
    if (!a) {
        a = new Arena;
        a->dev = dev;
        a->s = s;
    }
    return a;
}
}  // namespace

int arena_alloc(hipStream_t s, size_t bytes, void **p, Arena **out, size_t *off) {
    int rc = CKC_OK;
    Arena *a = arena_for(s, &rc);
    if (!a) return rc;
    bytes = (bytes + kAlign - 1) / kAlign * kAlign;
    std::lock_guard<std::mutex> lk(a->mu);
    if (a->top == 0 && a->overflow_live == 0) {
        // empty: grow to the high-water mark first if this request or an
        // earlier overflow asks for more than the buffer holds
        const size_t want = std::max(bytes, a->high);
        if (want > a->cap) {
            if (a->base) {
                // earlier calls on the stream may still use the old buffer
                CKC_HIP(hipStreamSynchronize(s));
                CKC_HIP(hipFree(a->base));
                a->base = nullptr;
                a->cap = 0;
            }
            // overflow buffers of earlier calls went back to the device's
            // default pool, which keeps them: return them to the device first
            hipMemPool_t pool;
            if (a->high > 0 && hipDeviceGetDefaultMemPool(&pool, a->dev) == hipSuccess) {
                CKC_HIP(hipStreamSynchronize(s));
                (void)hipMemPoolTrimTo(pool, 0);
            }
            hipError_t e = hipMalloc((void **)&a->base, want);
            if (e != hipSuccess) {
                a->base = nullptr;
                ckc_set_error(std::string("scratch arena hipMalloc: ") + hipGetErrorString(e));
                (void)hipGetLastError();  // the failure is reported here, not by the next launch check
                return CKC_ENOMEM;
            }
            a->cap = want;
        }
    }
    if (a->top + bytes <= a->cap) {
        *p = a->base + a->top;
        *off = a->top;
        a->stack.push_back(Arena::Slot{*p, a->top, bytes, true});
        a->top += bytes;
    } else {
        hipError_t e = hipMallocAsync(p, bytes, s);
        if (e != hipSuccess) {
            *p = nullptr;
            ckc_set_error(std::string("hipMallocAsync: ") + hipGetErrorString(e));
            (void)hipGetLastError();  // reported here, not by the next launch check
            return CKC_ENOMEM;
        }
        *off = SIZE_MAX;
        a->overflow_live += bytes;
        a->stack.push_back(Arena::Slot{*p, SIZE_MAX, bytes, true});
    }
    a->high = std::max(a->high, a->top + a->overflow_live);
    *out = a;
    return CKC_OK;
}

void arena_release(Arena *a, size_t off, void *p, hipStream_t s) {
    (void)off;
    std::lock_guard<std::mutex> lk(a->mu);
    // mark the slot released (search from the top: releases are nearly LIFO)
    for (size_t i = a->stack.size(); i-- > 0;) {
        Arena::Slot &sl = a->stack[i];
        if (!sl.live || sl.ptr != p) continue;
        if (sl.off == SIZE_MAX) {
            (void)hipFreeAsync(p, s);
            a->overflow_live -= sl.bytes;
        }
        sl.live = false;
        break;
    }
    // pop released slots off the top; the arena's top falls to the lowest
    // popped arena slot
    while (!a->stack.empty() && !a->stack.back().live) {
        if (a->stack.back().off != SIZE_MAX) a->top = a->stack.back().off;
        a->stack.pop_back();
    }
}

void arena_trim() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto it = g_arenas.begin(); it != g_arenas.end();) {
        Arena *a = it->second;
        bool drop = false;
        if (it->first.first == dev) {
            std::lock_guard<std::mutex> la(a->mu);
            if (a->top == 0 && a->overflow_live == 0 && hipStreamSynchronize(a->s) == hipSuccess) {
                if (a->base) (void)hipFree(a->base);
                drop = true;
            }
        }
        if (drop) {
            delete a;
            it = g_arenas.erase(it);
        } else {
            ++it;
        }
    }
}

int arena_trim_stream(hipStream_t s) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        ckc_set_error(std::string("hipGetDevice: ") + hipGetErrorString(e));
        return CKC_EDEVICE;
    }
    Arena *a = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_arenas.find({dev, s});
        if (it == g_arenas.end()) return CKC_OK;
        a = it->second;
        {
            std::lock_guard<std::mutex> la(a->mu);
            if (a->top != 0 || a->overflow_live != 0) {
                ckc_set_error("ckc_stream_release: a call on the stream still holds scratch");
                return CKC_EINVAL;
            }
        }
        g_arenas.erase(it);
    }
    // the stream's queued work may still use the buffer
    e = hipStreamSynchronize(s);
    if (a->base) (void)hipFree(a->base);
    delete a;
    // overflow buffers went back to the device's default pool: return what
    // it caches to the device so that later hipMalloc calls can use it
    hipMemPool_t pool;
    if (e == hipSuccess && hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) (void)hipMemPoolTrimTo(pool, 0);
    if (e != hipSuccess) {
        ckc_set_error(std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
        return CKC_EDEVICE;
    }
    return CKC_OK;
}

int arena_reserve_stream(hipStream_t s, size_t bytes) {
    int rc = CKC_OK;
    Arena *a = arena_for(s, &rc);
    if (!a) return rc;
    bytes = (bytes + kAlign - 1) / kAlign * kAlign;
    std::lock_guard<std::mutex> lk(a->mu);
    CKC_REQUIRE(a->top == 0 && a->overflow_live == 0, CKC_EINVAL,
                "ckc_stream_reserve: a call on the stream still holds scratch");
    if (bytes > a->cap) {
        CKC_HIP(hipStreamSynchronize(s));
        if (a->base) {
            CKC_HIP(hipFree(a->base));
            a->base = nullptr;
            a->cap = 0;
        }
        hipMemPool_t pool;
        if (hipDeviceGetDefaultMemPool(&pool, a->dev) == hipSuccess) (void)hipMemPoolTrimTo(pool, 0);
        hipError_t e = hipMalloc((void **)&a->base, bytes);
        if (e != hipSuccess) {
            a->base = nullptr;
            ckc_set_error(std::string("ckc_stream_reserve hipMalloc: ") + hipGetErrorString(e));
            (void)hipGetLastError();  // reported here, not by the next launch check
            return CKC_ENOMEM;
        }
        a->cap = bytes;
    }
    a->high = std::max(a->high, bytes);
    return CKC_OK;
}

thread_local FixedScratch *t_fixed_scratch = nullptr;

int fixed_alloc(FixedScratch *f, size_t bytes, void **p, size_t *off) {
    CKC_REQUIRE(f->top + bytes <= f->cap, CKC_ENOMEM,
                "fixed scratch exhausted: " + std::to_string(f->top + bytes) + " bytes needed, " +
                    std::to_string(f->cap) + " available");
    *p = f->base + f->top;
    *off = f->top;
    f->top += bytes;
    f->high = std::max(f->high, f->top);
    return CKC_OK;
}

void fixed_release(FixedScratch *f, size_t off, size_t bytes) {
    // stack-wise: only the topmost buffer lowers the top (work on one stream
    // runs in order, so a later buffer may reuse what queued kernels read)
    if (off + bytes == f->top) f->top = off;
}

extern "C" int ckc_stream_release(void *stream) { return arena_trim_stream((hipStream_t)stream); }
extern "C" int ckc_stream_reserve(void *stream, size_t bytes) {
    return arena_reserve_stream((hipStream_t)stream, bytes);
}
