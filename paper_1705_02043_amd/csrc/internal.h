// Internal declarations of the periodic KIFMM library (host side).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <cstdint>
#include <stdexcept>
#include <string>
#include <utility>
#include <vector>

#include "pkifmm.h"
#include "topology.h"

namespace pk {

struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define PK_HIP(call)                                                                      \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            throw ::pk::Error(PKIFMM_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

constexpr int kM2LGroups = 8;  // fixed groups of offsets per M2L launch (bounded temporary)

// A caller's device allocator (pkifmm_config::alloc/free), with the stream of the call in progress.
struct Allocator {
    void* ctx = nullptr;
    void* (*alloc)(void*, size_t, void*) = nullptr;
    void (*free)(void*, void*, void*) = nullptr;
    void* stream = nullptr;
};
// The allocator of the plan whose entry point (or build thread) is running on this thread; NULL:
// hipMalloc / hipFree.
extern thread_local const Allocator* g_alloc;
struct AllocScope {
    const Allocator* prev;
    explicit AllocScope(const Allocator* a) : prev(g_alloc) { g_alloc = (a && a->alloc) ? a : nullptr; }
    ~AllocScope() { g_alloc = prev; }
    AllocScope(const AllocScope&) = delete;
    AllocScope& operator=(const AllocScope&) = delete;
};

// Device buffer owned by a plan: from the caller's allocator when one is in scope, else hipMalloc;
// released through whichever made it.
template <class T>
struct DBuf {
    T* p = nullptr;
    size_t n = 0;
    const Allocator* owner = nullptr;
    DBuf() = default;
    DBuf(const DBuf&) = delete;
    DBuf& operator=(const DBuf&) = delete;
    ~DBuf() { release(); }
    void release() {
        if (p) {
            if (owner) owner->free(owner->ctx, p, owner->stream);
            else (void)hipFree(p);
        }
        p = nullptr;
        n = 0;
        owner = nullptr;
    }
    void ensure(size_t count) {
        if (count <= n && p) return;
        release();
        size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
        if (g_alloc) {
            p = static_cast<T*>(g_alloc->alloc(g_alloc->ctx, bytes, g_alloc->stream));
            if (!p) throw Error(PKIFMM_ERR_OOM, "the caller's allocator returned NULL for " + std::to_string(bytes) + " bytes");
            owner = g_alloc;
        } else if (hipMalloc(&p, bytes) != hipSuccess) {
            p = nullptr;
            throw Error(PKIFMM_ERR_OOM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
        }
        n = std::max<size_t>(count, 1);
    }
    void swap(DBuf& o) {
        std::swap(p, o.p);
        std::swap(n, o.n);
        std::swap(owner, o.owner);
    }
    void upload(const std::vector<T>& h, hipStream_t s) {
        ensure(h.size());
        if (!h.empty()) PK_HIP(hipMemcpyAsync(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
    }
};

// Page-locked host buffer owned by a plan (device-to-host copies without a staging copy).
template <class T>
struct PinnedBuf {
    T* p = nullptr;
    size_t n = 0;
    PinnedBuf() = default;
    PinnedBuf(const PinnedBuf&) = delete;
    PinnedBuf& operator=(const PinnedBuf&) = delete;
    ~PinnedBuf() { release(); }
    void release() {
        if (p) (void)hipHostFree(p);
        p = nullptr;
        n = 0;
    }
    void ensure(size_t count) {
        if (count <= n && p) return;
        release();
        size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
        if (hipHostMalloc((void**)&p, bytes, hipHostMallocDefault) != hipSuccess) {
            p = nullptr;
            throw Error(PKIFMM_ERR_OOM, "hipHostMalloc of " + std::to_string(bytes) + " bytes failed");
        }
        n = std::max<size_t>(count, 1);
    }
};

}  // namespace pk
