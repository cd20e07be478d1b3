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

constexpr int kMaxLevel = 21;
constexpr int kNumM2L = 316;   // offsets in [-3,3]^3 with |delta|_inf >= 2
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

// ---------------------------------------------------------------- tree (host topology)

struct HostTree {
    std::vector<int> level, ix, iy, iz, begin, end, parent;
    std::vector<int> child;       // [nbox][8], -1 absent
    std::vector<int> leaf_id;     // box -> leaf index or -1
    std::vector<int> leaves;      // leaf index -> box
    std::vector<int> level_start; // boxes of level l are [level_start[l], level_start[l+1])
    int depth = 0;
    int nbox() const { return (int)level.size(); }
    bool is_leaf(int b) const {
        for (int o = 0; o < 8; ++o)
            if (child[8 * b + o] >= 0) return false;
        return true;
    }
};

struct Entry {
    int src;      // source box
    int8_t sx, sy, sz;   // image shift, each in {-1, 0, 1}
    bool operator<(const Entry& o) const {
        if (src != o.src) return src < o.src;
        if (sx != o.sx) return sx < o.sx;
        if (sy != o.sy) return sy < o.sy;
        return sz < o.sz;
    }
    bool operator==(const Entry& o) const { return src == o.src && sx == o.sx && sy == o.sy && sz == o.sz; }
};

struct HostLists {
    // CSR over boxes
    std::vector<int64_t> u_off, v_off, w_off, x_off;
    std::vector<Entry> u, v, w, x;
};

void build_tree_host(const uint64_t* sorted_keys, int64_t n, int s, HostTree& t);
void build_lists_host(const HostTree& t, unsigned periodic_mask, HostLists& l);
void add_root_ring(const HostTree& t, unsigned periodic_mask, int near_layers, HostLists& l);
void merge_forest(const std::vector<HostTree>& trees, const std::vector<HostLists>& lists,
                  const std::vector<int64_t>& poff, HostTree& t, HostLists& l, std::vector<int>& box_prob);
int m2l_offset_index(int dx, int dy, int dz);   // -> 0..315
void m2l_offset_vector(int idx, int& dx, int& dy, int& dz);

}  // namespace pk
