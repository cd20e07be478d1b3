// Point-wise kernels: wrap/validate/quantise/Morton keys, radix sort,
// gathers and density permutations.  All are HBM-bound streaming kernels with
// one point per thread and coalesced SoA accesses.
#include <algorithm>

#include <rocprim/device/device_radix_sort.hpp>

#include "launch.h"

namespace pk {

namespace {

__device__ __forceinline__ uint64_t spread3(uint32_t v) {
    uint64_t x = v & 0x1fffff;
    x = (x | (x << 32)) & 0x1f00000000ffffull;
    x = (x | (x << 16)) & 0x1f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

// Periodic axes: w = v - floor(v), a result of exactly 1.0 (from a tiny
// negative v) becomes 0.0.  Other axes: the closed [0, 1] is accepted.
// Quantisation: min(floor(w * 2^21), 2^21 - 1), exact in double.
__global__ void k_keys(const double* __restrict__ xyz, int64_t n, double L, unsigned mask,
                       uint64_t* __restrict__ keys, uint32_t* __restrict__ vals, double* __restrict__ u,
                       int* __restrict__ err) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t q[3];
    bool bad = false;
    for (int c = 0; c < 3; ++c) {
        double v = xyz[3 * i + c] / L;
        double w;
        if (mask & (1u << c)) {
            if (!isfinite(v)) bad = true;
            w = v - floor(v);
            if (w >= 1.0) w = 0.0;
        } else {
            if (!(v >= 0.0 && v <= 1.0)) bad = true;
            w = v;
        }
        if (bad) w = 0.0;
        u[c * n + i] = w;
        double f = floor(w * 2097152.0);
        q[c] = (uint32_t)fmin(f, 2097151.0);
    }
    if (bad) atomicOr(err, 1);
    keys[i] = (spread3(q[0]) << 2) | (spread3(q[1]) << 1) | spread3(q[2]);
    vals[i] = (uint32_t)i;
}

__global__ void k_gather_points(const double* __restrict__ u, const uint32_t* __restrict__ perm, int64_t n,
                                double* __restrict__ xs) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t j = perm[i];
    xs[i] = u[j];
    xs[n + i] = u[n + j];
    xs[2 * n + i] = u[2 * n + j];
}

// offsets from the leaf centre as integers in units of 2^-29 h (h the leaf's edge): the
// centre (i + 1/2) 2^-l is dyadic, so x - c is exact in double and the rounding to that grid
// (at most 2^-30 h) is the only approximation; |offset| <= 2^28.
// One workgroup per leaf (leaves[blockIdx.x]), threads over its points.
__global__ void k_leaf_offsets(const double* __restrict__ xs, int64_t n, const int* __restrict__ leaves,
                               const int* __restrict__ box_begin, const int* __restrict__ box_end,
                               const int* __restrict__ lv, const int* __restrict__ bx, const int* __restrict__ by,
                               const int* __restrict__ bz, int* __restrict__ ioff) {
    const int b = leaves[blockIdx.x];
    const double h = ldexp(1.0, -lv[b]);
    const double cx = (bx[b] + 0.5) * h, cy = (by[b] + 0.5) * h, cz = (bz[b] + 0.5) * h;
    const int e = lv[b] + 29;
    for (int64_t i = box_begin[b] + threadIdx.x; i < box_end[b]; i += blockDim.x) {
        ioff[i] = (int)rint(ldexp(xs[i] - cx, e));
        ioff[n + i] = (int)rint(ldexp(xs[n + i] - cy, e));
        ioff[2 * n + i] = (int)rint(ldexp(xs[2 * n + i] - cz, e));
    }
}

// points j >= n_dens (separate targets) carry zero density
__global__ void k_permute_density(const double* __restrict__ dens, const uint32_t* __restrict__ perm, int64_t n,
                                  int64_t n_dens, int R, int k, double* __restrict__ ds, float* __restrict__ ds32) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t j = perm[i];
    for (int r = 0; r < R; ++r)
        for (int c = 0; c < k; ++c) {
            double v = (int64_t)j < n_dens ? dens[((int64_t)r * n_dens + j) * k + c] : 0.0;
            ds[((int64_t)r * k + c) * n + i] = v;
            if (ds32) ds32[((int64_t)r * k + c) * n + i] = (float)v;
        }
}

// only points j >= t_first are targets; target j is output row j - t_first of n_out
__global__ void k_unpermute(const double* __restrict__ pot, const uint32_t* __restrict__ perm, int64_t n,
                            int64_t t_first, int64_t n_out, int R, int k, double scale, double* __restrict__ out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t j = (int64_t)perm[i] - t_first;
    if (j < 0) return;
    for (int r = 0; r < R; ++r)
        for (int c = 0; c < k; ++c)
            out[((int64_t)r * n_out + j) * k + c] = scale * pot[((int64_t)r * k + c) * n + i];
}

// Separate targets: per leaf (one workgroup each), the key (leaf begin, is target) of each of its
// sorted points, so that a stable sort by it puts each leaf's sources before its targets and
// keeps both in (Morton key, index) order; and the leaf's source count.
__global__ void k_role_keys(const int* __restrict__ leaves, const int* __restrict__ box_begin,
                            const int* __restrict__ box_end, const uint32_t* __restrict__ perm, int64_t n_src,
                            uint64_t* __restrict__ keys, int* __restrict__ n_sources) {
    __shared__ int sh[256];
    const int b = leaves[blockIdx.x];
    const int b0 = box_begin[b], b1 = box_end[b];
    int cnt = 0;
    for (int i = b0 + threadIdx.x; i < b1; i += 256) {
        const bool trg = (int64_t)perm[i] >= n_src;
        keys[i] = ((uint64_t)b0 << 1) | (trg ? 1u : 0u);
        cnt += trg ? 0 : 1;
    }
    sh[threadIdx.x] = cnt;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) n_sources[blockIdx.x] = sh[0];
}

// one workgroup per (problem, rhs x component): the sum and the sum of magnitudes;
// deterministic tree reduction in LDS
__global__ void k_density_sums(const double* __restrict__ ds, int64_t n, const int64_t* __restrict__ off,
                               double* __restrict__ out) {
    __shared__ double sh[2][256];
    const double* src = ds + (int64_t)blockIdx.y * n;
    double acc = 0.0, mag = 0.0;
    for (int64_t i = off[blockIdx.x] + threadIdx.x; i < off[blockIdx.x + 1]; i += 256) {
        acc += src[i];
        mag += fabs(src[i]);
    }
    sh[0][threadIdx.x] = acc;
    sh[1][threadIdx.x] = mag;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + w];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int64_t o = 2 * ((int64_t)blockIdx.x * gridDim.y + blockIdx.y);
        out[o] = sh[0][0];
        out[o + 1] = sh[1][0];
    }
}

// Pairs of points whose separation the mixed form's integer coordinates could round to zero
// although they are different points or different images: points in different cells of the
// finest (2^-21) grid, or one point and another's periodic image, closer than `delta` in every
// coordinate.  Points in one cell share a leaf and meet there without an image, where the
// kernels guard zero separations anyway.  One thread per sorted point: a point within delta of
// a face of its cell looks through the neighbouring cells across those faces (their key
// ranges found by binary search inside the point's problem; periodic axes wrap with an image
// shift, other axes stop at the box) for a point closer than delta.  Sets *flag on a find,
// and also, conservatively, when a neighbouring cell holds more than kScan points.
constexpr int kScan = 64;
__global__ void k_close_pairs(const uint64_t* __restrict__ keys, const double* __restrict__ xs, int64_t n,
                              const int64_t* __restrict__ off, int n_prob, unsigned mask, double delta,
                              int* __restrict__ flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double cell = 1.0 / 2097152.0;
    double x[3];
    int c[3], lo[3], hi[3];
    bool any = false;
    for (int a = 0; a < 3; ++a) {
        x[a] = xs[a * n + i];
        c[a] = (int)fmin(floor(x[a] * 2097152.0), 2097151.0);
        lo[a] = x[a] - c[a] * cell < delta ? -1 : 0;
        hi[a] = (c[a] + 1) * cell - x[a] < delta ? 1 : 0;
        any = any || lo[a] || hi[a];
    }
    if (!any) return;
    int q0 = 0, q1 = n_prob;   // the problem of point i: last q with off[q] <= i
    while (q1 - q0 > 1) {
        const int m = (q0 + q1) >> 1;
        if (off[m] <= i) q0 = m;
        else q1 = m;
    }
    const int64_t pb = off[q0], pe = off[q0 + 1];
    for (int ox = lo[0]; ox <= hi[0]; ++ox)
        for (int oy = lo[1]; oy <= hi[1]; ++oy)
            for (int oz = lo[2]; oz <= hi[2]; ++oz) {
                if (ox == 0 && oy == 0 && oz == 0) continue;
                const int o[3] = {ox, oy, oz};
                uint32_t nc[3];
                double shift[3];
                bool ok = true;
                for (int a = 0; a < 3; ++a) {
                    int v = c[a] + o[a];
                    shift[a] = 0.0;
                    if (v < 0 || v >= 2097152) {
                        if (!(mask & (1u << a))) ok = false;
                        shift[a] = v < 0 ? -1.0 : 1.0;
                        v = v < 0 ? v + 2097152 : v - 2097152;
                    }
                    nc[a] = (uint32_t)v;
                }
                if (!ok) continue;
                const uint64_t key = (spread3(nc[0]) << 2) | (spread3(nc[1]) << 1) | spread3(nc[2]);
                int64_t l = pb, h = pe;
                while (l < h) {   // first key >= key
                    const int64_t m = l + ((h - l) >> 1);
                    if (keys[m] < key) l = m + 1;
                    else h = m;
                }
                for (int64_t j = l, cnt = 0; j < pe && keys[j] == key; ++j, ++cnt) {
                    if (cnt >= kScan) {
                        atomicOr(flag, 1);
                        return;
                    }
                    double dmax = 0.0;
                    for (int a = 0; a < 3; ++a) dmax = fmax(dmax, fabs(x[a] - (xs[a * n + j] + shift[a])));
                    if (dmax < delta) {
                        atomicOr(flag, 1);
                        return;
                    }
                }
            }
}

// Triply periodic Laplace: the far-field term the root's equivalent density cannot carry.  The
// zero-mean Ewald kernel (raw 1/r normalisation) has laplacian 4 pi away from its lattice
// points, so as a function of the source position it is harmonic plus (2 pi / 3) |y - c|^2; the
// equivalent density matches the sources on harmonic functions only, so the far field lacks
// (2 pi / 3) (sum_s q_s |y_s - c|^2 - sum_j phi_j |y_j - c|^2), one constant per problem and
// right-hand side, added to every potential.  One workgroup per (problem, right-hand side);
// deterministic LDS reductions.  Root of problem q: box q; its equivalent points c + 0.525 u_j.
__global__ void k_tp_background(const double* __restrict__ ds, const double* __restrict__ xs, int64_t n,
                                const int64_t* __restrict__ off, const double* __restrict__ phi_u, int R,
                                const double* __restrict__ usurf, int n_surf, double* __restrict__ pot) {
    __shared__ double sh[256];
    const int q = blockIdx.x, r = blockIdx.y;
    const int64_t b0 = off[q], b1 = off[q + 1];
    double acc = 0.0;
    for (int64_t i = b0 + threadIdx.x; i < b1; i += 256) {
        const double dx = xs[i] - 0.5, dy = xs[n + i] - 0.5, dz = xs[2 * n + i] - 0.5;
        acc += ds[(int64_t)r * n + i] * (dx * dx + dy * dy + dz * dz);
    }
    const double* phi = phi_u + ((int64_t)q * R + r) * n_surf;
    for (int j = threadIdx.x; j < n_surf; j += 256) {
        const double ux = usurf[3 * j], uy = usurf[3 * j + 1], uz = usurf[3 * j + 2];
        acc -= phi[j] * (0.525 * 0.525) * (ux * ux + uy * uy + uz * uz);
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    const double c = (2.0 * M_PI / 3.0) * sh[0];
    for (int64_t i = b0 + threadIdx.x; i < b1; i += 256) pot[(int64_t)r * n + i] += c;
}

__global__ void k_fill_zero(double* __restrict__ x, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        x[i] = 0.0;
}

// Children of split boxes: for split box i (level child_level - 1, sorted-key range
// [begin, end), integer coordinates ix, iy, iz) and octant o, the key range of the child cell,
// found by two binary searches over the box's keys.  box: [n_split][5] = begin, end, ix, iy, iz;
// out: [n_split][8][2] = first, end (empty when equal).
__global__ void k_tree_children(const uint64_t* __restrict__ keys, const int* __restrict__ box, int n_split,
                                int child_level, int* __restrict__ out) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= 8 * n_split) return;
    const int i = g >> 3, o = g & 7;
    const int* bx = box + 5 * i;
    const uint32_t cx = 2 * bx[2] + ((o >> 2) & 1), cy = 2 * bx[3] + ((o >> 1) & 1), cz = 2 * bx[4] + (o & 1);
    const int sh = 3 * (21 - child_level);
    const uint64_t prefix = (spread3(cx) << 2) | (spread3(cy) << 1) | spread3(cz);
    const uint64_t klo = prefix << sh, khi = ((prefix + 1) << sh) - 1;
    int lo = bx[0], hi = bx[1];
    while (lo < hi) {          // first key >= klo
        const int mid = lo + ((hi - lo) >> 1);
        if (keys[mid] < klo) lo = mid + 1;
        else hi = mid;
    }
    const int a = lo;
    hi = bx[1];
    while (lo < hi) {          // first key > khi
        const int mid = lo + ((hi - lo) >> 1);
        if (keys[mid] <= khi) lo = mid + 1;
        else hi = mid;
    }
    out[2 * g] = a;
    out[2 * g + 1] = lo;
}

// Segment of every key-sorted point (segment q holds the input positions [off[q], off[q+1]))
// and the point's position in the key order.
__global__ void k_segment_of(const uint32_t* __restrict__ idx, int64_t n, const int64_t* __restrict__ off, int n_seg,
                             uint32_t* __restrict__ seg, uint32_t* __restrict__ pos) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int64_t v = idx[j];
    int lo = 0, hi = n_seg;   // off[lo] <= v < off[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= v) lo = mid;
        else hi = mid;
    }
    seg[j] = (uint32_t)lo;
    pos[j] = (uint32_t)j;
}

__global__ void k_gather_pairs(const uint32_t* __restrict__ pos, int64_t n, const uint64_t* __restrict__ kin,
                               const uint32_t* __restrict__ vin, uint64_t* __restrict__ kout,
                               uint32_t* __restrict__ vout) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const uint32_t p = pos[j];
    kout[j] = kin[p];
    vout[j] = vin[p];
}

__global__ void k_add_into(double* __restrict__ y, const double* __restrict__ x, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] += x[i];
}

inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

void launch_fill_zero(double* x, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)std::min<int64_t>(nblk(n, 256), 4096)), dim3(256), 0, s, x, n);
    PK_HIP(hipGetLastError());
}

void launch_tree_children(const uint64_t* keys, const int* box, int n_split, int child_level, int* out,
                          hipStream_t s) {
    if (n_split == 0) return;
    hipLaunchKernelGGL(k_tree_children, dim3(nblk(8 * (int64_t)n_split, 256)), dim3(256), 0, s, keys, box, n_split,
                       child_level, out);
    PK_HIP(hipGetLastError());
}

void launch_add_into(double* y, const double* x, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_add_into, dim3((unsigned)std::min<int64_t>(nblk(n, 256), 4096)), dim3(256), 0, s, y, x, n);
    PK_HIP(hipGetLastError());
}

void launch_keys(const double* xyz, int64_t n, double L, unsigned mask, uint64_t* keys, uint32_t* vals, double* u,
                 int* err, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_keys, dim3(nblk(n, 256)), dim3(256), 0, s, xyz, n, L, mask, keys, vals, u, err);
    PK_HIP(hipGetLastError());
}

void radix_sort_pairs(uint64_t* kin, uint64_t* kout, uint32_t* vin, uint32_t* vout, int64_t n, DBuf<char>& temp,
                      hipStream_t s, int n_seg, const int64_t* off, int end_bit) {
    if (n == 0) return;
    size_t bytes = 0;
    if (n_seg > 1) {
        // one full-chip sort of every key, then a stable sort by segment: the input holds each
        // segment contiguously, so this is each segment sorted on its own with ties in input
        // order (a segmented sort runs one workgroup per segment, a few for the whole chip)
        const int seg_bits = 32 - __builtin_clz((unsigned)(n_seg - 1));
        uint32_t* nil = nullptr;
        size_t b1 = 0, b2 = 0;
        PK_HIP(rocprim::radix_sort_pairs(nullptr, b1, kin, kout, vin, vout, (size_t)n, 0, 63, s));
        PK_HIP(rocprim::radix_sort_pairs(nullptr, b2, nil, nil, nil, nil, (size_t)n, 0, seg_bits, s));
        auto al = [](size_t b) { return (b + 255) / 256 * 256; };
        const size_t rb = al(std::max(b1, b2)), n4 = al(sizeof(uint32_t) * n), n8 = al(sizeof(uint64_t) * n);
        temp.ensure(rb + 5 * n4 + n8);
        char* base = temp.p;
        uint32_t* seg = reinterpret_cast<uint32_t*>(base + rb);
        uint32_t* seg2 = reinterpret_cast<uint32_t*>(base + rb + n4);
        uint32_t* pos = reinterpret_cast<uint32_t*>(base + rb + 2 * n4);
        uint32_t* pos2 = reinterpret_cast<uint32_t*>(base + rb + 3 * n4);
        uint32_t* vtmp = reinterpret_cast<uint32_t*>(base + rb + 4 * n4);
        uint64_t* ktmp = reinterpret_cast<uint64_t*>(base + rb + 5 * n4);
        PK_HIP(rocprim::radix_sort_pairs(base, b1, kin, ktmp, vin, vtmp, (size_t)n, 0, 63, s));
        hipLaunchKernelGGL(k_segment_of, dim3(nblk(n, 256)), dim3(256), 0, s, vtmp, n, off, n_seg, seg, pos);
        PK_HIP(hipGetLastError());
        PK_HIP(rocprim::radix_sort_pairs(base, b2, seg, seg2, pos, pos2, (size_t)n, 0, seg_bits, s));
        hipLaunchKernelGGL(k_gather_pairs, dim3(nblk(n, 256)), dim3(256), 0, s, pos2, n, ktmp, vtmp, kout, vout);
        PK_HIP(hipGetLastError());
        return;
    }
    PK_HIP(rocprim::radix_sort_pairs(nullptr, bytes, kin, kout, vin, vout, (size_t)n, 0, end_bit, s));
    temp.ensure(bytes);
    PK_HIP(rocprim::radix_sort_pairs(temp.p, bytes, kin, kout, vin, vout, (size_t)n, 0, end_bit, s));
}

void launch_gather_points(const double* u, const uint32_t* perm, int64_t n, double* xs, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_gather_points, dim3(nblk(n, 256)), dim3(256), 0, s, u, perm, n, xs);
    PK_HIP(hipGetLastError());
}

void launch_leaf_offsets(const double* xs, int64_t n, const int* leaves, int n_leaves, const int* box_begin,
                         const int* box_end, const int* lv, const int* bx, const int* by, const int* bz, int* ioff,
                         hipStream_t s) {
    if (n == 0 || n_leaves == 0) return;
    hipLaunchKernelGGL(k_leaf_offsets, dim3(n_leaves), dim3(256), 0, s, xs, n, leaves, box_begin, box_end, lv, bx, by,
                       bz, ioff);
    PK_HIP(hipGetLastError());
}

void launch_permute_density(const double* dens, const uint32_t* perm, int64_t n, int64_t n_dens, int R, int k,
                            double* ds, float* ds32, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_permute_density, dim3(nblk(n, 256)), dim3(256), 0, s, dens, perm, n, n_dens, R, k, ds, ds32);
    PK_HIP(hipGetLastError());
}

void launch_unpermute(const double* pot, const uint32_t* perm, int64_t n, int64_t t_first, int64_t n_out, int R,
                      int k, double scale, double* out, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_unpermute, dim3(nblk(n, 256)), dim3(256), 0, s, pot, perm, n, t_first, n_out, R, k, scale,
                       out);
    PK_HIP(hipGetLastError());
}

void launch_role_keys(const int* leaves, int n_leaves, const int* box_begin, const int* box_end, const uint32_t* perm,
                      int64_t n_src, uint64_t* keys, int* n_sources, hipStream_t s) {
    if (n_leaves == 0) return;
    hipLaunchKernelGGL(k_role_keys, dim3(n_leaves), dim3(256), 0, s, leaves, box_begin, box_end, perm, n_src, keys,
                       n_sources);
    PK_HIP(hipGetLastError());
}

void launch_close_pairs(const uint64_t* keys, const double* xs, int64_t n, const int64_t* off, int n_prob,
                        unsigned mask, double delta, int* flag, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_close_pairs, dim3(nblk(n, 256)), dim3(256), 0, s, keys, xs, n, off, n_prob, mask, delta,
                       flag);
    PK_HIP(hipGetLastError());
}

void launch_tp_background(const double* ds, const double* xs, int64_t n, const int64_t* off, int n_prob,
                          const double* phi_u, int R, const double* usurf, int n_surf, double* pot, hipStream_t s) {
    if (n == 0 || n_prob == 0) return;
    hipLaunchKernelGGL(k_tp_background, dim3(n_prob, R), dim3(256), 0, s, ds, xs, n, off, phi_u, R, usurf, n_surf,
                       pot);
    PK_HIP(hipGetLastError());
}

void launch_density_sums(const double* ds, int64_t n, int R, int k, const int64_t* off, int n_prob, double* out,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_density_sums, dim3(n_prob, R * k), dim3(256), 0, s, ds, n, off, out);
    PK_HIP(hipGetLastError());
}

}  // namespace pk
