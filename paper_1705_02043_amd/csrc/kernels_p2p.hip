// Direct kernel sums of the evaluation pass:
//   S2M  (leaf points -> the leaf's upward check surface),
//   X    (leaf points  -> a box's downward check surface),
//   U    (leaf points  -> the points of an adjacent leaf or of its image),
//   W    (upward equivalent surface of a box -> a leaf's points),
//   L2T  (a leaf's downward equivalent surface -> its own points).
// All are q_t = sum_s K(x_t - y_s) phi_s with the raw kernels 1/|r| and
// I/|r| + r r^T/|r|^3 (the 1/(4 pi), 1/(8 pi) factors are applied once at the
// end of the pass).  A zero separation contributes nothing.
//
// One workgroup of 256 threads owns up to 2*256 targets held in registers and
// walks its list of source segments; each segment is staged through LDS in
// tiles of 256 sources, loaded coalesced from the Morton-sorted SoA arrays
// (or generated from the surface grid), and every thread sweeps the tile.
// Sources of one tile are read by all lanes at the same LDS address
// (broadcast, no bank conflicts).
//
// Mixed precision: coordinates are float offsets from the target leaf centre
// (source offsets plus the exact dyadic difference of the box centres), the
// kernel is evaluated in float32 with v_rsq_f32, partial sums over 32 sources
// are kept in float32 and added into float64 accumulators.
#include "launch.h"

namespace pk {

namespace {

constexpr int kThreads = 256;
constexpr int kTPT = 2;                 // targets per thread
constexpr double kInner = 0.525;        // half of 1.05
constexpr double kOuter = 1.475;        // half of 2.95

template <typename T> struct Vec3 { T x, y, z; };

__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsq(double x) { return rsqrt(x); }

template <int KD, typename T>
__device__ __forceinline__ void interact(T tx, T ty, T tz, T sx, T sy, T sz, const T* d, T* acc) {
    T dx = tx - sx, dy = ty - sy, dz = tz - sz;
    T r2 = dx * dx + dy * dy + dz * dz;
    T ri = r2 > T(0) ? rsq(r2) : T(0);
    if constexpr (KD == 1) {
        acc[0] += d[0] * ri;
    } else {
        T fdr = (d[0] * dx + d[1] * dy + d[2] * dz) * (ri * ri);
        acc[0] += ri * (d[0] + dx * fdr);
        acc[1] += ri * (d[1] + dy * fdr);
        acc[2] += ri * (d[2] + dz * fdr);
    }
}

// float32 interaction from a precomputed separation (mixed mode).  Only a leaf's own
// segment can hold a zero separation (coincident points share a leaf; a point never
// meets its own image), so the guard is compiled in only for that segment.
template <int KD, bool GUARD>
__device__ __forceinline__ void interact_d(float dx, float dy, float dz, const float* d, float* acc) {
    float r2 = dx * dx + dy * dy + dz * dz;
    float ri = GUARD ? (r2 > 0.f ? rsq(r2) : 0.f) : rsq(r2);
    if constexpr (KD == 1) {
        acc[0] += d[0] * ri;
    } else {
        float fdr = (d[0] * dx + d[1] * dy + d[2] * dz) * (ri * ri);
        acc[0] += ri * (d[0] + dx * fdr);
        acc[1] += ri * (d[1] + dy * fdr);
        acc[2] += ri * (d[2] + dz * fdr);
    }
}

__device__ __forceinline__ double box_h(const P2PArgs& a, int b) { return ldexp(1.0, -a.box_level[b]); }

template <int KD, bool MIXED>
__global__ __launch_bounds__(kThreads) void k_p2p(P2PArgs a, int r) {
    using T = typename std::conditional<MIXED, float, double>::type;
    __shared__ T s_x[kThreads], s_y[kThreads], s_z[kThreads], s_d[KD][kThreads];
    __shared__ float s_lx[MIXED ? kThreads : 1], s_ly[MIXED ? kThreads : 1], s_lz[MIXED ? kThreads : 1];

    // persistent: workgroup g takes items g, g + grid, ... (items are ordered longest first)
    for (int item = blockIdx.x; item < a.n_work; item += gridDim.x) {
    __syncthreads();
    const Work w = a.work[item];
    const double* __restrict__ c_usurf = a.usurf;
    const int kn = KD * a.n_surf;
    const int64_t n = a.n;
    const int tid = threadIdx.x;

    // target box centre and edge (the origin of the mixed-precision offsets)
    const double th = box_h(a, w.tbox);
    const double tcx = (a.box_ix[w.tbox] + 0.5) * th;
    const double tcy = (a.box_iy[w.tbox] + 0.5) * th;
    const double tcz = (a.box_iz[w.tbox] + 0.5) * th;

    double tx[kTPT], ty[kTPT], tz[kTPT];
    double acc[kTPT][KD];
    for (int j = 0; j < kTPT; ++j) {
        for (int c = 0; c < KD; ++c) acc[j][c] = 0.0;
        int t = w.t0 + min(tid + j * kThreads, max(w.tcount - 1, 0));
        double x, y, z;   // absolute (FP64) or relative to the target centre (mixed)
        if (w.tkind == 0) {
            if (MIXED) {   // hi + lo float pair, exact sum in double
                x = (double)a.off[t] + (double)a.off[3 * n + t];
                y = (double)a.off[n + t] + (double)a.off[4 * n + t];
                z = (double)a.off[2 * n + t] + (double)a.off[5 * n + t];
            } else {
                x = a.xs[t]; y = a.xs[n + t]; z = a.xs[2 * n + t];
            }
        } else {
            double f = (w.tkind == 1 ? kInner : kOuter) * th;
            x = f * c_usurf[3 * t]; y = f * c_usurf[3 * t + 1]; z = f * c_usurf[3 * t + 2];
            if (!MIXED) { x += tcx; y += tcy; z += tcz; }
        }
        tx[j] = x; ty[j] = y; tz[j] = z;
    }

    for (int sg = w.seg0; sg < w.seg1; ++sg) {
        const Seg seg = a.segs[sg];
        const int b = seg.box;
        const double sh = box_h(a, b);
        const double shx = (double)(seg.shift / 9 - 1), shy = (double)((seg.shift / 3) % 3 - 1),
                     shz = (double)(seg.shift % 3 - 1);
        const double scx = (a.box_ix[b] + 0.5) * sh + shx;
        const double scy = (a.box_iy[b] + 0.5) * sh + shy;
        const double scz = (a.box_iz[b] + 0.5) * sh + shz;
        // source-centre minus target-centre: exact dyadic value (mixed mode origin shift)
        const double dcx = scx - tcx, dcy = scy - tcy, dcz = scz - tcz;
        int count, base = 0;
        if (seg.kind == 0) {
            base = a.box_begin[b];
            count = a.box_end[b] - base;
        } else {
            count = a.n_surf;
        }
        // per-segment target coordinates relative to the source frame; in the mixed
        // mode a float hi + lo pair, so that only the final differences are rounded
        T ux[kTPT], uy[kTPT], uz[kTPT];
        float lx[kTPT], ly[kTPT], lz[kTPT];
        for (int j = 0; j < kTPT; ++j) {
            if (MIXED) {
                double vx = tx[j] - dcx, vy = ty[j] - dcy, vz = tz[j] - dcz;
                ux[j] = (float)vx; uy[j] = (float)vy; uz[j] = (float)vz;
                lx[j] = (float)(vx - (double)ux[j]); ly[j] = (float)(vy - (double)uy[j]);
                lz[j] = (float)(vz - (double)uz[j]);
            } else {
                ux[j] = (T)(tx[j] - shx); uy[j] = (T)(ty[j] - shy); uz[j] = (T)(tz[j] - shz);
                lx[j] = ly[j] = lz[j] = 0.f;
            }
        }
        const bool self_seg = seg.kind == 0 && b == w.tbox && seg.shift == 13;
        const double* phi = seg.kind == 1 ? a.phi_u : a.phi_d;
        const double sf = (seg.kind == 1 ? kInner : kOuter) * sh;
        for (int c0 = 0; c0 < count; c0 += kThreads) {
            const int cnt = min(kThreads, count - c0);
            __syncthreads();
            if (tid < cnt) {
                const int s = c0 + tid;
                if (seg.kind == 0) {
                    const int64_t q = base + s;
                    if (MIXED) {
                        s_x[tid] = a.off[q]; s_y[tid] = a.off[n + q]; s_z[tid] = a.off[2 * n + q];
                        s_lx[tid] = a.off[3 * n + q]; s_ly[tid] = a.off[4 * n + q]; s_lz[tid] = a.off[5 * n + q];
                        for (int c = 0; c < KD; ++c) s_d[c][tid] = (T)a.ds32[((int64_t)r * KD + c) * n + q];
                    } else {
                        s_x[tid] = a.xs[q]; s_y[tid] = a.xs[n + q]; s_z[tid] = a.xs[2 * n + q];
                        for (int c = 0; c < KD; ++c) s_d[c][tid] = (T)a.ds[((int64_t)r * KD + c) * n + q];
                    }
                } else {
                    double px = sf * c_usurf[3 * s], py = sf * c_usurf[3 * s + 1], pz = sf * c_usurf[3 * s + 2];
                    if (!MIXED) { px += scx - shx; py += scy - shy; pz += scz - shz; }
                    s_x[tid] = (T)px; s_y[tid] = (T)py; s_z[tid] = (T)pz;
                    const double* src = phi + ((int64_t)b * a.R + r) * kn + KD * s;
                    for (int c = 0; c < KD; ++c) s_d[c][tid] = (T)src[c];
                }
            }
            __syncthreads();
            if constexpr (MIXED) {
                for (int j0 = 0; j0 < cnt; j0 += 32) {
                    const int j1 = min(cnt, j0 + 32);
                    T part[kTPT][KD];
                    for (int j = 0; j < kTPT; ++j)
                        for (int c = 0; c < KD; ++c) part[j][c] = T(0);
                    for (int q = j0; q < j1; ++q) {
                        T d[KD];
                        for (int c = 0; c < KD; ++c) d[c] = s_d[c][q];
                        const float sx = s_x[q], sy = s_y[q], sz = s_z[q];
                        const float slx = s_lx[q], sly = s_ly[q], slz = s_lz[q];
                        if (self_seg) {
                            for (int j = 0; j < kTPT; ++j)
                                interact_d<KD, true>((ux[j] - sx) + (lx[j] - slx), (uy[j] - sy) + (ly[j] - sly),
                                                     (uz[j] - sz) + (lz[j] - slz), d, part[j]);
                        } else {
                            for (int j = 0; j < kTPT; ++j)
                                interact_d<KD, false>((ux[j] - sx) + (lx[j] - slx), (uy[j] - sy) + (ly[j] - sly),
                                                      (uz[j] - sz) + (lz[j] - slz), d, part[j]);
                        }
                    }
                    for (int j = 0; j < kTPT; ++j)
                        for (int c = 0; c < KD; ++c) acc[j][c] += (double)part[j][c];
                }
            } else {
                for (int q = 0; q < cnt; ++q) {
                    T d[KD];
                    for (int c = 0; c < KD; ++c) d[c] = s_d[c][q];
                    for (int j = 0; j < kTPT; ++j) {
                        T part[KD];
                        for (int c = 0; c < KD; ++c) part[c] = acc[j][c];
                        interact<KD, T>(ux[j], uy[j], uz[j], s_x[q], s_y[q], s_z[q], d, part);
                        for (int c = 0; c < KD; ++c) acc[j][c] = part[c];
                    }
                }
            }
        }
    }
    for (int j = 0; j < kTPT; ++j) {
        const int lt = tid + j * kThreads;
        if (lt >= w.tcount) continue;
        const int t = w.t0 + lt;
        if (w.tkind == 0) {
            for (int c = 0; c < KD; ++c) {
                double* o = a.out_pts + ((int64_t)r * KD + c) * n + t;
                *o = a.accumulate_pts ? *o + acc[j][c] : acc[j][c];
            }
        } else {
            double* q = a.out_surf + ((int64_t)w.tbox * a.R + r) * kn + KD * t;
            for (int c = 0; c < KD; ++c) q[c] += acc[j][c];
        }
    }
    }   // work items
}

// Points to a surface (S2M: a leaf's own points to its upward check surface; X list:
// leaf points to a box's downward check surface), float64.  A workgroup owns up
// to 64 surface targets; its 256 threads form 4 groups that sweep interleaved
// quarters of every source tile, and the four partial sums are added in a
// fixed order at the end.
template <int KD>
__global__ __launch_bounds__(kThreads) void k_p2s(P2PArgs a, int r) {
    __shared__ double s_x[kThreads], s_y[kThreads], s_z[kThreads], s_d[KD][kThreads];
    __shared__ double s_red[4][64][KD];
    const Work w = a.work[blockIdx.x];
    const int kn = KD * a.n_surf;
    const int64_t n = a.n;
    const int tid = threadIdx.x;
    const int lt = tid & 63, grp = tid >> 6;
    const double th = box_h(a, w.tbox);
    const double f = (w.tkind == 1 ? kInner : kOuter) * th;
    const int t = w.t0 + min(lt, w.tcount - 1);
    const double tx = (a.box_ix[w.tbox] + 0.5) * th + f * a.usurf[3 * t];
    const double ty = (a.box_iy[w.tbox] + 0.5) * th + f * a.usurf[3 * t + 1];
    const double tz = (a.box_iz[w.tbox] + 0.5) * th + f * a.usurf[3 * t + 2];
    double acc[KD];
    for (int c = 0; c < KD; ++c) acc[c] = 0.0;
    for (int sg = w.seg0; sg < w.seg1; ++sg) {
        const Seg seg = a.segs[sg];
        const int b = seg.box;
        const double shx = (double)(seg.shift / 9 - 1), shy = (double)((seg.shift / 3) % 3 - 1),
                     shz = (double)(seg.shift % 3 - 1);
        const double ux = tx - shx, uy = ty - shy, uz = tz - shz;
        const int base = a.box_begin[b], count = a.box_end[b] - base;
        for (int c0 = 0; c0 < count; c0 += kThreads) {
            const int cnt = min(kThreads, count - c0);
            __syncthreads();
            if (tid < cnt) {
                const int64_t q = base + c0 + tid;
                s_x[tid] = a.xs[q]; s_y[tid] = a.xs[n + q]; s_z[tid] = a.xs[2 * n + q];
                for (int c = 0; c < KD; ++c) s_d[c][tid] = a.ds[((int64_t)r * KD + c) * n + q];
            }
            __syncthreads();
            for (int q = grp; q < cnt; q += 4) {
                double d[KD];
                for (int c = 0; c < KD; ++c) d[c] = s_d[c][q];
                interact<KD, double>(ux, uy, uz, s_x[q], s_y[q], s_z[q], d, acc);
            }
        }
    }
    for (int c = 0; c < KD; ++c) s_red[grp][lt][c] = acc[c];
    __syncthreads();
    if (grp == 0 && lt < w.tcount) {
        double* q = a.out_surf + ((int64_t)w.tbox * a.R + r) * kn + KD * (w.t0 + lt);
        for (int c = 0; c < KD; ++c) q[c] += ((s_red[0][lt][c] + s_red[1][lt][c]) + s_red[2][lt][c]) + s_red[3][lt][c];
    }
}

}  // namespace

void launch_p2s(const P2PArgs& a, hipStream_t s) {
    if (a.n_work == 0) return;
    for (int r = 0; r < a.R; ++r) {
        if (a.kernel == PKIFMM_LAPLACE) hipLaunchKernelGGL((k_p2s<1>), dim3(a.n_work), dim3(kThreads), 0, s, a, r);
        else hipLaunchKernelGGL((k_p2s<3>), dim3(a.n_work), dim3(kThreads), 0, s, a, r);
        PK_HIP(hipGetLastError());
    }
}

void launch_p2p(const P2PArgs& a, bool mixed, hipStream_t s, int max_groups) {
    if (a.n_work == 0) return;
    const int grid = max_groups > 0 ? std::min(a.n_work, max_groups) : a.n_work;
    for (int r = 0; r < a.R; ++r) {
        if (a.kernel == PKIFMM_LAPLACE) {
            if (mixed) hipLaunchKernelGGL((k_p2p<1, true>), dim3(grid), dim3(kThreads), 0, s, a, r);
            else hipLaunchKernelGGL((k_p2p<1, false>), dim3(grid), dim3(kThreads), 0, s, a, r);
        } else {
            if (mixed) hipLaunchKernelGGL((k_p2p<3, true>), dim3(grid), dim3(kThreads), 0, s, a, r);
            else hipLaunchKernelGGL((k_p2p<3, false>), dim3(grid), dim3(kThreads), 0, s, a, r);
        }
        PK_HIP(hipGetLastError());
    }
}

}  // namespace pk
