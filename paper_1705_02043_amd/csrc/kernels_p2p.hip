// Direct kernel sums of the evaluation pass:
//   U    (leaf points  -> the points of an adjacent leaf or of its image),
//   W    (a small leaf's points, or a box's upward equivalent surface -> a leaf's points),
//   X    (leaf points  -> a small leaf's points, or a box's downward check surface),
//   S2M  (leaf points  -> the leaf's upward check surface),
//   L2T  (a leaf's downward equivalent surface -> its own points).
// All are q_t = sum_s K(x_t - y_s) phi_s with the raw kernels 1/|r| and
// I/|r| + r r^T/|r|^3 (the 1/(4 pi), 1/(8 pi) factors are applied once at the
// end of the pass).  A zero separation contributes nothing.
//
// Points-target kernel (k_p2p): one workgroup of 256 threads owns up to 2*256
// targets held in registers and walks its list of source segments; each
// segment is staged through LDS in tiles of 256 sources, loaded coalesced
// from the Morton-sorted SoA arrays (or generated from the surface grid), and
// every thread sweeps the tile; all lanes read the same LDS word (broadcast).
// The geometry of a pair is computed once for a block of RB right-hand sides.
//
// U-list pairs evaluated once (segment kind 3, one right-hand side): the kernel is
// symmetric, K(-d) = K(d), so a pair of adjacent leaves B, A (A in U(B) with shift p,
// B in U(A) with -p) is swept by one workgroup holding B's targets.  Within a tile the
// sources are taken in groups of 64 and rotated across the wave (lane i meets source
// (i + j) mod 64 at step j), so at every step each lane adds its pair's reverse term
// into a different per-wave float64 LDS accumulator with an LDS atomic add
// (ds_add_f64; the float32 LDS atomic is an order of magnitude slower on this chip):
// no two lanes touch one address in a step and the wave's LDS operations execute in
// order, so each source's sum is formed in a fixed order.  After each group the four
// waves are combined in a fixed order and each source's sum is written once to a
// partial slot; a gather kernel adds the slots of every leaf in list order.  Results
// are deterministic and do not depend on scheduling.
//
// Mixed precision (U lists and direct W/X): each point is stored as an integer offset
// from its leaf centre in units of 2^-29 h (h the leaf's edge).  For a pair of leaves the
// offsets are brought to the unit 2^-29 H of the larger leaf (an exact or rounded shift) and
// the centre difference, an exact multiple of that unit, is added to the targets once per
// segment, so every separation is an exact integer difference rounded once to float32; the
// kernel is evaluated in float32 with v_rsq_f32 on these scaled separations and the sums are
// multiplied back by 2^29 / H (both kernels are homogeneous of degree -1).  Partial sums over
// 32 sources are kept in float32 and added into float64 accumulators.
//
// One right-hand side: each 64-source group of a tile is stored twice in a row in LDS, one
// record (coordinates and densities) per source, so that the rotated sweep reads every step
// at a constant offset from one address per lane (no index arithmetic in the inner loop).
#include <climits>
#include <type_traits>

#include "launch.h"

namespace pk {

namespace {

constexpr int kThreads = 256;
constexpr int kTPT = 2;                 // targets per thread
constexpr double kInner = 0.525;        // half of 1.05
constexpr double kOuter = 1.475;        // half of 2.95

__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
// 1/sqrt(x) in float64 without branches: the hardware estimate v_rsq_f64 refined by two
// Newton steps y <- y + y (1 - x y^2) / 2 (each roughly doubles the correct bits).  Valid for
// the normal, positive x that occur here (separations >= ~1e-7); x = 0 is guarded by callers.
__device__ __forceinline__ double rsq(double x) {
    double y = __builtin_amdgcn_rsq(x);
    double e = fma(-x * y, y, 1.0);
    y = fma(0.5 * y, e, y);
    e = fma(-x * y, y, 1.0);
    return fma(0.5 * y, e, y);
}

// 1/|d| from r2 = |d|^2; with GUARD, 0 for a zero separation (a pair that contributes
// nothing).  Float separations are integers (the mixed form's units), so a non-zero r2 is at
// least 1 and rsq(r2) <= 1 <= r2: min(rsq(r2), r2) is rsq(r2) there and 0 at r2 = 0 (where
// rsq gives +inf), one instruction.  A zero separation occurs in a leaf's own segment
// (coincident points share a leaf, and a point never meets its own image exactly in float64),
// so only that segment is guarded, unless set-up found points of different leaves or images
// so close that their integer positions may coincide (P2PArgs::guard_all): then every
// segment of the mixed form is, and such points meet as coincident points.
template <bool GUARD>
__device__ __forceinline__ float rinv(float r2) { return GUARD ? fminf(rsq(r2), r2) : rsq(r2); }
template <bool GUARD>
__device__ __forceinline__ double rinv(double r2) { return GUARD ? (r2 > 0.0 ? rsq(r2) : 0.0) : rsq(r2); }

// K(d) applied to RB densities; with GUARD a zero separation contributes nothing.
template <int KD, int RB, bool GUARD, typename T>
__device__ __forceinline__ void interact(T dx, T dy, T dz, const T* d, T* acc) {
    T r2 = dx * dx + dy * dy + dz * dz;
    T ri = rinv<GUARD>(r2);
    if constexpr (KD == 1) {
#pragma unroll
        for (int q = 0; q < RB; ++q) acc[q] += d[q] * ri;
    } else {
        T ri2 = ri * ri;
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            const T* f = d + 3 * q;
            T fdr = (f[0] * dx + f[1] * dy + f[2] * dz) * ri2;
            acc[3 * q + 0] += ri * (f[0] + dx * fdr);
            acc[3 * q + 1] += ri * (f[1] + dy * fdr);
            acc[3 * q + 2] += ri * (f[2] + dz * fdr);
        }
    }
}

// K(d) applied both ways: fs (the source's density) into acc_t, ft (the target's) into acc_s.
// Only used between different leaves; GUARD as for interact.
template <int KD, bool GUARD, typename T>
__device__ __forceinline__ void interact_both(T dx, T dy, T dz, const T* fs, T* acc_t, const T* ft, T* acc_s) {
    T r2 = dx * dx + dy * dy + dz * dz;
    T ri = rinv<GUARD>(r2);
    if constexpr (KD == 1) {
        acc_t[0] += fs[0] * ri;
        acc_s[0] += ft[0] * ri;
    } else {
        T ri2 = ri * ri;
        T a = (fs[0] * dx + fs[1] * dy + fs[2] * dz) * ri2;
        T b = (ft[0] * dx + ft[1] * dy + ft[2] * dz) * ri2;
        acc_t[0] += ri * (fs[0] + dx * a);
        acc_t[1] += ri * (fs[1] + dy * a);
        acc_t[2] += ri * (fs[2] + dz * a);
        acc_s[0] += ri * (ft[0] + dx * b);
        acc_s[1] += ri * (ft[1] + dy * b);
        acc_s[2] += ri * (ft[2] + dz * b);
    }
}

__device__ __forceinline__ double box_h(const P2PArgs& a, int b) { return ldexp(1.0, -a.box_level[b]); }

// a staged source: coordinates and densities, one LDS record
template <int KD, typename C, typename T>
struct alignas(16) SrcRec {
    C x, y, z;
    T d[KD];
};

// v / 2^k rounded to nearest (ties up), for the integer offsets of a finer leaf
__device__ __forceinline__ int shr_round(int v, int k) { return (v + ((1 << k) >> 1)) >> k; }
// LDS slot of tile source i: with one right-hand side each 64-source group is stored twice
template <int RB>
__device__ __forceinline__ int slot_of(int i) { return RB == 1 ? ((i >> 6) << 7) + (i & 63) : i; }
// one component of a separation: exact integer difference (mixed form, wrapping as the
// hardware does, in unsigned arithmetic), rounded once to float; or a float64 difference
template <bool MIXED>
__device__ __forceinline__ float sep(int t, int s) { return (float)(int)((unsigned)t - (unsigned)s); }
template <bool MIXED>
__device__ __forceinline__ double sep(double t, double s) { return t - s; }

// One-way segments get a loop per number of target slots in use (waves whose second slots are
// all padding skip them) only in the float32 Laplace form with 16 right-hand sides: there the
// extra code leaves the residency unchanged (188 -> 241 VGPRs, two waves per SIMD either way)
// and the batched forest's near field runs 10 % faster, bit for bit the same.  Elsewhere it
// either costs a wave per SIMD (the 4-RHS Stokes form: 168 -> 210 VGPRs, three waves to two,
// 19 % slower) or, with one right-hand side (one-way segments are the leaves' own, a few per
// cent of the pairs), measured slower.
template <int KD, bool MIXED, int RB>
constexpr bool kOneWaySlots = KD == 1 && MIXED && RB == 16;
// The float32 Stokes form with 4 right-hand sides (168 VGPRs, three waves per SIMD) and the
// float64 Stokes form with one (the leaf pass of W and L2T work; 124 VGPRs) keep their loops as
// they are and add only a one-target copy for waves without second targets, which their
// registers allow (the float64 4-RHS form would go from 156 to 190 VGPRs, three waves to two).
template <int KD, bool MIXED, int RB>
constexpr bool kOneWayOne = KD == 3 && ((MIXED && RB == 4) || (!MIXED && RB == 1));

template <int KD, bool MIXED, int RB>
__global__ __launch_bounds__(kThreads) void k_p2p(P2PArgs a, int r0) {
    using T = typename std::conditional<MIXED, float, double>::type;   // kernel arithmetic
    using C = typename std::conditional<MIXED, int, double>::type;     // staged coordinates
    constexpr int ND = KD * RB;
    // one-RHS passes store each 64-source group of a tile twice in a row, so that the rotated
    // sweep of the pair-once segments reads LDS at a constant offset from one address per wave
    // (one record per source, so that each step is one or two vector reads); several
    // right-hand sides read separate arrays, each at one address for the whole workgroup
    constexpr bool kRec = RB == 1;
    __shared__ SrcRec<KD, C, T> s_src[kRec ? 2 * kThreads : 1];
    __shared__ C s_x[kRec ? 1 : kThreads], s_y[kRec ? 1 : kThreads], s_z[kRec ? 1 : kThreads];
    __shared__ T s_d[ND][kRec ? 1 : kThreads];
    auto put = [&](int q, C x, C y, C z, const T* d) {
        if constexpr (kRec) {
            SrcRec<KD, C, T> r;
            r.x = x; r.y = y; r.z = z;
            for (int c = 0; c < KD; ++c) r.d[c] = d[c];
            s_src[q] = r;
        } else {
            s_x[q] = x; s_y[q] = y; s_z[q] = z;
            for (int c = 0; c < ND; ++c) s_d[c][q] = d[c];
        }
    };
    auto get = [&](int q, C& x, C& y, C& z, T* d) {
        if constexpr (kRec) {
            const SrcRec<KD, C, T> r = s_src[q];
            x = r.x; y = r.y; z = r.z;
            for (int c = 0; c < KD; ++c) d[c] = r.d[c];
        } else {
            x = s_x[q]; y = s_y[q]; z = s_z[q];
            for (int c = 0; c < ND; ++c) d[c] = s_d[c][q];
        }
    };
    // kind-3 segments: per-wave running sums of the reverse terms of a 64-source group, in two
    // halves (a source met before and after the rotation wraps)
    constexpr int NW = RB == 1 ? kThreads / 64 : 1;
    __shared__ double s_dacc[NW][KD][128];

    const double* __restrict__ usurf = a.usurf;
    const int kn = KD * a.n_surf;
    const int64_t n = a.n;
    const int tid = threadIdx.x;
    if constexpr (RB == 1) {
        for (int i = tid; i < NW * KD * 128; i += kThreads) (&s_dacc[0][0][0])[i] = 0.0;
    }
    // the grid may be smaller than the item list (a capped residency leaves room on every
    // compute unit for the concurrent tree passes): then workgroups take the next item from a
    // counter, in list order; every workgroup leaves once the list is exhausted
    __shared__ int s_item;
    for (int wi = blockIdx.x;;) {
    if (a.work_counter) {
        __syncthreads();
        if (tid == 0) s_item = (int)atomicAdd(a.work_counter, 1ull);
        __syncthreads();
        wi = s_item;
    }
    if (wi >= a.n_work) break;
    const Work w = a.work[wi];
    // Target slots: thread tid holds slots s and s + 256, s = 64 ((wave + item) mod 4) + lane.
    // In the pair-once sweep a wave whose second slots all lie past the item's targets skips
    // them (two == false); rotating the slot blocks with the item index spreads those lighter
    // waves over the SIMDs.  A target keeps its lane, and so the order in which it meets its
    // sources.  The rotation is a per-wave scalar added to tid wherever a slot is formed: one
    // more vector register live across the item would cost the 4-RHS Stokes variant (168
    // VGPRs, three waves per SIMD) a third of its residency.
    const int wv0 = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int tshift = (((wv0 + wi) & 3) - wv0) << 6;
    const bool two = ((wv0 + wi) & 3) * 64 + kThreads < w.tcount;   // uniform per wave
    // target box centre and edge
    const int tlev = a.box_level[w.tbox];
    const double th = ldexp(1.0, -tlev);
    const double tcx = (a.box_ix[w.tbox] + 0.5) * th;
    const double tcy = (a.box_iy[w.tbox] + 0.5) * th;
    const double tcz = (a.box_iz[w.tbox] + 0.5) * th;

    double acc[kTPT][ND];
    T dt[kTPT][KD];                        // the targets' own densities (kind-3 reverse terms); 0 for padding
    for (int j = 0; j < kTPT; ++j) {
        for (int c = 0; c < ND; ++c) acc[j][c] = 0.0;
        const int t = w.t0 + min(tid + tshift + j * kThreads, max(w.tcount - 1, 0));
        const bool real = tid + tshift + j * kThreads < w.tcount;
        for (int c = 0; c < KD; ++c) {
            const int64_t di = ((int64_t)r0 * KD + c) * n + t;
            dt[j][c] = real ? (MIXED ? (T)a.ds32[di] : (T)a.ds[di]) : T(0);
        }
    }

    for (int sg = w.seg0; sg < w.seg1; ++sg) {
        const Seg seg = a.segs[sg];
        const int b = seg.box;
        const int slev = a.box_level[b];
        const double sh = ldexp(1.0, -slev);
        const double shx = (double)(seg.shift / 9 - 1), shy = (double)((seg.shift / 3) % 3 - 1),
                     shz = (double)(seg.shift % 3 - 1);
        const double scx = (a.box_ix[b] + 0.5) * sh + shx;
        const double scy = (a.box_iy[b] + 0.5) * sh + shy;
        const double scz = (a.box_iz[b] + 0.5) * sh + shz;
        const bool pts = seg.kind == 0 || seg.kind == 3;
        int count, base = 0;
        if (pts) {
            base = a.box_begin[b];
            count = a.box_send[b] - base;
        } else {
            count = a.n_surf;
        }
        const bool self_seg = seg.kind == 0 && b == w.tbox && seg.shift == 13;
        // Mixed form: separations in integers, in units u = 2^-29 H with H the larger of the
        // two leaves' edges (|separation| <= 2H component-wise for U, W and X pairs, so every
        // difference fits); each leaf's offsets are rounded to that unit, the centre difference
        // is an exact multiple of it, and the float kernel's results are scaled by 1/u (both
        // kernels are homogeneous of degree -1).  Float64 form: absolute coordinates.
        const int lc = min(tlev, slev);
        const int kt = tlev - lc, ks = slev - lc;
        const double inv_u = MIXED ? ldexp(1.0, lc + 29) : 1.0;
        C ux[kTPT], uy[kTPT], uz[kTPT];
        for (int j = 0; j < kTPT; ++j) {
            const int t = w.t0 + min(tid + tshift + j * kThreads, max(w.tcount - 1, 0));
            if constexpr (MIXED) {
                const int e = lc + 29;
                ux[j] = shr_round(a.ioff[t], kt) + (int)ldexp(tcx - scx, e);
                uy[j] = shr_round(a.ioff[n + t], kt) + (int)ldexp(tcy - scy, e);
                uz[j] = shr_round(a.ioff[2 * n + t], kt) + (int)ldexp(tcz - scz, e);
            } else {
                ux[j] = a.xs[t] - shx; uy[j] = a.xs[n + t] - shy; uz[j] = a.xs[2 * n + t] - shz;
            }
        }
        const double* phi = seg.kind == 1 ? a.phi_u : a.phi_d;
        const int64_t pcol = seg.kind == 4 ? seg.slot : (int64_t)b;   // density column block
        const double sf = (seg.kind == 1 ? kInner : kOuter) * sh;
        for (int c0 = 0; c0 < count; c0 += kThreads) {
            const int cnt = min(kThreads, count - c0);
            __syncthreads();
            const int sl = slot_of<RB>(tid);
            if (tid < cnt) {
                const int s = c0 + tid;
                C cx, cy, cz;
                T dv[ND];
                if (pts) {
                    const int64_t q = base + s;
                    if constexpr (MIXED) {
                        cx = shr_round(a.ioff[q], ks); cy = shr_round(a.ioff[n + q], ks);
                        cz = shr_round(a.ioff[2 * n + q], ks);
                        for (int c = 0; c < ND; ++c) dv[c] = a.ds32[((int64_t)r0 * KD + c) * n + q];
                    } else {
                        cx = a.xs[q]; cy = a.xs[n + q]; cz = a.xs[2 * n + q];
                        for (int c = 0; c < ND; ++c) dv[c] = a.ds[((int64_t)r0 * KD + c) * n + q];
                    }
                } else {   // surface sources exist only in the float64 passes
                    if constexpr (!MIXED) {
                        cx = sf * usurf[3 * s] + scx - shx;
                        cy = sf * usurf[3 * s + 1] + scy - shy;
                        cz = sf * usurf[3 * s + 2] + scz - shz;
                        for (int q = 0; q < RB; ++q) {
                            const double* src = phi + ((int64_t)pcol * a.R + r0 + q) * kn + KD * s;
                            for (int c = 0; c < KD; ++c) dv[KD * q + c] = src[c];
                        }
                    }
                }
                put(sl, cx, cy, cz, dv);
                if constexpr (kRec) put(sl + 64, cx, cy, cz, dv);
            } else if (seg.kind == 3 && tid < ((cnt + 63) & ~63)) {
                // padding of the last 64-source group: far from every target (integers: the
                // farthest value, never equal to a target's), zero density; its own reverse
                // sums are computed and discarded
                const C far = MIXED ? (C)INT_MIN : (C)1.0e6;
                T zero[ND];
                for (int c = 0; c < ND; ++c) zero[c] = T(0);
                put(sl, far, far, far, zero);
                if constexpr (kRec) put(sl + 64, far, far, far, zero);
            }
            __syncthreads();
            if constexpr (RB == 1) {
                if (seg.kind == 3) {
                    const int lane = tid & 63, wv = tid >> 6;
                    auto sweep = [&](auto guard, auto slots) {
                        constexpr bool G = decltype(guard)::value;
                        constexpr int NT = decltype(slots)::value;   // target slots in use
                        for (int g0 = 0; g0 < cnt; g0 += 64) {
                            const int gs = 2 * g0;              // slot of the group's first copy
                            for (int h = 0; h < 64; h += 32) {
                                T part[NT][KD];
                                for (int j = 0; j < NT; ++j)
                                    for (int c = 0; c < KD; ++c) part[j][c] = T(0);
                                const int q0 = gs + lane + h;   // this lane's source at step 0 of the half
                                double* dacc = &s_dacc[wv][0][lane + h];
#pragma unroll
                                for (int jj = 0; jj < 32; ++jj) {
                                    const int q = q0 + jj;
                                    T d[KD], cs[KD];
                                    C sx, sy, sz;
                                    get(q, sx, sy, sz, d);
                                    for (int c = 0; c < KD; ++c) cs[c] = T(0);
                                    for (int j = 0; j < NT; ++j)
                                        interact_both<KD, G, T>(sep<MIXED>(ux[j], sx), sep<MIXED>(uy[j], sy),
                                                                sep<MIXED>(uz[j], sz), d, part[j], dt[j], cs);
                                    for (int c = 0; c < KD; ++c)
                                        __hip_atomic_fetch_add(dacc + c * 128 + jj, (double)cs[c], __ATOMIC_RELAXED,
                                                               __HIP_MEMORY_SCOPE_WAVEFRONT);
                                }
                                for (int j = 0; j < NT; ++j)
                                    for (int c = 0; c < KD; ++c) acc[j][c] += (double)part[j][c] * inv_u;
                            }
                            __syncthreads();
                            if (tid < min(64, cnt - g0))
                                for (int c = 0; c < KD; ++c) {
                                    double v = 0.0;
                                    for (int u = 0; u < NW; ++u) v += s_dacc[u][c][tid] + s_dacc[u][c][tid + 64];
                                    a.mpart[(int64_t)c * a.n_slots + seg.slot + c0 + g0 + tid] = v * inv_u;
                                }
                            __syncthreads();
                            // each lane clears its own two slots; every add of the next group follows
                            // in program order
                            for (int c = 0; c < KD; ++c) { s_dacc[wv][c][lane] = 0.0; s_dacc[wv][c][lane + 64] = 0.0; }
                            __asm__ volatile("" ::: "memory");
                        }
                    };
                    auto go = [&](auto guard) {
                        if (two) sweep(guard, std::integral_constant<int, 2>{});
                        else sweep(guard, std::integral_constant<int, 1>{});
                    };
                    if constexpr (MIXED) {
                        if (a.guard_all) go(std::true_type{});
                        else go(std::false_type{});
                    } else {
                        go(std::false_type{});
                    }
                    continue;
                }
            }
            if constexpr (kOneWaySlots<KD, MIXED, RB>) {
                // the guard and the number of target slots in use fixed per segment, one loop each
                auto oneway = [&](auto guard, auto slots) {
                    constexpr bool G = decltype(guard)::value;
                    constexpr int NT = decltype(slots)::value;
                    if constexpr (MIXED) {
                        for (int j0 = 0; j0 < cnt; j0 += 32) {
                            const int j1 = min(cnt, j0 + 32);
                            T part[NT][ND];
                            for (int j = 0; j < NT; ++j)
                                for (int c = 0; c < ND; ++c) part[j][c] = T(0);
                            for (int q = j0; q < j1; ++q) {
                                T d[ND];
                                C sx, sy, sz;
                                get(slot_of<RB>(q), sx, sy, sz, d);
                                for (int j = 0; j < NT; ++j)
                                    interact<KD, RB, G, T>(sep<MIXED>(ux[j], sx), sep<MIXED>(uy[j], sy),
                                                           sep<MIXED>(uz[j], sz), d, part[j]);
                            }
                            for (int j = 0; j < NT; ++j)
                                for (int c = 0; c < ND; ++c) acc[j][c] += (double)part[j][c] * inv_u;
                        }
                    } else {
                        for (int q = 0; q < cnt; ++q) {
                            T d[ND];
                            C sx, sy, sz;
                            get(slot_of<RB>(q), sx, sy, sz, d);
                            for (int j = 0; j < NT; ++j)
                                interact<KD, RB, G, T>(ux[j] - sx, uy[j] - sy, uz[j] - sz, d, acc[j]);
                        }
                    }
                };
                auto by_slots = [&](auto guard) {
                    if (two) oneway(guard, std::integral_constant<int, 2>{});
                    else oneway(guard, std::integral_constant<int, 1>{});
                };
                if (self_seg || (MIXED && a.guard_all)) by_slots(std::true_type{});
                else by_slots(std::false_type{});
                continue;
            }
            if constexpr (kOneWayOne<KD, MIXED, RB> && !MIXED) {
                if (!two) {      // no second target slot in use: the one-target copy of the loop below
                    for (int q = 0; q < cnt; ++q) {
                        T d[ND];
                        C sx, sy, sz;
                        get(slot_of<RB>(q), sx, sy, sz, d);
                        if (self_seg)
                            interact<KD, RB, true, T>(ux[0] - sx, uy[0] - sy, uz[0] - sz, d, acc[0]);
                        else
                            interact<KD, RB, false, T>(ux[0] - sx, uy[0] - sy, uz[0] - sz, d, acc[0]);
                    }
                    continue;
                }
            }
            if constexpr (kOneWayOne<KD, MIXED, RB> && MIXED) {
                if (!two) {      // no second target slot in use: the one-target copy of the loop below
                    for (int j0 = 0; j0 < cnt; j0 += 32) {
                        const int j1 = min(cnt, j0 + 32);
                        T part[ND];
                        for (int c = 0; c < ND; ++c) part[c] = T(0);
                        for (int q = j0; q < j1; ++q) {
                            T d[ND];
                            C sx, sy, sz;
                            get(slot_of<RB>(q), sx, sy, sz, d);
                            if (self_seg || a.guard_all)
                                interact<KD, RB, true, T>(sep<MIXED>(ux[0], sx), sep<MIXED>(uy[0], sy),
                                                          sep<MIXED>(uz[0], sz), d, part);
                            else
                                interact<KD, RB, false, T>(sep<MIXED>(ux[0], sx), sep<MIXED>(uy[0], sy),
                                                           sep<MIXED>(uz[0], sz), d, part);
                        }
                        for (int c = 0; c < ND; ++c) acc[0][c] += (double)part[c] * inv_u;
                    }
                    continue;
                }
            }
            if constexpr (MIXED) {
                for (int j0 = 0; j0 < cnt; j0 += 32) {
                    const int j1 = min(cnt, j0 + 32);
                    T part[kTPT][ND];
                    for (int j = 0; j < kTPT; ++j)
                        for (int c = 0; c < ND; ++c) part[j][c] = T(0);
                    for (int q = j0; q < j1; ++q) {
                        T d[ND];
                        C sx, sy, sz;
                        get(slot_of<RB>(q), sx, sy, sz, d);
                        if (self_seg || a.guard_all) {
                            for (int j = 0; j < kTPT; ++j)
                                interact<KD, RB, true, T>(sep<MIXED>(ux[j], sx), sep<MIXED>(uy[j], sy),
                                                          sep<MIXED>(uz[j], sz), d, part[j]);
                        } else {
                            for (int j = 0; j < kTPT; ++j)
                                interact<KD, RB, false, T>(sep<MIXED>(ux[j], sx), sep<MIXED>(uy[j], sy),
                                                           sep<MIXED>(uz[j], sz), d, part[j]);
                        }
                    }
                    for (int j = 0; j < kTPT; ++j)
                        for (int c = 0; c < ND; ++c) acc[j][c] += (double)part[j][c] * inv_u;
                }
            } else {
                for (int q = 0; q < cnt; ++q) {
                    T d[ND];
                    C sx, sy, sz;
                    get(slot_of<RB>(q), sx, sy, sz, d);
                    for (int j = 0; j < kTPT; ++j) {
                        if (self_seg)
                            interact<KD, RB, true, T>(ux[j] - sx, uy[j] - sy, uz[j] - sz, d, acc[j]);
                        else
                            interact<KD, RB, false, T>(ux[j] - sx, uy[j] - sy, uz[j] - sz, d, acc[j]);
                    }
                }
            }
        }
    }
    for (int j = 0; j < kTPT; ++j) {
        const int lt = tid + tshift + j * kThreads;
        if (lt >= w.tcount) continue;
        const int t = w.t0 + lt;
        for (int c = 0; c < ND; ++c) {
            double* o = a.out_pts + ((int64_t)r0 * KD + c) * n + t;
            *o = a.accumulate_pts ? *o + acc[j][c] : acc[j][c];
        }
    }
    if (!a.work_counter) wi += gridDim.x;
    }   // work items
}

// Points to a surface (S2M: a leaf's own points to its upward check surface; X list:
// leaf points to a box's downward check surface), float64.  A workgroup owns up
// to 64 surface targets; its 256 threads form 4 groups that sweep interleaved
// quarters of every source tile, and the four partial sums are added in a
// fixed order at the end.  RB right-hand sides share each pair's geometry.
template <int KD, int RB>
__global__ __launch_bounds__(kThreads) void k_p2s(P2PArgs a, int r0) {
    constexpr int ND = KD * RB;
    __shared__ double s_x[kThreads], s_y[kThreads], s_z[kThreads], s_d[ND][kThreads];
    __shared__ double s_red[4][64][ND];
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
    double acc[ND];
    for (int c = 0; c < ND; ++c) acc[c] = 0.0;
    for (int sg = w.seg0; sg < w.seg1; ++sg) {
        const Seg seg = a.segs[sg];
        const int b = seg.box;
        const double shx = (double)(seg.shift / 9 - 1), shy = (double)((seg.shift / 3) % 3 - 1),
                     shz = (double)(seg.shift % 3 - 1);
        const double ux = tx - shx, uy = ty - shy, uz = tz - shz;
        const int base = a.box_begin[b], count = a.box_send[b] - base;
        for (int c0 = 0; c0 < count; c0 += kThreads) {
            const int cnt = min(kThreads, count - c0);
            __syncthreads();
            if (tid < cnt) {
                const int64_t q = base + c0 + tid;
                s_x[tid] = a.xs[q]; s_y[tid] = a.xs[n + q]; s_z[tid] = a.xs[2 * n + q];
                for (int c = 0; c < ND; ++c) s_d[c][tid] = a.ds[((int64_t)r0 * KD + c) * n + q];
            }
            __syncthreads();
            for (int q = grp; q < cnt; q += 4) {
                double d[ND];
                for (int c = 0; c < ND; ++c) d[c] = s_d[c][q];
                interact<KD, RB, true, double>(ux - s_x[q], uy - s_y[q], uz - s_z[q], d, acc);
            }
        }
    }
    for (int c = 0; c < ND; ++c) s_red[grp][lt][c] = acc[c];
    __syncthreads();
    if (grp == 0 && lt < w.tcount)
        for (int rr = 0; rr < RB; ++rr) {
            double* q = a.out_surf + ((int64_t)w.tbox * a.R + r0 + rr) * kn + KD * (w.t0 + lt);
            for (int c = 0; c < KD; ++c) {
                const int e = KD * rr + c;
                q[c] += ((s_red[0][lt][e] + s_red[1][lt][e]) + s_red[2][lt][e]) + s_red[3][lt][e];
            }
        }
}

__global__ __launch_bounds__(kThreads) void k_mutual_gather(const double* __restrict__ mpart, int64_t n_slots, int kd,
                                                           const int* __restrict__ in_box,
                                                           const int64_t* __restrict__ in_off,
                                                           const int64_t* __restrict__ in_slot,
                                                           const int* __restrict__ box_begin,
                                                           const int* __restrict__ box_end, int64_t n,
                                                           double* __restrict__ out) {
    const int j = blockIdx.x, c = blockIdx.y;
    const int b = in_box[j];
    const int base = box_begin[b], cnt = box_end[b] - base;
    const int64_t e0 = in_off[j], e1 = in_off[j + 1];
    const double* __restrict__ pc = mpart + (int64_t)c * n_slots;
    for (int i = threadIdx.x; i < cnt; i += kThreads) {
        double s = 0.0;
        for (int64_t e = e0; e < e1; e += 8) {      // eight loads in flight, added in list order
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = e + u < e1 ? pc[in_slot[e + u] + i] : 0.0;
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (e + u < e1) s += v[u];
        }
        out[(int64_t)c * n + base + i] += s;
    }
}

template <int KD, bool MIXED, int RB>
void launch_block(const P2PArgs& a, int r0, hipStream_t s) {
    // every launch of a right-hand-side block takes the item list from the start: the counter
    // is cleared before each one, by a kernel (no memset node under graph capture)
    if (a.work_counter) launch_fill_zero(reinterpret_cast<double*>(a.work_counter), 1, s);
    const int grid = a.work_counter ? std::min(a.n_work, a.grid_cap) : a.n_work;
    hipLaunchKernelGGL((k_p2p<KD, MIXED, RB>), dim3(grid), dim3(kThreads), 0, s, a, r0);
    PK_HIP(hipGetLastError());
}

template <int KD, bool MIXED>
void launch_rhs(const P2PArgs& a, hipStream_t s) {
    // right-hand sides in blocks: up to 16 (Laplace) or 4 (Stokes), capped by a.rb_max, share one
    // geometry pass (each right-hand side's sums are formed in the same order whatever the block)
    const int cap = a.rb_max > 0 ? a.rb_max : 16;
    int r0 = 0;
    while (r0 < a.R) {
        const int left = std::min(a.R - r0, cap);
        if (KD == 1 && left >= 16) { launch_block<KD, MIXED, 16>(a, r0, s); r0 += 16; }
        else if (KD == 1 && left >= 8) { launch_block<KD, MIXED, 8>(a, r0, s); r0 += 8; }
        else if (left >= 4) { launch_block<KD, MIXED, 4>(a, r0, s); r0 += 4; }
        else if (left >= 2) { launch_block<KD, MIXED, 2>(a, r0, s); r0 += 2; }
        else { launch_block<KD, MIXED, 1>(a, r0, s); r0 += 1; }
    }
}

}  // namespace

template <int KD, int RB>
void launch_p2s_block(const P2PArgs& a, int r0, hipStream_t s) {
    hipLaunchKernelGGL((k_p2s<KD, RB>), dim3(a.n_work), dim3(kThreads), 0, s, a, r0);
    PK_HIP(hipGetLastError());
}

void launch_p2s(const P2PArgs& a, hipStream_t s) {
    if (a.n_work == 0) return;
    // right-hand sides in blocks: up to 8 (Laplace) or 4 (Stokes), capped by a.rb_max, share one
    // geometry pass
    const int cap = a.rb_max > 0 ? a.rb_max : 8;
    for (int r0 = 0; r0 < a.R;) {
        const int left = std::min(a.R - r0, cap);
        if (a.kernel == PKIFMM_LAPLACE) {
            if (left >= 8) { launch_p2s_block<1, 8>(a, r0, s); r0 += 8; }
            else if (left >= 4) { launch_p2s_block<1, 4>(a, r0, s); r0 += 4; }
            else if (left >= 2) { launch_p2s_block<1, 2>(a, r0, s); r0 += 2; }
            else { launch_p2s_block<1, 1>(a, r0, s); r0 += 1; }
        } else {
            if (left >= 4) { launch_p2s_block<3, 4>(a, r0, s); r0 += 4; }
            else if (left >= 2) { launch_p2s_block<3, 2>(a, r0, s); r0 += 2; }
            else { launch_p2s_block<3, 1>(a, r0, s); r0 += 1; }
        }
    }
}

void launch_mutual_gather(const double* mpart, int64_t n_slots, int kd, const int* in_box, const int64_t* in_off,
                          const int64_t* in_slot, int n_in, const int* box_begin, const int* box_end, int64_t n,
                          double* out, hipStream_t s) {
    if (n_in == 0) return;
    hipLaunchKernelGGL(k_mutual_gather, dim3(n_in, kd), dim3(kThreads), 0, s, mpart, n_slots, kd, in_box, in_off,
                       in_slot, box_begin, box_end, n, out);
    PK_HIP(hipGetLastError());
}

void launch_p2p(const P2PArgs& a, bool mixed, hipStream_t s) {
    if (a.n_work == 0) return;
    if (a.kernel == PKIFMM_LAPLACE) {
        if (mixed) launch_rhs<1, true>(a, s);
        else launch_rhs<1, false>(a, s);
    } else {
        if (mixed) launch_rhs<3, true>(a, s);
        else launch_rhs<3, false>(a, s);
    }
}

}  // namespace pk
