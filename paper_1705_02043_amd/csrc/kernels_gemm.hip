// Dense operator products of the evaluation pass: upward/downward
// check-to-equivalent solves (U^T then V S^+), M2M, L2L, M2L and the root
// far-field operator.  All are "grouped gather GEMMs": a tile multiplies one
// operator (column-major M x K) with up to 64 gathered input columns and
// writes (or accumulates into) scattered output columns, each with its own
// scale (the 2^l factors of the homogeneous kernels).  The K dimension may be
// split into blocks that gather from different input columns: M2M multiplies
// [M2M_0 | ... | M2M_7] with the stacked densities of a parent's eight
// children in one pass (absent children read as zero).
//
// Float64 on the matrix cores: v_mfma_f64_16x16x4f64.  A 64x64 output tile
// per workgroup (four waves, 32x32 each = 2x2 MFMA blocks), K staged through
// LDS 32 at a time with the next slice prefetched into registers while the
// current one is multiplied.  Tiles are laid out operator-major and mapped so
// that the tiles of one operator run on the same XCD (its L2 keeps the
// operator rows).  Launches with few tiles (the upper tree levels) split K
// over several workgroups; the partial tiles are summed in a fixed order by a
// second kernel, so results do not depend on scheduling.
#include "launch.h"

namespace pk {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int TM = 64, TN = 64, TK = 32, PAD = 2;
constexpr int kPerThread = TM * TK / 256;    // elements of A (and of B) per thread per K slice

// column j of a tile: its input column (K block kb), output column and scale
__device__ __forceinline__ int gemm_in(const GemmArgs& a, int j, int kb) {
    if (a.rhs > 0) {
        const int e = j / a.rhs;
        return a.in_col[e] * a.rhs + (j - e * a.rhs);
    }
    return a.in_col[(int64_t)j * 8 + kb];
}
__device__ __forceinline__ int gemm_out(const GemmArgs& a, int j) {
    if (a.rhs > 0) {
        const int e = j / a.rhs;
        return a.out_col[e] * a.rhs + (j - e * a.rhs);
    }
    return a.out_col[j];
}
__device__ __forceinline__ double gemm_scale(const GemmArgs& a, int j) {
    return a.scale[a.rhs > 0 ? j / a.rhs : j];
}

struct Stage {     // one thread's share of a K slice: kPerThread elements of A and of B
    double a[kPerThread], b[kPerThread];
};

__device__ __forceinline__ void load_stage(const GemmArgs& a, const Tile& t, const double* __restrict__ A,
                                           const int* s_in, int nkb, int k0, int k_end, int tid, Stage& st) {
#pragma unroll
    for (int e = 0; e < kPerThread; ++e) {
        const int idx = tid + 256 * e;
        const int m = idx & (TM - 1), kk = idx / TM;
        const int row = t.row0 + m, k = k0 + kk;
        st.a[e] = (row < a.M && k < k_end) ? A[row + (int64_t)k * a.M] : 0.0;
        const int kk2 = idx & (TK - 1), nn = idx / TK;
        const int k2 = k0 + kk2;
        double v = 0.0;
        if (k2 < k_end) {
            const int kb = nkb == 1 ? 0 : k2 / a.kblock;
            const int col = s_in[nn * nkb + kb];
            if (col >= 0) v = a.B[(int64_t)col * a.ldb + (k2 - kb * a.kblock)];
        }
        st.b[e] = v;
    }
}

__global__ __launch_bounds__(256) void k_gemm_mfma_f64(GemmArgs a, int split, double* __restrict__ partial) {
    // XCD-aware order: workgroup i runs on XCD i % 8; give each XCD a contiguous range
    const int n_items = a.n_tiles * split;
    const int per = (n_items + 7) / 8;
    const int logical = (blockIdx.x % 8) * per + blockIdx.x / 8;
    if (logical >= n_items) return;
    const int tile_id = logical / split, part = logical % split;
    const Tile t = a.tiles[tile_id];
    const double* __restrict__ A = a.ops + (int64_t)t.op * a.op_stride;
    const int kchunk = ((a.K + split - 1) / split + TK - 1) / TK * TK;
    const int k_begin = part * kchunk, k_end = min(a.K, k_begin + kchunk);
    __shared__ double sA[TK][TM + PAD];
    __shared__ double sB[TK][TN + PAD];
    __shared__ int s_in[TN * 8];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
    const int nkb = a.in_stride;
    for (int i = tid; i < TN * nkb; i += 256) {
        int c = i / nkb;
        s_in[i] = c < t.ncol ? gemm_in(a, t.col0 + c, i % nkb) : -1;
    }
    v4d acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
    __syncthreads();
    Stage st;
    if (k_begin < k_end) load_stage(a, t, A, s_in, nkb, k_begin, k_end, tid, st);
    for (int k0 = k_begin; k0 < k_end; k0 += TK) {
#pragma unroll
        for (int e = 0; e < kPerThread; ++e) {
            const int idx = tid + 256 * e;
            sA[idx / TM][idx & (TM - 1)] = st.a[e];
            sB[idx & (TK - 1)][idx / TK] = st.b[e];
        }
        __syncthreads();
        if (k0 + TK < k_end) load_stage(a, t, A, s_in, nkb, k0 + TK, k_end, tid, st);   // next slice in flight
#pragma unroll
        for (int ks = 0; ks < TK; ks += 4) {
            const int kr = ks + (lane >> 4);
            double af[2], bf[2];
            for (int i = 0; i < 2; ++i) af[i] = sA[kr][wm + 16 * i + (lane & 15)];
            for (int j = 0; j < 2; ++j) bf[j] = sB[kr][wn + 16 * j + (lane & 15)];
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
    // D layout of the f64 16x16 block: lane holds column (lane & 15) and rows (lane >> 4) + 4 v
    if (split > 1) {
        double* P = partial + ((int64_t)tile_id * split + part) * (TM * TN);
        for (int j = 0; j < 2; ++j)
            for (int i = 0; i < 2; ++i)
                for (int v = 0; v < 4; ++v) {
                    const int rr = wm + 16 * i + (lane >> 4) + 4 * v, cc = wn + 16 * j + (lane & 15);
                    P[cc * TM + rr] = acc[i][j][v];
                }
        return;
    }
    for (int j = 0; j < 2; ++j) {
        const int n = wn + 16 * j + (lane & 15);
        if (n >= t.ncol) continue;
        const int oc = gemm_out(a, t.col0 + n);
        const double sc = gemm_scale(a, t.col0 + n);
        double* C = a.C + (int64_t)oc * a.ldc;
        for (int i = 0; i < 2; ++i)
            for (int v = 0; v < 4; ++v) {
                const int row = t.row0 + wm + 16 * i + (lane >> 4) + 4 * v;
                if (row >= a.M) continue;
                const double r = sc * acc[i][j][v];
                C[row] = a.accumulate ? C[row] + r : r;
            }
    }
}

// sum of the split-K partial tiles in a fixed order, then scale and store/accumulate
__global__ __launch_bounds__(256) void k_gemm_split_reduce(GemmArgs a, int split, const double* __restrict__ partial) {
    const Tile t = a.tiles[blockIdx.x];
    const double* P = partial + (int64_t)blockIdx.x * split * (TM * TN);
    for (int e = threadIdx.x; e < TM * TN; e += 256) {
        const int cc = e / TM, rr = e % TM;
        const int row = t.row0 + rr;
        if (cc >= t.ncol || row >= a.M) continue;
        double s = 0.0;
        for (int q = 0; q < split; ++q) s += P[(int64_t)q * (TM * TN) + e];
        const int oc = gemm_out(a, t.col0 + cc);
        double* C = a.C + (int64_t)oc * a.ldc;
        const double r = gemm_scale(a, t.col0 + cc) * s;
        C[row] = a.accumulate ? C[row] + r : r;
    }
}

__global__ void k_segment_reduce(const double* __restrict__ temp, const int64_t* __restrict__ off,
                                 const int* __restrict__ boxes, int R, int kn, double* __restrict__ q) {
    const int b = boxes[blockIdx.x];
    const int r = blockIdx.y;
    const int64_t e0 = off[b], e1 = off[b + 1];
    for (int row = threadIdx.x; row < kn; row += blockDim.x) {
        double s = 0.0;
        for (int64_t e = e0; e < e1; ++e) s += temp[(e * R + r) * kn + row];
        q[((int64_t)b * R + r) * kn + row] += s;
    }
}

}  // namespace

int gemm_split_factor(int, int K) {
    // K chunks of about 128: a function of K alone, so that the summation order (and so
    // every result bit) does not depend on how many problems or boxes share the launch
    return std::max(1, std::min(8, K / 128));
}

void launch_gemm(const GemmArgs& a, hipStream_t s, double* partial, int64_t partial_cap) {
    if (a.n_tiles == 0) return;
    if (a.in_stride < 1 || a.in_stride > 8 || a.kblock * a.in_stride < a.K)
        throw Error(PKIFMM_ERR_INVALID_ARG, "gemm: bad K blocking");
    int split = partial ? gemm_split_factor(a.n_tiles, a.K) : 1;
    if ((int64_t)a.n_tiles * split * TM * TN > partial_cap) split = 1;
    const int per = (a.n_tiles * split + 7) / 8;
    hipLaunchKernelGGL(k_gemm_mfma_f64, dim3(8 * per), dim3(256), 0, s, a, split, partial);
    PK_HIP(hipGetLastError());
    if (split > 1) {
        hipLaunchKernelGGL(k_gemm_split_reduce, dim3(a.n_tiles), dim3(256), 0, s, a, split, (const double*)partial);
        PK_HIP(hipGetLastError());
    }
}

void launch_segment_reduce(const double* temp, const int64_t* off, const int* boxes, int nboxes, int R, int kn,
                           double* q, hipStream_t s) {
    if (nboxes == 0) return;
    hipLaunchKernelGGL(k_segment_reduce, dim3(nboxes, R), dim3(256), 0, s, temp, off, boxes, R, kn, q);
    PK_HIP(hipGetLastError());
}

}  // namespace pk
