// Dense operator products of the evaluation pass: upward/downward
// check-to-equivalent solves (U^T then V S^+), M2M, L2L, M2L and the root
// far-field operator.  All are "grouped gather GEMMs": a tile multiplies one
// operator (column-major M x K) with up to 64 gathered input columns and
// writes (or accumulates into) scattered output columns, each with its own
// scale (the 2^l factors of the homogeneous kernels).
//
// Float64 path: 64x64 output tiles, K staged through LDS in steps of 16,
// 4x4 register micro-tiles per thread.
#include "launch.h"

namespace pk {

namespace {

constexpr int TM = 64, TN = 64, TK = 16;

__global__ __launch_bounds__(256) void k_gemm_f64(GemmArgs a) {
    const Tile t = a.tiles[blockIdx.x];
    const double* __restrict__ A = a.ops + (int64_t)t.op * a.op_stride;
    __shared__ double sA[TK][TM + 1];
    __shared__ double sB[TK][TN + 1];
    __shared__ int s_in[TN];
    const int tid = threadIdx.x;
    const int tx = tid & 15, ty = tid >> 4;
    if (tid < TN) s_in[tid] = tid < t.ncol ? a.in_col[t.col0 + tid] : -1;
    double acc[4][4];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
    __syncthreads();
    for (int k0 = 0; k0 < a.K; k0 += TK) {
        for (int e = 0; e < 4; ++e) {
            int idx = tid + 256 * e;
            int m = idx & (TM - 1), kk = idx >> 6;
            int row = t.row0 + m, k = k0 + kk;
            sA[kk][m] = (row < a.M && k < a.K) ? A[row + (int64_t)k * a.M] : 0.0;
            int kk2 = idx & (TK - 1), nn = idx >> 4;
            int col = s_in[nn];
            int k2 = k0 + kk2;
            sB[kk2][nn] = (col >= 0 && k2 < a.K) ? a.B[(int64_t)col * a.ldb + k2] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < TK; ++kk) {
            double av[4], bv[4];
            for (int i = 0; i < 4; ++i) av[i] = sA[kk][ty + 16 * i];
            for (int j = 0; j < 4; ++j) bv[j] = sB[kk][tx + 16 * j];
            for (int i = 0; i < 4; ++i)
                for (int j = 0; j < 4; ++j) acc[i][j] = fma(av[i], bv[j], acc[i][j]);
        }
        __syncthreads();
    }
    for (int j = 0; j < 4; ++j) {
        int n = tx + 16 * j;
        if (n >= t.ncol) continue;
        int oc = a.out_col[t.col0 + n];
        double sc = a.scale[t.col0 + n];
        double* C = a.C + (int64_t)oc * a.ldc;
        for (int i = 0; i < 4; ++i) {
            int row = t.row0 + ty + 16 * i;
            if (row >= a.M) continue;
            double v = sc * acc[i][j];
            C[row] = a.accumulate ? C[row] + v : v;
        }
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

void launch_gemm(const GemmArgs& a, hipStream_t s) {
    if (a.n_tiles == 0) return;
    hipLaunchKernelGGL(k_gemm_f64, dim3(a.n_tiles), dim3(256), 0, s, a);
    PK_HIP(hipGetLastError());
}

void launch_segment_reduce(const double* temp, const int64_t* off, const int* boxes, int nboxes, int R, int kn,
                           double* q, hipStream_t s) {
    if (nboxes == 0) return;
    hipLaunchKernelGGL(k_segment_reduce, dim3(nboxes, R), dim3(256), 0, s, temp, off, boxes, R, kn, q);
    PK_HIP(hipGetLastError());
}

}  // namespace pk
