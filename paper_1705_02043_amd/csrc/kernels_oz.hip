// M2L of the mixed-precision form on the int8 matrix cores, with exact accumulation.
//
// Each row i of an operator A (kn x kn) is written as 2^e_i sum_{t=1..S} d_t[i,:] 2^-7t with
// integer digits (|d_1| <= 127, |d_t| <= 64 after the first), each column c of the upward
// densities B the same way with 2^f_c; then
//     (A B)[i,c] ~= 2^(e_i + f_c) sum_{t+u <= S+1} 2^-7(t+u) (D_t G_u)[i,c],
// where every D_t G_u is an int8 x int8 product accumulated exactly in int32
// (v_mfma_i32_16x16x64_i8).  Products with the same t+u share a scale and one int32
// accumulator; the S diagonals are converted to float64 and added smallest first.  The only
// approximation is the truncation of the digit expansions (about 2^-7S of a row's largest
// entry times a column's largest entry per term), so the rounding of a float32 or bf16 GEMM
// never enters: it is the exact-integer splitting of Ozaki et al. applied to the V-list M2L
// translations (Section 2.2; one operator per offset, shared by every level and periodic
// shift).  The float64 form keeps its float64 GEMM.
//
// Layouts (int8): operator slices [op][S][Mp][Kp], row-major, K contiguous; column slices
// [S][col][Kp].  Mp and Kp are kn rounded up to 64 and the padding is zero, so the GEMM has no
// bounds checks in its K loop.  Output tiles, gathered input columns, output columns and
// scales are those of the float64 grouped GEMM (Tile lists of 64 x 64, per-entry column lists
// with the right-hand side expanded on the device).
#include "launch.h"

namespace pk {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int kTile = 64;     // output rows and columns per workgroup; K per stage

// digits of x / 2^e in base 2^7, rounded to nearest at every level (exact in float64)
template <int S>
__device__ __forceinline__ void digits(double x, int e, int8_t* d) {
    double r = ldexp(x, -e);
#pragma unroll
    for (int t = 0; t < S; ++t) {
        const double v = r * 128.0;
        const double q = rint(v);
        d[t] = (int8_t)(int)q;
        r = v - q;
    }
}

// exponent e with max |x| < 2^e * 127/128 (0 for an all-zero vector)
__device__ __forceinline__ int scale_exponent(double m) {
    if (!(m > 0.0)) return 0;
    int e;
    (void)frexp(m * (128.0 / 127.0), &e);
    return e;
}

// per operator row: exponent from the row's largest entry (column-major operators)
__global__ void k_oz_row_exp(const double* __restrict__ ops, int n_ops, int M, int K, int Mp, int* __restrict__ e) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)n_ops * Mp) return;
    const int op = (int)(i / Mp), row = (int)(i % Mp);
    double m = 0.0;
    if (row < M) {
        const double* A = ops + (int64_t)op * M * K + row;
        for (int k = 0; k < K; ++k) m = fmax(m, fabs(A[(int64_t)k * M]));
    }
    e[i] = scale_exponent(m);
}

// per (operator, row, 16 consecutive k): S slices of 16 digits each, one 16-byte store per slice
template <int S>
__global__ void k_oz_row_slices(const double* __restrict__ ops, int n_ops, int M, int K, int Mp, int Kp,
                                const int* __restrict__ e, int8_t* __restrict__ out) {
    const int kq = Kp / 16;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)n_ops * Mp * kq) return;
    const int row = (int)(i % Mp);
    const int64_t rest = i / Mp;
    const int k0 = (int)(rest % kq) * 16, op = (int)(rest / kq);
    const int ex = e[(int64_t)op * Mp + row];
    unsigned w[S][4];
    for (int t = 0; t < S; ++t)
        for (int q = 0; q < 4; ++q) w[t][q] = 0u;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int k = k0 + j;
        int8_t dj[S];
        if (row < M && k < K) digits<S>(ops[(int64_t)op * M * K + (int64_t)k * M + row], ex, dj);
        else for (int t = 0; t < S; ++t) dj[t] = 0;
        for (int t = 0; t < S; ++t) w[t][j >> 2] |= (unsigned)(uint8_t)dj[t] << (8 * (j & 3));
    }
    for (int t = 0; t < S; ++t) {
        int8_t* o = out + (((int64_t)op * S + t) * Mp + row) * Kp + k0;
        *(uint4*)o = make_uint4(w[t][0], w[t][1], w[t][2], w[t][3]);
    }
}

// one workgroup per column of B (column c at B + c * ldb, K rows): exponent and S slices
template <int S>
__global__ __launch_bounds__(256) void k_oz_col_slices(const double* __restrict__ B, int64_t ldb, int K, int Kp,
                                                      int64_t ncols, int8_t* __restrict__ out, int* __restrict__ e) {
    const int64_t c = blockIdx.x;
    const double* col = B + c * ldb;
    __shared__ double s_m[256];
    double m = 0.0;
    for (int k = threadIdx.x; k < K; k += 256) m = fmax(m, fabs(col[k]));
    s_m[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s_m[threadIdx.x] = fmax(s_m[threadIdx.x], s_m[threadIdx.x + w]);
        __syncthreads();
    }
    const int ex = scale_exponent(s_m[0]);
    if (threadIdx.x == 0) e[c] = ex;
    for (int k = threadIdx.x; k < Kp; k += 256) {
        int8_t d[S];
        if (k < K) digits<S>(col[k], ex, d);
        else for (int t = 0; t < S; ++t) d[t] = 0;
        for (int t = 0; t < S; ++t) out[((int64_t)t * ncols + c) * Kp + k] = d[t];
    }
}

// Grouped gather GEMM on the sliced operands.  A 64 x 64 output tile per workgroup: four waves,
// 32 x 32 each = 2 x 2 blocks of 16 x 16; K staged through LDS 64 at a time (all S slices of
// the A rows and the gathered B columns), the next stage loaded into registers while the
// current one is multiplied.  Rows of LDS are padded to 80 bytes.
template <int S>
__global__ __launch_bounds__(256) void k_gemm_oz(OzArgs a) {
    const int per = (a.n_tiles + 7) / 8;                  // XCD-aware order, as the float64 GEMM
    const int logical = (blockIdx.x % 8) * per + blockIdx.x / 8;
    if (logical >= a.n_tiles) return;
    const Tile t = a.tiles[logical];
    const int8_t* __restrict__ A = a.a_sl + (int64_t)t.op * S * a.Mp * a.Kp;
    __shared__ v4i sA[S][kTile][5];
    __shared__ v4i sB[S][kTile][5];
    __shared__ int s_in[kTile];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
    if (tid < kTile) {
        const int j = t.col0 + tid, e = j / a.rhs;
        s_in[tid] = tid < t.ncol ? a.in_col[e] * a.rhs + (j - e * a.rhs) : -1;
    }
    __syncthreads();
    // this thread's share of a stage: 16 bytes at (lane % 4) * 16 of row/column
    // 16 * wave + 4 * ((lane / 4) % 4) + lane / 16: four consecutive lanes load one row's 64
    // contiguous bytes, and the 16 lanes of a quarter-wave store rows r, r+4, r+8, r+12, which the
    // 80-byte row stride places in distinct LDS banks
    const int sr = 16 * wave + 4 * ((lane >> 2) & 3) + (lane >> 4), sq = lane & 3;
    const int bcol = s_in[sr];
    const int8_t* ap = A + (int64_t)(t.row0 + sr) * a.Kp + sq * 16;
    // a padding column reads column 0 of the slices (in bounds) and is masked to zero
    const int8_t* bp = a.b_sl + (int64_t)(bcol >= 0 ? bcol : 0) * a.Kp + sq * 16;
    const int bmask = bcol >= 0 ? -1 : 0;
    const int64_t astride = (int64_t)a.Mp * a.Kp;
    v4i ra[S], rb[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
        ra[s] = *(const v4i*)(ap + s * astride);
        rb[s] = *(const v4i*)(bp + s * a.b_slice_stride);
    }
    v4i acc[S][2][2];
#pragma unroll
    for (int g = 0; g < S; ++g)
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) acc[g][i][j] = v4i{0, 0, 0, 0};
    for (int k0 = 0; k0 < a.Kp; k0 += kTile) {
#pragma unroll
        for (int s = 0; s < S; ++s) {
            sA[s][sr][sq] = ra[s];
            sB[s][sr][sq] = rb[s] & bmask;
        }
        __syncthreads();
        if (k0 + kTile < a.Kp) {                          // next stage in flight
            const int kn = k0 + kTile;
#pragma unroll
            for (int s = 0; s < S; ++s) {
                ra[s] = *(const v4i*)(ap + s * astride + kn);
                rb[s] = *(const v4i*)(bp + s * a.b_slice_stride + kn);
            }
        }
        v4i af[S][2], bf[S][2];
#pragma unroll
        for (int s = 0; s < S; ++s)
            for (int i = 0; i < 2; ++i) {
                af[s][i] = sA[s][wm + 16 * i + (lane & 15)][lane >> 4];
                bf[s][i] = sB[s][wn + 16 * i + (lane & 15)][lane >> 4];
            }
#pragma unroll
        for (int ta = 0; ta < S; ++ta)
#pragma unroll
            for (int ub = 0; ub < S - ta; ++ub)
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j)
                        acc[ta + ub][i][j] =
                            __builtin_amdgcn_mfma_i32_16x16x64_i8(af[ta][i], bf[ub][j], acc[ta + ub][i][j], 0, 0, 0);
        __syncthreads();
    }
    // D layout of a 16 x 16 block: lane holds column (lane & 15) and rows (lane >> 4) * 4 + v
    for (int j = 0; j < 2; ++j) {
        const int n = wn + 16 * j + (lane & 15);
        if (n >= t.ncol) continue;
        const int fe = s_in[n] >= 0 ? a.b_exp[s_in[n]] : 0;
        const int jj = t.col0 + n, e = jj / a.rhs;
        const int oc = a.out_col[e] * a.rhs + (jj - e * a.rhs);
        const double sc = a.scale[e];
        double* C = a.C + (int64_t)oc * a.ldc;
        for (int i = 0; i < 2; ++i)
            for (int v = 0; v < 4; ++v) {
                const int row = t.row0 + wm + 16 * i + (lane >> 4) * 4 + v;
                if (row >= a.M) continue;
                double val = 0.0;
#pragma unroll
                for (int g = S - 1; g >= 0; --g) val += ldexp((double)acc[g][i][j][v], -7 * (g + 2));
                const double r = sc * ldexp(val, a.a_exp[(int64_t)t.op * a.Mp + row] + fe);
                C[row] = a.accumulate ? C[row] + r : r;
            }
    }
}

}  // namespace

int oz_padded(int n) { return (n + kTile - 1) / kTile * kTile; }

void launch_oz_slice_operators(const double* ops, int n_ops, int M, int K, int8_t* out, int* e, hipStream_t s) {
    const int Mp = oz_padded(M), Kp = oz_padded(K);
    const int64_t nr = (int64_t)n_ops * Mp;
    hipLaunchKernelGGL(k_oz_row_exp, dim3((unsigned)((nr + 255) / 256)), dim3(256), 0, s, ops, n_ops, M, K, Mp, e);
    PK_HIP(hipGetLastError());
    const int64_t nq = nr * (Kp / 16);
    hipLaunchKernelGGL(k_oz_row_slices<kOzSlices>, dim3((unsigned)((nq + 255) / 256)), dim3(256), 0, s, ops, n_ops, M,
                       K, Mp, Kp, e, out);
    PK_HIP(hipGetLastError());
}

void launch_oz_slice_columns(const double* B, int64_t ldb, int K, int64_t ncols, int8_t* out, int* e, hipStream_t s) {
    if (ncols == 0) return;
    hipLaunchKernelGGL(k_oz_col_slices<kOzSlices>, dim3((unsigned)ncols), dim3(256), 0, s, B, ldb, K, oz_padded(K),
                       ncols, out, e);
    PK_HIP(hipGetLastError());
}

void launch_gemm_oz(const OzArgs& a, hipStream_t s) {
    if (a.n_tiles == 0) return;
    hipLaunchKernelGGL(k_gemm_oz<kOzSlices>, dim3((unsigned)((a.n_tiles + 7) / 8 * 8)), dim3(256), 0, s, a);
    PK_HIP(hipGetLastError());
}

}  // namespace pk
