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
// [S][col][Kp].  Mp is kn rounded up to 128 (the tile's rows) and Kp to 64, and the padding is
// zero, so the GEMM has no bounds checks in its K loop.  Gathered input columns, output columns
// and scales are those of the float64 grouped GEMM (per-entry column lists with the right-hand
// side expanded on the device).  Two tilings give the same bits (the int32 sums are exact and
// the epilogue is the same): 64 x 64 tiles (the float64 GEMM's list, column block outer), and
// 128 x 64 tiles in operator, row block, column block order, so that the workgroups of one XCD
// that run together share an operator row block in L2 (half the L2 misses, at one workgroup
// per compute unit).  Which one is faster depends on the workload and on what runs beside it;
// it is a tuning choice.
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

// LDS position (in 16-byte chunks) of chunk c of staged row r: the four 16-byte chunks of a
// 64-byte row are permuted by XOR with (r / 2) mod 4.  Measured on gfx950 with a probe of 16
// waves: 16-byte reads of one chunk from 16 consecutive rows (a fragment) and 16-byte writes of
// four consecutive lanes to one row's four chunks run at the conflict-free rate with this
// permutation, while rows padded to 80 bytes, plain 64-byte rows and the XOR with (r / 4) mod 4
// or ((r / 2) XOR (r / 8)) mod 4 read at half of it.
__device__ __forceinline__ int oz_swz(int r, int c) { return r * 4 + (c ^ ((r >> 1) & 3)); }

// Per-tile epilogue data: the exponents of the tile's rows and, per column, its exponent, output
// column and scale.  Fetched right after the column list, before the first stage's loads, and
// parked in LDS once those are in, so that the epilogue reads LDS instead of waiting on a chain
// of dependent global loads.
template <int BM>
struct OzEpi {
    int ae[BM];
    int fe[kTile], oc[kTile];
    double sc[kTile];
};

// thread tid < BM fetches the exponent of row tid, BM <= tid < BM + 64 the data of column tid - BM
template <int BM>
__device__ __forceinline__ void oz_epi_fetch(const OzArgs& a, const Tile& t, const int* s_in, int tid, int& qi,
                                             int& qo, double& qs) {
    if (tid < BM) {
        const int row = t.row0 + tid;
        qi = row < a.M ? a.a_exp[(int64_t)t.op * a.Mp + row] : 0;
    } else if (tid < BM + kTile) {
        const int n = tid - BM;
        if (n < t.ncol) {
            const int jj = t.col0 + n, e = jj / a.rhs;
            qi = a.b_exp[s_in[n]];
            qo = a.out_col[e] * a.rhs + (jj - e * a.rhs);
            qs = a.scale[e];
        }
    }
}

template <int BM>
__device__ __forceinline__ void oz_epi_park(OzEpi<BM>& p, int tid, int qi, int qo, double qs) {
    if (tid < BM) {
        p.ae[tid] = qi;
    } else if (tid < BM + kTile) {
        p.fe[tid - BM] = qi;
        p.oc[tid - BM] = qo;
        p.sc[tid - BM] = qs;
    }
}

// A wave's 32 x 32 block of the tile (rows wm.., columns wn..) from its S diagonals: the D layout
// of a 16 x 16 block gives a lane column lane % 16 and rows 4 (lane / 16) + v, v < 4, so each lane
// writes four consecutive rows of a column (two 16-byte stores where aligned and in range).
template <int S, int BM>
__device__ __forceinline__ void oz_epilogue(const OzArgs& a, const Tile& t, const OzEpi<BM>& p,
                                            const v4i (&acc)[S][2][2], int wm, int wn, int lane) {
    typedef double v2d __attribute__((ext_vector_type(2)));
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int n = wn + 16 * j + (lane & 15);
        if (n >= t.ncol) continue;
        const int fe = p.fe[n];
        const double sc = p.sc[n];
        double* C = a.C + (int64_t)p.oc[n] * a.ldc;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int lr = wm + 16 * i + (lane >> 4) * 4;
            const int row = t.row0 + lr;
            double o[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                double val = 0.0;
#pragma unroll
                for (int g = S - 1; g >= 0; --g) val += ldexp((double)acc[g][i][j][v], -7 * (g + 2));
                o[v] = sc * ldexp(val, p.ae[lr + v] + fe);
            }
            double* c = C + row;
            if (row + 3 < a.M && ((uintptr_t)c & 15) == 0) {
                v2d lo = v2d{o[0], o[1]}, hi = v2d{o[2], o[3]};
                if (a.accumulate) {
                    lo = ((const v2d*)c)[0] + lo;
                    hi = ((const v2d*)c)[1] + hi;
                }
                ((v2d*)c)[0] = lo;
                ((v2d*)c)[1] = hi;
            } else {
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    if (row + v < a.M) c[v] = a.accumulate ? c[v] + o[v] : o[v];
            }
        }
    }
}

// Grouped gather GEMM on the sliced operands, 64-row tiles.  A 64 x 64 output tile per workgroup: four waves,
// 32 x 32 each = 2 x 2 blocks of 16 x 16; K staged through LDS 64 at a time (all S slices of
// the A rows and the gathered B columns, swizzled as oz_swz), the next stage loaded into
// registers while the current one is multiplied.
template <int S>
__global__ __launch_bounds__(256) void k_gemm_oz64(OzArgs a) {
    const int per = (a.n_tiles + 7) / 8;                  // XCD-aware order, as the float64 GEMM
    const int logical = (blockIdx.x % 8) * per + blockIdx.x / 8;
    if (logical >= a.n_tiles) return;
    const Tile t = a.tiles[logical];
    const int8_t* __restrict__ A = a.a_sl + (int64_t)t.op * S * a.Mp * a.Kp;
    __shared__ v4i sA[S][kTile * 4];
    __shared__ v4i sB[S][kTile * 4];
    __shared__ int s_in[kTile];
    __shared__ OzEpi<kTile> s_epi;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
    if (tid < kTile) {
        const int j = t.col0 + tid, e = j / a.rhs;
        s_in[tid] = tid < t.ncol ? a.in_col[e] * a.rhs + (j - e * a.rhs) : -1;
    }
    __syncthreads();
    int qi = 0, qo = 0;
    double qs = 0.0;
    oz_epi_fetch<kTile>(a, t, s_in, tid, qi, qo, qs);
    // this thread's share of a stage: 16-byte chunk tid % 4 of row/column tid / 4, for every
    // slice: four consecutive lanes load one row's 64 contiguous bytes
    const int sr = tid >> 2, sq = tid & 3;
    const int ws = oz_swz(sr, sq);
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
    oz_epi_park<kTile>(s_epi, tid, qi, qo, qs);           // read after the first barrier below
    v4i acc[S][2][2];
#pragma unroll
    for (int g = 0; g < S; ++g)
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) acc[g][i][j] = v4i{0, 0, 0, 0};
    for (int k0 = 0; k0 < a.Kp; k0 += kTile) {
#pragma unroll
        for (int s = 0; s < S; ++s) {
            sA[s][ws] = ra[s];
            sB[s][ws] = rb[s] & bmask;
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
                af[s][i] = sA[s][oz_swz(wm + 16 * i + (lane & 15), lane >> 4)];
                bf[s][i] = sB[s][oz_swz(wn + 16 * i + (lane & 15), lane >> 4)];
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
    oz_epilogue<S, kTile>(a, t, s_epi, acc, wm, wn, lane);
}



// Grouped gather GEMM on the sliced operands, 128-row tiles.  A 128 x 64 output tile per workgroup of eight
// waves, two per SIMD, each 32 x 32 (2 x 2 blocks of 16 x 16, S x 4 int32 accumulator blocks).
// K is staged through LDS 64 at a time (all S slices of the 128 operator rows and of the 64
// gathered columns) in two buffers, one barrier per stage: during stage k a wave multiplies
// from one buffer, writes stage k + 1 (loaded into registers during stage k - 1) to the other
// and loads stage k + 2, and reads the fragments of slice ta + 1 while slice ta is multiplied.
// Per stage a wave reads (2 + 2) x S fragments for 4 x S(S+1)/2 matrix instructions; the two
// waves of a SIMD overlap each other's reads and matrix instructions.
template <int S>
__global__ __launch_bounds__(512, 1) void k_gemm_oz128(OzArgs a) {
    constexpr int BM = kOzRows, BN = kTile, ROWS = BM + BN;
    constexpr int kStage = S * ROWS * 4;                  // one stage buffer, in 16-byte chunks
    static_assert(S % 2 == 0, "the column staging splits the slices in two halves");
    const int per = (a.n_tiles + 7) / 8;                  // XCD-aware order, as the float64 GEMM
    const int logical = (blockIdx.x % 8) * per + blockIdx.x / 8;
    if (logical >= a.n_tiles) return;
    const Tile t = a.tiles[logical];
    const int8_t* __restrict__ A = a.a_sl + (int64_t)t.op * S * a.Mp * a.Kp;
    __shared__ v4i sm[2 * kStage];
    __shared__ int s_in[BN];
    __shared__ OzEpi<BM> s_epi;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = (wave & 3) * 32, wn = (wave >> 2) * 32;
    if (tid < BN) {
        const int j = t.col0 + tid, e = j / a.rhs;
        s_in[tid] = tid < t.ncol ? a.in_col[e] * a.rhs + (j - e * a.rhs) : -1;
    }
    __syncthreads();
    int qi = 0, qo = 0;
    double qs = 0.0;
    oz_epi_fetch<BM>(a, t, s_in, tid, qi, qo, qs);
    // staging: thread tid moves 16-byte chunk c = tid % 4 of operator row r = tid / 4 for every
    // slice, and of gathered column r % 64 for slices (r / 64) S/2 .. (r / 64) S/2 + S/2 - 1;
    // four consecutive lanes read one row's 64 contiguous bytes.  A padding column reads column
    // 0 of the slices (in bounds); its outputs are never stored.
    const int c = tid & 3, r = tid >> 2, rb = r & 63;
    const int sb0 = __builtin_amdgcn_readfirstlane((tid >> 8) * (S / 2));   // uniform per wave
    const int bcol = s_in[rb];
    // per-lane 32-bit offsets from wave-uniform slice bases (the scalar-base load form)
    const unsigned oa = (unsigned)(r * a.Kp + c * 16);
    const unsigned ob = (unsigned)((bcol >= 0 ? bcol : 0) * a.Kp + c * 16);
    const int8_t* ar = A + (int64_t)t.row0 * a.Kp;
    const int64_t astride = (int64_t)a.Mp * a.Kp;
    const int wa = oz_swz(r, c), wb = oz_swz(BM + rb, c);
    v4i ra[S], rbv[S / 2];
    auto load = [&](int k0) {
#pragma unroll
        for (int s = 0; s < S; ++s) ra[s] = *(const v4i*)(ar + s * astride + k0 + oa);
        const int8_t* bs = a.b_sl + sb0 * a.b_slice_stride + k0;
#pragma unroll
        for (int h = 0; h < S / 2; ++h) rbv[h] = *(const v4i*)(bs + h * a.b_slice_stride + ob);
    };
    auto store = [&](v4i* buf) {
#pragma unroll
        for (int s = 0; s < S; ++s) buf[s * ROWS * 4 + wa] = ra[s];
#pragma unroll
        for (int h = 0; h < S / 2; ++h) buf[(sb0 + h) * ROWS * 4 + wb] = rbv[h];
    };
    // fragment positions: A block i (rows wm + 16 i + lane % 16), B block j (columns
    // wn + 16 j + lane % 16), K chunk lane / 16
    int fa[2], fb[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) fa[i] = oz_swz(wm + 16 * i + (lane & 15), lane >> 4);
#pragma unroll
    for (int j = 0; j < 2; ++j) fb[j] = oz_swz(BM + wn + 16 * j + (lane & 15), lane >> 4);
    v4i acc[S][2][2];
#pragma unroll
    for (int g = 0; g < S; ++g)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[g][i][j] = v4i{0, 0, 0, 0};
    const int nk = a.Kp / kTile;
    load(0);
    store(sm);
    oz_epi_park<BM>(s_epi, tid, qi, qo, qs);
    if (nk > 1) load(kTile);
    __syncthreads();
    for (int k = 0; k < nk; ++k) {
        const v4i* cur = sm + (k & 1) * kStage;
        v4i* nxt = sm + ((k + 1) & 1) * kStage;
        v4i bf[S][2], af[2][2];
#pragma unroll
        for (int i = 0; i < 2; ++i) af[0][i] = cur[fa[i]];
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
            for (int j = 0; j < 2; ++j) bf[s][j] = cur[s * ROWS * 4 + fb[j]];
#pragma unroll
        for (int ta = 0; ta < S; ++ta) {
            if (ta + 1 < S) {
#pragma unroll
                for (int i = 0; i < 2; ++i) af[(ta + 1) & 1][i] = cur[(ta + 1) * ROWS * 4 + fa[i]];
            }
#pragma unroll
            for (int ub = 0; ub < S - ta; ++ub)
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j)
                        acc[ta + ub][i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(af[ta & 1][i], bf[ub][j],
                                                                                   acc[ta + ub][i][j], 0, 0, 0);
            if (ta == 1 && k + 1 < nk) {            // stage k + 1 to the other buffer, stage k + 2 in flight
                store(nxt);
                if (k + 2 < nk) load((k + 2) * kTile);
            }
        }
        __syncthreads();
    }
    oz_epilogue<S, BM>(a, t, s_epi, acc, wm, wn, lane);
}

}  // namespace

int oz_padded(int n) { return (n + kTile - 1) / kTile * kTile; }
int oz_rows_padded(int n) { return (n + kOzRows - 1) / kOzRows * kOzRows; }

void launch_oz_slice_operators(const double* ops, int n_ops, int M, int K, int8_t* out, int* e, hipStream_t s) {
    const int Mp = oz_rows_padded(M), Kp = oz_padded(K);
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

void launch_gemm_oz(const OzArgs& a, int rows, hipStream_t s) {
    if (a.n_tiles == 0) return;
    if (rows == kOzRows)
        hipLaunchKernelGGL(k_gemm_oz128<kOzSlices>, dim3((unsigned)((a.n_tiles + 7) / 8 * 8)), dim3(512), 0, s, a);
    else
        hipLaunchKernelGGL(k_gemm_oz64<kOzSlices>, dim3((unsigned)((a.n_tiles + 7) / 8 * 8)), dim3(256), 0, s, a);
    PK_HIP(hipGetLastError());
}

}  // namespace pk
