// Kernel launchers shared between the schedule (plan.hip) and the kernel files.
#pragma once

#include "internal.h"

namespace pk {

// ---- points and densities (kernels_points.hip)
// Coordinates are divided by L, periodic axes wrapped into [0,1), the others checked to lie in [0,1]; then quantised and
// interleaved.  xyz: [n][3] input order.  Writes keys, values
// (= input index) and the wrapped coordinates u [3][n] (SoA).  Bit 0 of *err is
// set for a coordinate outside the box or not finite.
void launch_keys(const double* xyz, int64_t n, double L, unsigned mask, uint64_t* keys,
                 uint32_t* vals, double* u, int* err, hipStream_t s);
// Stable radix sort of (key, index) pairs on key bits [0, end_bit); temp storage is grown as
// needed.  With n_seg > 1 each segment [off[i], off[i+1]) is sorted on its own (off: device,
// n_seg+1, off[0] = 0, off[n_seg] = n; all 63 key bits), ties in input order.
void radix_sort_pairs(uint64_t* keys_in, uint64_t* keys_out, uint32_t* vals_in, uint32_t* vals_out,
                      int64_t n, DBuf<char>& temp, hipStream_t s, int n_seg = 1, const int64_t* off = nullptr,
                      int end_bit = 63);
// Sorted SoA coordinates xs[3][n] = u[:, perm]; per-point float offsets from the
// centre of the point's leaf (every leaf box listed once in leaves).
void launch_gather_points(const double* u, const uint32_t* perm, int64_t n, double* xs, hipStream_t s);
void launch_leaf_offsets(const double* xs, int64_t n, const int* leaves, int n_leaves, const int* box_begin,
                         const int* box_end, const int* box_level, const int* box_ix, const int* box_iy,
                         const int* box_iz, int* ioff, hipStream_t s);
// density [R][n_dens][k] input order -> ds [R][k][n] sorted (double) and optionally float; points
// with input index >= n_dens (separate targets) get zero density
void launch_permute_density(const double* dens, const uint32_t* perm, int64_t n, int64_t n_dens, int R, int k,
                            double* ds, float* ds32, hipStream_t s);
// pot_sorted [R][k][n] -> out [R][n_out][k], times scale: the point of input index j >= t_first is
// output row j - t_first (t_first = 0: every point; separate targets: the first target's index)
void launch_unpermute(const double* pot, const uint32_t* perm, int64_t n, int64_t t_first, int64_t n_out, int R,
                      int k, double scale, double* out, hipStream_t s);
// separate targets: keys[i] = (begin of i's leaf) << 1 | (perm[i] >= n_src) for the sorted points
// of every listed leaf, and n_sources[j] = the source count of leaf j
void launch_role_keys(const int* leaves, int n_leaves, const int* box_begin, const int* box_end, const uint32_t* perm,
                      int64_t n_src, uint64_t* keys, int* n_sources, hipStream_t s);
// x[0..n) = 0 with a kernel (no memset node under graph capture)
void launch_fill_zero(double* x, int64_t n, hipStream_t s);
// children key ranges of split boxes (box: [n_split][5] = begin, end, ix, iy, iz at level
// child_level - 1; out: [n_split][8][2] = first, end); keys sorted, device
void launch_tree_children(const uint64_t* keys, const int* box, int n_split, int child_level, int* out,
                          hipStream_t s);
// y[0..n) += x[0..n)
void launch_add_into(double* y, const double* x, int64_t n, hipStream_t s);
// per-problem, per-RHS, per-component sums and sums of magnitudes of the sorted densities
// (neutrality check): out [n_prob][R*k][2]; problem i owns sorted points [off[i], off[i+1])
// (off: device)
void launch_density_sums(const double* ds, int64_t n, int R, int k, const int64_t* off, int n_prob, double* out,
                         hipStream_t s);
// triply periodic Laplace: adds to every sorted potential pot [R][n] (raw 1/r units) its problem's
// far-field background constant (2 pi / 3)(sum_s q_s |y_s - c|^2 - sum_j phi_j |y_j - c|^2), c the
// box centre, phi the root's upward equivalent density (root of problem q: column block q of phi_u)
void launch_tp_background(const double* ds, const double* xs, int64_t n, const int64_t* off, int n_prob,
                          const double* phi_u, int R, const double* usurf, int n_surf, double* pot, hipStream_t s);
// sets *flag if two different points, or a point and another point's periodic image, lie in
// different cells of the 2^-21 grid and closer than delta in every coordinate (keys and xs
// sorted, per problem; xs the wrapped unit-box coordinates [3][n])
void launch_close_pairs(const uint64_t* keys, const double* xs, int64_t n, const int64_t* off, int n_prob,
                        unsigned mask, double delta, int* flag, hipStream_t s);

// ---- direct interactions (kernels_p2p.hip)
struct Seg {         // one source segment
    int kind;        // 0: points of box, 1: inner surface (phi_u), 2: outer surface (phi_d),
                     // 3: points of box, both ways (a U-list pair evaluated once: the box's
                     //    points also receive the item's targets, into partial slots),
                     // 4: outer surface of box, density from phi_d's column block `slot`
                     //    (the root's far-field density of step d)
    int box;
    int shift;       // (sx+1)*9 + (sy+1)*3 + (sz+1)
    int64_t slot = 0;   // kind 3: first partial slot (one per point of box); kind 4: column block
};
struct Work {        // one workgroup's targets and its segment range
    int tbox;        // target box
    int tkind;       // 0: points, 1: inner surface (downward check), 2: outer surface (upward check)
    int t0, tcount;  // first target (sorted index for points, surface index for surfaces) and count
    int seg0, seg1;
};
struct P2PArgs {
    int kernel;          // 1 Laplace, 2 Stokes
    int n_surf;          // surface points per box
    int R;               // right-hand sides
    int64_t n;           // points
    const double* xs;    // [3][n] sorted absolute coordinates
    const int* ioff;     // [3][n] offsets from the leaf centre in units of 2^-29 h_leaf (mixed)
    const double* ds;    // [R][k][n] sorted densities
    const float* ds32;   // [R][k][n] (mixed)
    const double* phi_u; // [nbox*R][kn]
    const double* phi_d;
    const int* box_level;
    const int* box_ix;
    const int* box_iy;
    const int* box_iz;
    const int* box_begin;
    const int* box_end;
    const int* box_send; // end of the box's sources (a leaf with separate targets holds its sources
                         // first, then its targets; otherwise box_end)
    const double* usurf; // [n_surf][3] unit surface grid on [-1,1]^3
    const Seg* segs;
    const Work* work;
    int n_work;
    double* out_pts;     // [R][k][n] sorted potentials (targets = points)
    int accumulate_pts;  // add into out_pts instead of storing
    double* out_surf;    // [nbox*R][kn] check potentials (targets = surfaces), accumulated
    double* mpart;       // [k][n_slots] kind-3 partial sums (float64), written once each
    int64_t n_slots;
    int grid_cap;        // k_p2p with work_counter: this many workgroups take items from the counter
    int rb_max;          // most right-hand sides sharing one pass over the geometry (0: the kernel's most)
    int guard_all;       // mixed form: guard zero separations in every segment (set when points of
                         // different leaves or images may round to one integer position)
    unsigned long long* work_counter;   // one word, cleared by launch_p2p before each launch of a
                                        // right-hand-side block; NULL: one workgroup per item
};
// right-hand sides are processed in blocks that share each pair's geometry; segments of
// kind 3 require R == 1
void launch_p2p(const P2PArgs& a, bool mixed, hipStream_t s);
// out[c][begin(b) + i] += sum over e in [in_off[j], in_off[j+1]) of mpart[c][in_slot[e] + i]
// for the leaves b = in_box[j], j < n_in (the other side of the kind-3 segments), in entry order
void launch_mutual_gather(const double* mpart, int64_t n_slots, int kd, const int* in_box, const int64_t* in_off,
                          const int64_t* in_slot, int n_in, const int* box_begin, const int* box_end, int64_t n,
                          double* out, hipStream_t s);
// points to surfaces only (S2M, X), float64, up to 64 targets per work item
void launch_p2s(const P2PArgs& a, hipStream_t s);

// ---- dense operator products (kernels_gemm.hip)
struct Tile {
    int op;       // operator index
    int col0;     // first entry in the column lists
    int ncol;     // columns in this tile (<= 64)
    int row0;     // first row
};
struct GemmArgs {
    const double* ops;    // operator g at ops + g * op_stride, column-major M x K
    int64_t op_stride;
    int M, K;
    const double* B;      // column j at B + j * ldb
    int64_t ldb;
    double* C;            // column j at C + j * ldc
    int64_t ldc;
    const Tile* tiles;
    int n_tiles;
    const int* in_col;    // 8 slots per column entry; slot kb = input column of K block kb (-1: zero)
    int in_stride;        // K blocks used (1..8)
    int kblock;           // rows of B per K block
    const int* out_col;
    const double* scale;
    int accumulate;       // C = scale*Op*B (+ C)
    int rhs;              // > 0: in_col, out_col and scale hold one value per entry e, and column j of
                          // a tile is entry j / rhs with right-hand side r = j % rhs: input column
                          // in_col[e] * rhs + r, output column out_col[e] * rhs + r (one K block)
};
// partial: workspace for split-K partial tiles (NULL disables splitting), capacity in doubles
void launch_gemm(const GemmArgs& a, hipStream_t s, double* partial = nullptr, int64_t partial_cap = 0);
int gemm_split_factor(int n_tiles, int K);
// q[b] += sum_{e in [off[b], off[b+1])} temp[e]  over R columns each; rows kn
void launch_segment_reduce(const double* temp, const int64_t* off, const int* boxes, int nboxes,
                           int R, int kn, double* q, hipStream_t s);

// ---- M2L on the int8 matrix cores with exact accumulation (kernels_oz.hip), mixed form
constexpr int kOzSlices = 6;          // base-2^7 digits per operand entry
constexpr int kOzRows = 128;          // output rows per tile of the int8 GEMM (columns: 64)
struct OzArgs {
    const int8_t* a_sl;   // operator slices [op][kOzSlices][Mp][Kp]
    const int* a_exp;     // [op][Mp] row exponents
    int Mp, Kp, M;        // padded rows (multiple of kOzRows) and K (of 64), real rows
    const int8_t* b_sl;   // column slices [kOzSlices][ncols][Kp]
    const int* b_exp;     // [ncols] column exponents
    int64_t b_slice_stride;   // ncols * Kp
    double* C;            // column j at C + j * ldc
    int64_t ldc;
    const Tile* tiles;
    int n_tiles;
    const int* in_col;    // per entry: input box column (columns expanded as GemmArgs::rhs)
    const int* out_col;   // per entry: output slot
    const double* scale;  // per entry
    int rhs;              // right-hand sides (>= 1)
    int accumulate;
};
int oz_padded(int n);          // n rounded up to the GEMM's K stage (64)
int oz_rows_padded(int n);     // n rounded up to kOzRows
// operators: n_ops column-major M x K float64 matrices, consecutive
void launch_oz_slice_operators(const double* ops, int n_ops, int M, int K, int8_t* out, int* e, hipStream_t s);
// columns c < ncols of B (at B + c * ldb, K rows)
void launch_oz_slice_columns(const double* B, int64_t ldb, int K, int64_t ncols, int8_t* out, int* e, hipStream_t s);
// rows: 64 (tiles of the float64 GEMM's list) or kOzRows (the 128-row list); the same bits
void launch_gemm_oz(const OzArgs& a, int rows, hipStream_t s);

// ---- operator construction (kernels_ops.hip), raw kernels (no 1/(4pi), 1/(8pi))
// out[(k*i+a) + (k*j+b)*ld] = K(X_i - Y_j)_{ab}; X, Y: [m][3], [n][3]
void launch_kmat(int kernel, const double* X, int m, const double* Y, int n, double* out, int64_t ld,
                 hipStream_t s);
// far-field periodic kernel over images |p|_inf > near (1, 2 or 3; 1 for doubly periodic sums)
// between point sets (same layout)
void launch_far_kmat(int kernel, unsigned mask, const double* X, int m, const double* Y, int n, double* out,
                     int64_t ld, int near, hipStream_t s);
// small helpers for the SVD factors
void launch_pinv_factors(const double* U, const double* Vt, const double* S, int kn, int r, double* Ut_r,
                         double* VS, hipStream_t s);

}  // namespace pk
