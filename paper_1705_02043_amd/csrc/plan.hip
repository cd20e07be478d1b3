// The C interface: plan construction (operators), point set-up (tree and
// lists) and the evaluation schedule of the periodic KIFMM.
//
// Evaluation schedule (Algorithm 2, Stage 2, with step d folded into the
// downward pass; all arrays Morton-ordered, one column of kn = k n values per
// box and right-hand side):
//   1. permute densities into Morton order
//   2. S2M at the leaves (direct sums to the upward check surface)
//   3. upward pass, deepest level first: M2M from children, then the upward
//      check-to-equivalent solve phi = h (V S^+)(U^T q)
//   4. root far field: q^{B0,d} += M_root phi^{B0,u}
//   5. V-list M2L for every level at once (grouped by offset, summed per
//      target in a fixed order) and X-list direct sums to downward check
//      surfaces
//   6. downward pass, root first: L2L from the parent, downward solve
//   7. leaves: U-list direct sums, W-list M2T and L2T into the potentials
// W/X-list interactions take the cheaper of their two forms: a leaf with no more
// points than a surface acts (W) or is acted on (X) by direct sums instead of
// through its equivalent/check surface.
//   8. un-permute and apply 1/(4 pi) or 1/(8 pi) and 1/L
// With PKIFMM_FAR_STEP_D the root's downward solve writes its own column block
// (after the tree's boxes), the roots pass nothing down the tree, and every leaf's
// L2T item also evaluates that block on the root's outer surface: the paper's own
// step d.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <exception>
#include <future>
#include <system_error>
#include <memory>
#include <mutex>
#include <thread>
#include <type_traits>

#include "launch.h"
#include "opcache.h"

using namespace pk;

thread_local const Allocator* pk::g_alloc = nullptr;

namespace {

constexpr double kInnerHalf = 0.525;   // half edge of the 1.05 cube, in box edges
constexpr double kNeutralRel = 1e-12;  // SP/DP neutrality: |sum phi| <= this * sum |phi|
constexpr double kSolveCheckTol = 1e-13;   // normwise backward error of the solves on their kept subspace
// default relative cutoff of the check-to-equivalent solves: singular values <= 1e-11 s_max are
// dropped (below it the solve turns the tens-of-ulps rounding of its input into equivalent-density
// noise without improving accuracy against the exact periodic sums)
constexpr double kDefaultSvdCut = 1e-11;
// mixed form: points closer than this (unit-box coordinates) in every coordinate may share an
// integer position in the near field (at most 2 units of 2^-29 of a leaf edge <= 1 apart)
constexpr double kCloseDelta = 1.0 / (1 << 27);
constexpr double kOuterHalf = 1.475;   // half edge of the 2.95 cube

std::vector<double> unit_surface(int p) {
    std::vector<double> u;
    for (int i = 0; i < p; ++i)
        for (int j = 0; j < p; ++j)
            for (int k = 0; k < p; ++k) {
                bool face = i == 0 || i == p - 1 || j == 0 || j == p - 1 || k == 0 || k == p - 1;
                if (!face) continue;
                u.push_back(-1.0 + 2.0 * i / (p - 1));
                u.push_back(-1.0 + 2.0 * j / (p - 1));
                u.push_back(-1.0 + 2.0 * k / (p - 1));
            }
    return u;
}

std::vector<double> scaled(const std::vector<double>& u, double f, double cx, double cy, double cz) {
    std::vector<double> o(u.size());
    for (size_t i = 0; i < u.size(); i += 3) {
        o[i] = cx + f * u[i];
        o[i + 1] = cy + f * u[i + 1];
        o[i + 2] = cz + f * u[i + 2];
    }
    return o;
}

struct Gemm {      // host-side description of one grouped GEMM launch
    std::vector<Tile> tiles;
    std::vector<int> in, out;
    std::vector<double> scale;
};

struct GemmRange {
    int set = 0;            // 0: tree-pass GEMMs (levels, root), 1: M2L
    int tile0 = 0, ntile = 0;
};

struct SegRange {
    int set = 0;            // 0: S2M items, 1: leaf items (near field, W + L2T), 2: X items
    int work0 = 0, nwork = 0;
};

// Launch choices that change no result bit, chosen per (device architecture, kernel, periodic
// axes, p, precision, n_rhs) by pkifmm_autotune and read from a tuning file at plan creation.
struct Tuning {
    int near_wpc = 4;       // near-field workgroups per compute unit taking items from the counter
    int rb_near = 0;        // right-hand sides per near-field geometry pass (0: 16 Laplace, 4 Stokes)
    int rb_s2m = 0;         // right-hand sides per points-to-surface pass (0: 8 Laplace, 4 Stokes)
    int m2l_rows = 64;      // operator rows per tile of the mixed form's int8 M2L (64 or 128)
};
struct TuneRec {
    int R;
    Tuning t;
};

struct GemmSet {            // device copy of one Gemm description
    DBuf<Tile> tiles;
    DBuf<int> col_in, col_out;
    DBuf<double> col_scale;
};

// Device workspace of one evaluation: the plan's own buffers (pkifmm_evaluate), or regions of
// the library's static array (pkifmm_evaluate_noalloc).
struct Workspace {
    bool from_plan = true;
    double *ds = nullptr, *pot = nullptr, *q_u = nullptr, *phi_u = nullptr, *q_d = nullptr, *q_x = nullptr;
    double *phi_d = nullptr, *tmp = nullptr, *m2l_tmp = nullptr, *split_tmp = nullptr, *mpart = nullptr;
    double *sums = nullptr, *counter = nullptr;
    float* ds32 = nullptr;
    int8_t* phi_oz = nullptr;
    int* phi_oz_e = nullptr;
    int64_t split_cap = 0;      // doubles at split_tmp
};

// pkifmm_evaluate_noalloc's workspace: one array per GPU, held until the process ends.  Host
// code never uses the name itself as an address: each device's address of it is looked up once
// (scratch_address) and kept.
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device dev, which must be the current device.
void* scratch_address(int dev) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (dev < 0 || dev >= kMaxDevices) throw Error(PKIFMM_ERR_INVALID_ARG, "device ordinal beyond the static workspace table");
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        PK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) throw Error(PKIFMM_ERR_HIP, "static workspace has no device address");
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

}  // namespace

struct pkifmm_plan {
    Allocator allocator;                // first member: destroyed after every buffer it made
    pkifmm_config cfg{};
    int k = 1, n_surf = 0, kn = 0;
    int r_up = 0, r_dn = 0;
    std::vector<double> f_up_Ut, f_up_VS, f_dn_Ut, f_dn_VS;   // host copies of the solve factors (inspection)
    std::string last_error;
    hipStream_t setup_stream = nullptr;
    hipStream_t setup_stream2 = nullptr;        // uploads of the M2L work lists (built on a second host thread)
    hipStream_t setup_stream3 = nullptr;        // uploads of the near-field work lists (a third host thread)
    hipStream_t near_stream = nullptr;          // near field, concurrent with the end of M2L
    hipStream_t x_stream = nullptr;             // X list, beside the upward pass and M2L
    hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_xjoin = nullptr;
    hipEvent_t ev_done = nullptr;               // end of the last evaluation enqueued (all streams joined)
    hipStream_t capture_stream = nullptr;      // PKIFMM_GRAPH: the evaluation is captured here
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    int g_key_R = 0;
    bool capturing = false;
    const double* g_key_in = nullptr;
    double* g_key_out = nullptr;
    uint64_t g_key_gen = 0, generation = 0;
    int n_cu = 256;
    int dev = 0;                        // the device the plan was created on
    void* scratch_base = nullptr;       // that device's address of the static workspace

    // operators (device, float64, column-major kn x kn unless noted)
    DBuf<double> usurf;                 // [n][3]
    DBuf<double> up_Ut, up_VS, dn_Ut, dn_VS;   // U^T: r x kn, V S^+: kn x r
    DBuf<double> m2m, l2l;              // [8][kn*kn]
    DBuf<double> m2l;                   // [316][kn*kn]
    // mixed form: M2L operators and upward densities as int8 digit slices (kernels_oz.hip)
    DBuf<int8_t> m2l_oz;                // [316][kOzSlices][Mp][Kp]
    DBuf<int> m2l_oz_e;                 // [316][Mp] row exponents
    DBuf<int8_t> phi_oz;                // [kOzSlices][nbox*R][Kp]
    DBuf<int> phi_oz_e;                 // [nbox*R] column exponents
    DBuf<double> mroot;                 // [kn*kn]

    // points and tree (a forest: one tree per problem, boxes numbered level-major).  With separate
    // targets the points are the union: sources (input indices [0, n_src)) then targets; every leaf
    // holds its sources first ([begin, box_send)), then its targets ([box_tbeg, end))
    int64_t n = 0;
    int64_t n_src = 0;                  // density rows
    int64_t t_first = 0, n_out = 0;     // input index of the first target, potential rows
    bool separate = false;
    std::vector<int> box_send, box_tbeg;
    DBuf<int> b_send, leaf_nsrc;
    PinnedBuf<int> leaf_nsrc_host;
    DBuf<double> xyz_union;
    int n_problems = 1;
    std::vector<int64_t> prob_off_h;
    DBuf<int64_t> prob_off;
    std::vector<int> box_prob;
    bool have_points = false;
    HostTree tree;
    HostLists lists;
    std::vector<int64_t> perm_host;
    DBuf<uint64_t> keys_a, keys_b;
    DBuf<uint32_t> vals_a, perm;
    DBuf<double> u_wrapped, xs;
    DBuf<int> ioff;
    DBuf<char> sort_temp;
    DBuf<int> err_flag;                 // [0]: a coordinate out of the box; [1]: close points (mixed form)
    bool guard_all = false;             // mixed form: guard zero separations in every near-field segment
    DBuf<int> b_level, b_ix, b_iy, b_iz, b_begin, b_end, leaf_boxes;
    PinnedBuf<uint64_t> keys_host;
    DBuf<int> tree_box, tree_out;       // per-level split boxes and their children (device tree build)
    PinnedBuf<int> tree_out_host;
    // the host lists of the current points: for one problem built on a host thread that
    // set_points starts, so that an evaluation can enqueue its permutation, S2M and upward pass
    // first; every reader of the lists or of their statistics waits for it (lists_wait)
    std::shared_future<void> lists_ready;

    // work lists for the current R
    int R_built = -1;
    SegRange w_s2m, w_x, w_leaf_u, w_leaf_far;
    DBuf<Seg> segs[3];                  // per SegRange set
    DBuf<Work> work[3];
    // U-list pairs evaluated once (one right-hand side): partial slots and, per leaf that is
    // the other side of such pairs, its slots in a fixed order
    Tuning tune;                        // the choices of the evaluation being enqueued
    std::vector<TuneRec> tune_table;    // tuned choices of this plan's key, per n_rhs
    bool tune_fixed = false;            // pkifmm_autotune is timing `tune` itself
    std::string arch;                   // device architecture name (gfx950, ...)
    DBuf<double> counter;               // near-field work counter (one 64-bit word)
    bool mutual = false;
    int64_t n_slots = 0;
    int n_in = 0;
    DBuf<double> mpart;
    DBuf<int> in_box;
    DBuf<int64_t> in_off, in_slot;
    std::vector<GemmRange> g_m2m;       // per level
    std::vector<GemmRange> g_up1, g_up2, g_dn1, g_dn2, g_l2l;   // per level
    GemmRange g_root;
    std::vector<GemmRange> g_m2l;                        // per offset group
    std::vector<GemmRange> g_m2l_wide;                   // the same, 128-row tiles (mixed form)
    std::vector<std::pair<int, int>> m2l_targets;        // per group: (first, count) in v_gtargets
    DBuf<int64_t> v_goff;                                // per group: CSR over boxes of temp slots
    DBuf<int> v_gtargets;
    int m2l_slots = 1;
    int64_t split_need = 1;             // doubles of split-K partial tiles the tree passes use
    GemmSet gsets[2];                   // per GemmRange set

    // workspace
    DBuf<double> ds, q_u, phi_u, q_d, q_x, phi_d, tmp, m2l_tmp, pot, sums, split_tmp;
    DBuf<float> ds32;

    pkifmm_stats stats{};
    std::vector<std::vector<hipEvent_t>> pending_events;   // per timed evaluation: NUM_PHASES + 1
};

namespace {

int fail(pkifmm_plan* p, const Error& e) {
    if (p) p->last_error = e.what();
    return e.code;
}

int near_layers(const pkifmm_config& c) { return c.near_layers > 1 ? c.near_layers : 1; }

void check_config(const pkifmm_config& c) {
    if (c.kernel != PKIFMM_LAPLACE && c.kernel != PKIFMM_STOKES) throw Error(PKIFMM_ERR_INVALID_ARG, "kernel");
    if (c.periodic_mask & ~7u) throw Error(PKIFMM_ERR_INVALID_ARG, "periodic_mask");
    if (c.p < 4 || c.p > 16) throw Error(PKIFMM_ERR_INVALID_ARG, "p must be in [4, 16]");
    if (c.max_pts_per_leaf < 1) throw Error(PKIFMM_ERR_INVALID_ARG, "max_pts_per_leaf");
    if (c.precision != PKIFMM_FP64 && c.precision != PKIFMM_MIXED) throw Error(PKIFMM_ERR_INVALID_ARG, "precision");
    if (!(c.box_length > 0.0) || !std::isfinite(c.box_length)) throw Error(PKIFMM_ERR_INVALID_ARG, "box_length");
    if (c.svd_rel_threshold < 0.0 || c.svd_rel_threshold >= 1.0) throw Error(PKIFMM_ERR_INVALID_ARG, "svd_rel_threshold");
    const unsigned known = PKIFMM_SKIP_CHECKS | PKIFMM_PHASE_TIMING | PKIFMM_GRAPH | PKIFMM_FAR_STEP_D;
    if (c.flags & ~known) throw Error(PKIFMM_ERR_INVALID_ARG, "flags");
    if ((c.alloc == nullptr) != (c.free == nullptr)) throw Error(PKIFMM_ERR_INVALID_ARG, "alloc and free go together");
    if (c.near_layers < 0 || c.near_layers > 3) throw Error(PKIFMM_ERR_INVALID_ARG, "near_layers must be 0 .. 3");
    if (c.near_layers > 1 && __builtin_popcount(c.periodic_mask) == 2)
        throw Error(PKIFMM_ERR_UNSUPPORTED, "near_layers > 1 for doubly periodic sums");
}

void check_solve(const double* A_dev, int kn, int r, const std::vector<double>& hUt, const std::vector<double>& hVS,
                 double s_max);

// SVD of a kn x kn matrix on the device (rocSOLVER, one-sided bidiagonal QR);
// drops singular values <= thr * s_max and stores U^T (r x kn) and V S^+ (kn x r), on the device
// and in hUt, hVS; *s_max_out receives s_max.
int pinv_build(rocblas_handle h, hipStream_t s, const double* A_dev, int kn, double thr, DBuf<double>& Ut,
               DBuf<double>& VS, std::vector<double>& hUt, std::vector<double>& hVS, double* s_max_out) {
    DBuf<double> A, S, U, Vt, E;
    DBuf<rocblas_int> info;
    A.ensure((size_t)kn * kn);
    S.ensure(kn);
    U.ensure((size_t)kn * kn);
    Vt.ensure((size_t)kn * kn);
    E.ensure(kn);
    info.ensure(1);
    PK_HIP(hipMemcpyAsync(A.p, A_dev, sizeof(double) * kn * kn, hipMemcpyDeviceToDevice, s));
    rocblas_status st = rocsolver_dgesvd(h, rocblas_svect_all, rocblas_svect_all, kn, kn, A.p, kn, S.p, U.p, kn, Vt.p,
                                         kn, E.p, rocblas_outofplace, info.p);
    if (st != rocblas_status_success) throw Error(PKIFMM_ERR_HIP, "rocsolver_dgesvd failed");
    std::vector<double> sv(kn);
    rocblas_int inf = 0;
    PK_HIP(hipMemcpyAsync(sv.data(), S.p, sizeof(double) * kn, hipMemcpyDeviceToHost, s));
    PK_HIP(hipMemcpyAsync(&inf, info.p, sizeof(inf), hipMemcpyDeviceToHost, s));
    PK_HIP(hipStreamSynchronize(s));
    if (inf != 0) throw Error(PKIFMM_ERR_NUMERICS, "SVD did not converge");
    int r = 0;
    while (r < kn && sv[r] > thr * sv[0]) ++r;
    if (r == 0) throw Error(PKIFMM_ERR_NUMERICS, "zero matrix");
    Ut.ensure((size_t)r * kn);
    VS.ensure((size_t)kn * r);
    launch_pinv_factors(U.p, Vt.p, S.p, kn, r, Ut.p, VS.p, s);
    PK_HIP(hipStreamSynchronize(s));
    hUt.assign((size_t)r * kn, 0.0);
    hVS.assign((size_t)kn * r, 0.0);
    PK_HIP(hipMemcpy(hUt.data(), Ut.p, sizeof(double) * r * kn, hipMemcpyDeviceToHost));
    PK_HIP(hipMemcpy(hVS.data(), VS.p, sizeof(double) * kn * r, hipMemcpyDeviceToHost));
    *s_max_out = sv[0];
    check_solve(A_dev, kn, r, hUt, hVS, sv[0]);
    return r;
}

// Backward-stability self-check of a solve (Appendix B), normwise and on the kept subspace.
    // backward-stability self-check (Appendix B), normwise and on the kept subspace: for x = (V S^+) z,
    // which the truncation leaves intact, q = A x must come back with ||A (V S^+)(U^T q) - q|| at
    // the rounding level of ||A|| ||x|| = s_max ||x||, whatever the cutoff (measured 3e-17 ..
    // 3e-16 for Stokes p = 8 .. 16; a wrong factor gives order 1)
void check_solve(const double* A_dev, int kn, int r, const std::vector<double>& hUt, const std::vector<double>& hVS,
                 double s_max) {
    std::vector<double> hA((size_t)kn * kn);
    PK_HIP(hipMemcpy(hA.data(), A_dev, sizeof(double) * kn * kn, hipMemcpyDeviceToHost));
    std::vector<double> z(r), x(kn, 0.0), q(kn, 0.0), t(r, 0.0), ph(kn, 0.0), aq(kn, 0.0);
    for (int i = 0; i < r; ++i) z[i] = std::sin(1.0 + 0.37 * i);
    for (int j = 0; j < r; ++j)
        for (int i = 0; i < kn; ++i) x[i] += hVS[i + (size_t)j * kn] * z[j];
    for (int j = 0; j < kn; ++j)
        for (int i = 0; i < kn; ++i) q[i] += hA[i + (size_t)j * kn] * x[j];
    for (int j = 0; j < kn; ++j)
        for (int i = 0; i < r; ++i) t[i] += hUt[i + (size_t)j * r] * q[j];
    for (int j = 0; j < r; ++j)
        for (int i = 0; i < kn; ++i) ph[i] += hVS[i + (size_t)j * kn] * t[j];
    for (int j = 0; j < kn; ++j)
        for (int i = 0; i < kn; ++i) aq[i] += hA[i + (size_t)j * kn] * ph[j];
    double num = 0, xx = 0;
    for (int i = 0; i < kn; ++i) {
        num += (aq[i] - q[i]) * (aq[i] - q[i]);
        xx += x[i] * x[i];
    }
    if (!(std::sqrt(num) < kSolveCheckTol * s_max * std::sqrt(xx)))
        throw Error(PKIFMM_ERR_NUMERICS, "check-to-equivalent solve failed its backward-error check");
}

// in: nkb input columns per output column (K blocks), -1 for a zero block; ncols output columns
void add_gemm(Gemm& g, int op, int M, const int* in, const int* out, const double* sc, size_t ncols, int nkb = 1) {
    // eight input slots per column (K blocks; unused ones -1), then the column's output and
    // scale; one tile per 64 columns and 64 rows
    const size_t in0 = g.in.size(), col00 = g.out.size();
    g.in.resize(in0 + 8 * ncols, -1);
    int* gi = g.in.data() + in0;
    for (size_t c = 0; c < ncols; ++c)
        for (int kb = 0; kb < nkb; ++kb) gi[8 * c + kb] = in[c * nkb + kb];
    g.out.insert(g.out.end(), out, out + ncols);
    g.scale.insert(g.scale.end(), sc, sc + ncols);
    for (size_t c0 = 0; c0 < ncols; c0 += 64) {
        const int ncol = (int)std::min<size_t>(64, ncols - c0);
        for (int r0 = 0; r0 < M; r0 += 64) g.tiles.push_back(Tile{op, (int)(col00 + c0), ncol, r0});
    }
}

void add_gemm(Gemm& g, int op, int M, const std::vector<int>& in, const std::vector<int>& out,
              const std::vector<double>& sc, int nkb = 1) {
    add_gemm(g, op, M, in.data(), out.data(), sc.data(), out.size(), nkb);
}

double box_edge(const HostTree& t, int b) { return std::ldexp(1.0, -t.level[b]); }

// Octree of one problem from its device-sorted keys, level by level on the device: the host
// keeps the box table and decides which boxes split (more than s points); the children's key
// ranges come from two binary searches per (split box, octant) on the device.  Boxes are
// numbered exactly as a sequential pass over each level's boxes and octants would number them.
void build_tree_device(pkifmm_plan* P, const uint64_t* keys, int64_t n, int s_max, HostTree& t, hipStream_t s) {
    t = HostTree();
    auto add = [&](int lv, int x, int y, int z, int b0, int b1, int par) {
        t.level.push_back(lv); t.ix.push_back(x); t.iy.push_back(y); t.iz.push_back(z);
        t.begin.push_back(b0); t.end.push_back(b1); t.parent.push_back(par);
        for (int o = 0; o < 8; ++o) t.child.push_back(-1);
        return (int)t.level.size() - 1;
    };
    add(0, 0, 0, 0, 0, (int)n, -1);
    t.level_start.push_back(0);
    int lv = 0;
    std::vector<int> frontier{0}, split, box;
    while (!frontier.empty() && lv < kMaxLevel) {
        split.clear();
        box.clear();
        for (int b : frontier)
            if (t.end[b] - t.begin[b] > s_max) {
                split.push_back(b);
                box.insert(box.end(), {t.begin[b], t.end[b], t.ix[b], t.iy[b], t.iz[b]});
            }
        if (split.empty()) break;
        const int ns = (int)split.size();
        P->tree_box.upload(box, s);
        P->tree_out.ensure((size_t)16 * ns);
        P->tree_out_host.ensure((size_t)16 * ns);
        launch_tree_children(keys, P->tree_box.p, ns, lv + 1, P->tree_out.p, s);
        PK_HIP(hipMemcpyAsync(P->tree_out_host.p, P->tree_out.p, sizeof(int) * 16 * ns, hipMemcpyDeviceToHost, s));
        PK_HIP(hipStreamSynchronize(s));
        const int* r = P->tree_out_host.p;
        std::vector<int> next;
        for (int i = 0; i < ns; ++i) {
            const int b = split[i];
            for (int o = 0; o < 8; ++o) {
                const int a = r[16 * i + 2 * o], e = r[16 * i + 2 * o + 1];
                if (e <= a) continue;
                const int c = add(lv + 1, 2 * t.ix[b] + ((o >> 2) & 1), 2 * t.iy[b] + ((o >> 1) & 1),
                                  2 * t.iz[b] + (o & 1), a, e, b);
                t.child[8 * b + o] = c;
                next.push_back(c);
            }
        }
        if (next.empty()) break;
        ++lv;
        t.level_start.push_back(next.front());
        frontier.swap(next);
    }
    t.depth = lv;
    t.level_start.push_back(t.nbox());
    t.leaf_id.assign(t.nbox(), -1);
    for (int b = 0; b < t.nbox(); ++b)
        if (t.is_leaf(b)) {
            t.leaf_id[b] = (int)t.leaves.size();
            t.leaves.push_back(b);
        }
}

// The host lists and their statistics, once the thread that set_points started has built them;
// rethrows what building them threw.
void lists_wait(const pkifmm_plan* P) {
    std::shared_future<void> f = P->lists_ready;
    if (f.valid()) f.get();
}

// Before the points change or the plan goes: the lists thread has ended (its error, if any, is
// dropped with the lists it was building).
void lists_settle(pkifmm_plan* P) {
    if (P->lists_ready.valid()) P->lists_ready.wait();
    P->lists_ready = std::shared_future<void>();
}

// Sizes of the current lists and the number of near-field (U-list) point pairs.
void list_stats(pkifmm_plan* P) {
    const HostTree& t = P->tree;
    const HostLists& L = P->lists;
    auto& st = P->stats;
    st.n_u = (int64_t)L.u.size();
    st.n_v = (int64_t)L.v.size();
    st.n_w = (int64_t)L.w.size();
    st.n_x = (int64_t)L.x.size();
    int64_t up = 0;
    for (int b : t.leaves)
        for (int64_t e = L.u_off[b]; e < L.u_off[b + 1]; ++e) {
            const int a = L.u[e].src;
            up += (int64_t)(t.end[b] - P->box_tbeg[b]) * (P->box_send[a] - t.begin[a]);
        }
    st.u_pairs = up;
}

// Work lists of one (tree, R) are built in three stages, each uploaded on the setup stream
// into its own buffers, so that an evaluation can launch the kernels of a stage while the
// host builds the next one.

// The far field evaluated at the targets from the root's own density (step d) rather than
// handed down the tree
bool far_step_d(const pkifmm_plan* P) {
    return (P->cfg.flags & PKIFMM_FAR_STEP_D) != 0 && P->cfg.periodic_mask != 0;
}

// The per-level GEMMs of levels 0 .. kSplitLevels split K over several workgroups (few boxes
// per problem there: the launches are latency-bound); deeper levels never do, since their
// launches fill the chip and the partial tiles would cost more than they save.  The choice
// depends on the level alone, so a problem's summation order (and every result bit) is the
// same alone and in a batch.
constexpr int kSplitLevels = 3;

// Stage 1: S2M items, per-level and root GEMMs, workspace (the tree alone: no host lists).
void build_stage_tree(pkifmm_plan* P, int R) {
    const HostTree& t = P->tree;
    const int nb = t.nbox();
    const int ns = P->n_surf;
    std::vector<Seg> segs;
    std::vector<Work> work;
    const int kSelf = 13;
    // S2M: leaf points -> own upward check surface
    P->w_s2m = SegRange{0, (int)work.size(), 0};
    for (int b : t.leaves) {
        if (P->box_send[b] == t.begin[b]) continue;   // a leaf of targets only
        int s0 = (int)segs.size();
        segs.push_back(Seg{0, b, kSelf});
        for (int c0 = 0; c0 < ns; c0 += 64) work.push_back(Work{b, 2, c0, std::min(64, ns - c0), s0, s0 + 1});
    }
    P->w_s2m.nwork = (int)work.size() - P->w_s2m.work0;
    hipStream_t s = P->setup_stream;
    P->segs[0].upload(segs, s);
    P->work[0].upload(work, s);

    // GEMM launches
    Gemm g;
    const int kn = P->kn;
    auto range = [&](auto&& fill) {
        GemmRange r;
        r.set = 0;
        r.tile0 = (int)g.tiles.size();
        fill();
        r.ntile = (int)g.tiles.size() - r.tile0;
        return r;
    };
    const int depth = t.depth;
    P->g_m2m.assign(depth + 1, GemmRange());
    P->g_up1.assign(depth + 1, GemmRange());
    P->g_up2.assign(depth + 1, GemmRange());
    P->g_dn1.assign(depth + 1, GemmRange());
    P->g_dn2.assign(depth + 1, GemmRange());
    P->g_l2l.assign(depth + 1, GemmRange());
    for (int lv = 0; lv <= depth; ++lv) {
        const int b0 = t.level_start[lv], b1 = t.level_start[lv + 1];
        const double h = std::ldexp(1.0, -lv);
        // M2M into the non-leaf boxes of this level: [M2M_0 | ... | M2M_7] times the stacked
        // densities of the eight children (K blocked by octant), one launch
        P->g_m2m[lv] = range([&] {
            std::vector<int> in, out;
            std::vector<double> sc;
            for (int b = b0; b < b1; ++b) {
                if (t.is_leaf(b)) continue;
                for (int r = 0; r < R; ++r) {
                    for (int o = 0; o < 8; ++o) {
                        int c = t.child[8 * b + o];
                        in.push_back(c < 0 ? -1 : c * R + r);
                    }
                    out.push_back(b * R + r);
                    sc.push_back(1.0 / h);
                }
            }
            add_gemm(g, 0, kn, in, out, sc, 8);
        });
        std::vector<int> cols;
        std::vector<double> one, hs;
        for (int b = b0; b < b1; ++b)
            for (int r = 0; r < R; ++r) {
                cols.push_back(b * R + r);
                one.push_back(1.0);
                hs.push_back(h);
            }
        P->g_up1[lv] = range([&] { add_gemm(g, 0, P->r_up, cols, cols, one); });
        P->g_up2[lv] = range([&] { add_gemm(g, 0, kn, cols, cols, hs); });
        P->g_dn1[lv] = range([&] { add_gemm(g, 0, P->r_dn, cols, cols, one); });
        if (lv == 0 && far_step_d(P)) {   // the roots' far-field densities go to their own block
            std::vector<int> far_cols(cols.size());
            for (size_t i = 0; i < cols.size(); ++i) far_cols[i] = cols[i] - b0 * R + nb * R;
            P->g_dn2[lv] = range([&] { add_gemm(g, 0, kn, cols, far_cols, hs); });
        } else {
            P->g_dn2[lv] = range([&] { add_gemm(g, 0, kn, cols, cols, hs); });
        }
        if (lv >= 1)
            P->g_l2l[lv] = range([&] {
                const double hp = 2.0 * h;
                for (int o = 0; o < 8; ++o) {
                    std::vector<int> in, out;
                    std::vector<double> sc;
                    for (int b = b0; b < b1; ++b) {
                        int par = t.parent[b];
                        if (t.child[8 * par + o] != b) continue;
                        for (int r = 0; r < R; ++r) {
                            in.push_back(par * R + r);
                            out.push_back(b * R + r);
                            sc.push_back(1.0 / hp);
                        }
                    }
                    add_gemm(g, o, kn, in, out, sc);
                }
            });
    }
    P->g_root = range([&] {   // every problem's root
        std::vector<int> c;
        std::vector<double> one;
        for (int b = t.level_start[0]; b < t.level_start[1]; ++b)
            for (int r = 0; r < R; ++r) {
                c.push_back(b * R + r);
                one.push_back(1.0);
            }
        add_gemm(g, 0, kn, c, c, one);
    });
    GemmSet& G = P->gsets[0];
    G.tiles.upload(g.tiles, s);
    G.col_in.upload(g.in, s);
    G.col_out.upload(g.out, s);
    G.col_scale.upload(g.scale, s);

    // workspace
    const size_t cols = (size_t)nb * R;
    P->q_u.ensure(cols * kn);
    P->phi_u.ensure(cols * kn);
    P->q_d.ensure(cols * kn);
    P->q_x.ensure(cols * kn);
    const int n_roots = t.level_start[1] - t.level_start[0];
    P->phi_d.ensure((cols + (far_step_d(P) ? (size_t)n_roots * R : 0)) * kn);
    P->tmp.ensure(cols * kn);
    if (P->cfg.precision == PKIFMM_MIXED) {
        P->phi_oz.ensure((size_t)kOzSlices * cols * oz_padded(kn));
        P->phi_oz_e.ensure(cols);
    }
    P->ds.ensure((size_t)R * P->k * std::max<int64_t>(P->n, 1));
    if (P->cfg.precision == PKIFMM_MIXED) P->ds32.ensure((size_t)R * P->k * std::max<int64_t>(P->n, 1));
    P->pot.ensure((size_t)R * P->k * std::max<int64_t>(P->n, 1));
    P->sums.ensure((size_t)P->n_problems * R * P->k * 2);
    {   // split-K partial tiles: the largest small launch of the tree passes
        int64_t need = 1;
        auto consider = [&](const GemmRange& gr, int K) {
            if (gr.ntile == 0) return;
            need = std::max<int64_t>(need, (int64_t)gr.ntile * gemm_split_factor(gr.ntile, K) * 64 * 64);
        };
        for (int lv = 0; lv <= std::min(depth, kSplitLevels); ++lv) {
            consider(P->g_m2m[lv], 8 * kn);
            consider(P->g_up1[lv], kn); consider(P->g_up2[lv], P->r_up);
            consider(P->g_dn1[lv], kn); consider(P->g_dn2[lv], P->r_dn);
            consider(P->g_l2l[lv], kn);
        }
        consider(P->g_root, kn);
        P->split_need = need;
        P->split_tmp.ensure(need);
    }
    PK_HIP(hipStreamSynchronize(s));
}

// Stage 1b: X-list items (leaf points -> downward check surfaces), set 2.  W/X lists take the
// cheaper form of the interaction: a W-list box that is a leaf with no more points than a
// surface acts through its points, and a leaf with no more points than a surface takes its
// X-list sources directly at its points (both in the near-field items).
void build_stage_x(pkifmm_plan* P) {
    lists_wait(P);
    const HostTree& t = P->tree;
    const HostLists& L = P->lists;
    const int ns = P->n_surf;
    std::vector<Seg> segs;
    std::vector<Work> work;
    auto code = [](const Entry& e) { return (e.sx + 1) * 9 + (e.sy + 1) * 3 + (e.sz + 1); };
    auto small_leaf = [&](int b) { return t.is_leaf(b) && t.end[b] - t.begin[b] <= ns; };
    for (int b = 0; b < t.nbox(); ++b) {
        if (L.x_off[b + 1] == L.x_off[b] || small_leaf(b)) continue;
        int s0 = (int)segs.size();
        for (int64_t e = L.x_off[b]; e < L.x_off[b + 1]; ++e) segs.push_back(Seg{0, L.x[e].src, code(L.x[e])});
        int s1 = (int)segs.size();
        for (int c0 = 0; c0 < ns; c0 += 64) work.push_back(Work{b, 1, c0, std::min(64, ns - c0), s0, s1});
    }
    P->w_x = SegRange{2, 0, (int)work.size()};
    hipStream_t s = P->setup_stream;
    P->segs[2].upload(segs, s);
    P->work[2].upload(work, s);
    PK_HIP(hipStreamSynchronize(s));
}

// Stage 2: the leaf items (near field; W + L2T) and the two-way pair bookkeeping.
void build_stage_near(pkifmm_plan* P, int R) {
    lists_wait(P);
    const HostTree& t = P->tree;
    const HostLists& L = P->lists;
    const int nb = t.nbox();
    const int ns = P->n_surf;
    std::vector<Seg> segs;
    std::vector<Work> work;
    const int kSelf = 13;
    auto code = [](const Entry& e) { return (e.sx + 1) * 9 + (e.sy + 1) * 3 + (e.sz + 1); };
    auto small_leaf = [&](int b) { return t.is_leaf(b) && t.end[b] - t.begin[b] <= ns; };
    // Direct leaf-to-leaf pairs of different leaves are evaluated once when there is one
    // right-hand side: the kernel is symmetric, A in U(B) with shift p exactly when B in U(A)
    // with -p, and a small leaf A taken directly from W(B) is B taken directly from X(A) with
    // -p.  The leaf with more points (then the lower box index) owns the pair and holds the
    // targets; the other leaf's points get their sums through partial slots.
    const bool mutual = R == 1 && !P->separate;
    auto pts_of = [&](int b) { return t.end[b] - t.begin[b]; };
    auto src_of = [&](int b) { return P->box_send[b] - t.begin[b]; };      // sources of a box
    auto trg_of = [&](int b) { return t.end[b] - P->box_tbeg[b]; };        // targets of a leaf
    // is (src, shift code c) in box a's list?  Lists are sorted by (source, shift code).
    auto listed = [&](const std::vector<int64_t>& off, const std::vector<Entry>& v, int a, int s, int c) {
        auto lo = v.begin() + off[a], hi = v.begin() + off[a + 1];
        auto it = std::lower_bound(lo, hi, std::make_pair(s, c), [&](const Entry& e, const std::pair<int, int>& k) {
            return e.src < k.first || (e.src == k.first && code(e) < k.second);
        });
        return it != hi && it->src == s && code(*it) == c;
    };
    // which: 0 U entry, 1 direct W entry, 2 direct X entry of leaf b.  Returns 0: evaluate one
    // way, 1: own the pair, 2: the partner owns it
    auto d_role = [&](int b, const Entry& e, int which) {
        const int a = e.src;
        if (!mutual || a == b) return 0;
        const int mc = 26 - code(e);
        const bool mirrored = which == 0 ? listed(L.u_off, L.u, a, b, mc)
                              : which == 1 ? listed(L.x_off, L.x, a, b, mc)
                                           : listed(L.w_off, L.w, a, b, mc);
        if (!mirrored) return 0;
        const bool own = pts_of(b) > pts_of(a) || (pts_of(b) == pts_of(a) && b < a);
        return own ? 1 : 2;
    };
    int64_t n_slots = 0;
    std::vector<std::vector<int64_t>> incoming(mutual ? nb : 0);
    // near-field items (U lists and the direct W/X entries), one per chunk of up to 512 target
    // points: the leaves are split into contiguous ranges built on separate host threads and
    // concatenated in leaf order, so segments, slots and incoming lists come out exactly as one
    // sequential pass over the leaves would produce them
    auto near_pass = [&](SegRange& out) {
        out.set = 1;
        out.work0 = (int)work.size();
        const int nl = (int)t.leaves.size();
        const int nth = std::max(1, std::min(8, nl / 64));
        struct Part {
            std::vector<Seg> segs;
            std::vector<Work> work;
            std::vector<std::pair<int, int64_t>> inc;   // (other leaf, local slot)
            int64_t slots = 0;
            std::exception_ptr err;
        };
        std::vector<Part> parts(nth);
        auto run = [&](int th) {
            Part& pt = parts[th];
            try {
                const int l0 = (int)((int64_t)nl * th / nth), l1 = (int)((int64_t)nl * (th + 1) / nth);
                std::vector<Seg> near;     // one leaf's direct segments (roles decided once per leaf)
                for (int li = l0; li < l1; ++li) {
                    const int b = t.leaves[li];
                    const int cnt = trg_of(b);
                    if (cnt == 0) continue;
                    near.clear();
                    auto direct = [&](const Entry& en, int which) {
                        if (src_of(en.src) == 0) return;
                        const int role = d_role(b, en, which);
                        if (role != 2) near.push_back(Seg{role == 1 ? 3 : 0, en.src, code(en)});
                    };
                    for (int64_t e = L.u_off[b]; e < L.u_off[b + 1]; ++e) direct(L.u[e], 0);
                    for (int64_t e = L.w_off[b]; e < L.w_off[b + 1]; ++e)
                        if (small_leaf(L.w[e].src)) direct(L.w[e], 1);
                    if (small_leaf(b))
                        for (int64_t e = L.x_off[b]; e < L.x_off[b + 1]; ++e) direct(L.x[e], 2);
                    for (int c0 = 0; c0 < cnt; c0 += 512) {
                        const int tc = std::min(512, cnt - c0);
                        if (c0 > 0 && !mutual) {   // without two-way segments the chunks share one list
                            const Work w0 = pt.work.back();
                            pt.work.push_back(Work{b, 0, P->box_tbeg[b] + c0, tc, w0.seg0, w0.seg1});
                            continue;
                        }
                        const int s0 = (int)pt.segs.size();
                        for (Seg sg : near) {   // every chunk's two-way segments own their slots
                            if (sg.kind == 3) {
                                sg.slot = pt.slots;
                                pt.inc.push_back({sg.box, pt.slots});
                                pt.slots += pts_of(sg.box);
                            }
                            pt.segs.push_back(sg);
                        }
                        pt.work.push_back(Work{b, 0, P->box_tbeg[b] + c0, tc, s0, (int)pt.segs.size()});
                    }
                }
            } catch (...) {
                pt.err = std::current_exception();
            }
        };
        std::vector<std::thread> pool;
        for (int i = 1; i < nth; ++i) pool.emplace_back(run, i);
        run(0);
        for (auto& x : pool) x.join();
        for (Part& pt : parts) {
            if (pt.err) std::rethrow_exception(pt.err);
            const int sb = (int)segs.size();
            const int64_t slb = n_slots;
            for (Seg sg : pt.segs) {
                if (sg.kind == 3) sg.slot += slb;
                segs.push_back(sg);
            }
            for (Work w : pt.work) {
                w.seg0 += sb;
                w.seg1 += sb;
                work.push_back(w);
            }
            for (const auto& pr : pt.inc) incoming[pr.first].push_back(pr.second + slb);
            n_slots += pt.slots;
        }
        out.nwork = (int)work.size() - out.work0;
    };
    // W-list M2T (boxes that are not small leaves) and L2T, in float64 after the near field
    auto far_pass = [&](SegRange& out) {
        out.set = 1;
        out.work0 = (int)work.size();
        for (int b : t.leaves) {
            const int cnt = trg_of(b);
            if (cnt == 0) continue;
            const int s0 = (int)segs.size();
            for (int64_t e = L.w_off[b]; e < L.w_off[b + 1]; ++e)
                if (!small_leaf(L.w[e].src)) segs.push_back(Seg{1, L.w[e].src, code(L.w[e])});
            segs.push_back(Seg{2, b, kSelf});
            if (far_step_d(P)) {   // step d: the root's far-field density, column block nb + root
                int root = b;
                while (t.parent[root] >= 0) root = t.parent[root];
                segs.push_back(Seg{4, root, kSelf, (int64_t)nb + (root - t.level_start[0])});
            }
            const int s1 = (int)segs.size();
            for (int c0 = 0; c0 < cnt; c0 += 512)
                work.push_back(Work{b, 0, P->box_tbeg[b] + c0, std::min(512, cnt - c0), s0, s1});
        }
        out.nwork = (int)work.size() - out.work0;
    };
    near_pass(P->w_leaf_u);
    {   // longest items first, so the near-field kernel ends balanced
        const int w0 = P->w_leaf_u.work0, nw = (int)work.size() - w0;
        std::vector<int64_t> cost(nw);
        for (int i = 0; i < nw; ++i) {
            const Work& w = work[w0 + i];
            int64_t c = 0;
            for (int sg = w.seg0; sg < w.seg1; ++sg)   // a two-way segment costs about 4/3 of a one-way one
                c += (int64_t)src_of(segs[sg].box) * (segs[sg].kind == 3 ? 4 : 3);
            cost[i] = c * (int64_t)w.tcount;
        }
        std::vector<int> order(nw);
        for (int i = 0; i < nw; ++i) order[i] = i;
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost[x] > cost[y]; });
        std::vector<Work> sorted(nw);
        for (int i = 0; i < nw; ++i) sorted[i] = work[w0 + order[i]];
        std::copy(sorted.begin(), sorted.end(), work.begin() + w0);
    }
    far_pass(P->w_leaf_far);
    {   // ordered (target, source) pairs of the near field; a two-way segment counts both ways
        int64_t np = 0;
        for (int i = P->w_leaf_u.work0; i < P->w_leaf_u.work0 + P->w_leaf_u.nwork; ++i)
            for (int sg = work[i].seg0; sg < work[i].seg1; ++sg)
                np += (int64_t)work[i].tcount * src_of(segs[sg].box) * (segs[sg].kind == 3 ? 2 : 1);
        P->stats.near_pairs = np;
    }
    hipStream_t s = P->setup_stream3;
    P->mutual = mutual;
    P->n_slots = n_slots;
    P->n_in = 0;
    if (mutual) {
        std::vector<int> ib;
        std::vector<int64_t> io{0}, is;
        for (int b = 0; b < nb; ++b) {
            if (incoming[b].empty()) continue;
            ib.push_back(b);
            is.insert(is.end(), incoming[b].begin(), incoming[b].end());
            io.push_back((int64_t)is.size());
        }
        P->n_in = (int)ib.size();
        P->in_box.upload(ib, s);
        P->in_off.upload(io, s);
        P->in_slot.upload(is, s);
        P->mpart.ensure((size_t)P->k * std::max<int64_t>(n_slots, 1));
    }
    P->segs[1].upload(segs, s);
    P->work[1].upload(work, s);
    PK_HIP(hipStreamSynchronize(s));
}

// Stage 3: M2L GEMMs grouped by offset.
void build_stage_m2l(pkifmm_plan* P, int R) {
    lists_wait(P);
    const HostTree& t = P->tree;
    const HostLists& L = P->lists;
    const int nb = t.nbox();
    const int kn = P->kn;
    const bool mixed = P->cfg.precision == PKIFMM_MIXED;
    hipStream_t s = P->setup_stream2;
    Gemm g;
    auto range = [&](auto&& fill) {
        GemmRange r;
        r.set = 1;
        r.tile0 = (int)g.tiles.size();
        fill();
        r.ntile = (int)g.tiles.size() - r.tile0;
        return r;
    };
    // M2L grouped by offset; the 316 offsets are split into kM2LGroups fixed groups (by offset
    // index, so the per-target summation order never depends on the batch).  Within a group,
    // output column = the entry's slot in the group (a bounded temporary), summed per target
    // afterwards in entry order; groups are added to q_d one after another.
    {
        // one pass for the offsets, one for the per-group slots, one to lay the columns out by
        // offset (entry order kept within an offset); flat arrays throughout
        const int64_t nv = L.v_off[nb];
        std::vector<int16_t> vidx(nv);
        std::vector<int64_t> per_idx(kNumM2L + 1, 0);
        for (int b = 0; b < nb; ++b) {
            const int side = 1 << t.level[b];
            for (int64_t e = L.v_off[b]; e < L.v_off[b + 1]; ++e) {
                const Entry& v = L.v[e];
                const int idx = m2l_offset_index(t.ix[v.src] + v.sx * side - t.ix[b], t.iy[v.src] + v.sy * side - t.iy[b],
                                                 t.iz[v.src] + v.sz * side - t.iz[b]);
                if (idx < 0) throw Error(PKIFMM_ERR_NUMERICS, "V-list offset out of range");
                vidx[e] = (int16_t)idx;
                ++per_idx[idx + 1];
            }
        }
        for (int d = 0; d < kNumM2L; ++d) per_idx[d + 1] += per_idx[d];
        std::vector<int64_t> goff((size_t)kM2LGroups * (nb + 1), 0);
        std::vector<int> slot_count(kM2LGroups, 0);
        std::vector<std::vector<int>> gtarg(kM2LGroups);
        std::vector<int64_t> pos(per_idx.begin(), per_idx.end() - 1);
        // per entry (laid out by offset): source box, slot in its group, scale; the GEMMs expand
        // each entry into its R right-hand-side columns on the device
        std::vector<int> in_c((size_t)nv), out_c((size_t)nv);
        std::vector<double> sc_c((size_t)nv);
        for (int b = 0; b < nb; ++b) {
            for (int q = 0; q < kM2LGroups; ++q) goff[(size_t)q * (nb + 1) + b] = slot_count[q];
            const double sc = std::ldexp(1.0, t.level[b]);
            for (int64_t e = L.v_off[b]; e < L.v_off[b + 1]; ++e) {
                const int idx = vidx[e];
                const int q = idx * kM2LGroups / kNumM2L;
                const int slot = slot_count[q]++;
                const int64_t p0 = pos[idx]++;
                in_c[p0] = L.v[e].src;
                out_c[p0] = slot;
                sc_c[p0] = sc;
            }
            for (int q = 0; q < kM2LGroups; ++q)
                if (slot_count[q] > goff[(size_t)q * (nb + 1) + b]) gtarg[q].push_back(b);
        }
        for (int q = 0; q < kM2LGroups; ++q) goff[(size_t)q * (nb + 1) + nb] = slot_count[q];
        P->g_m2l.assign(kM2LGroups, GemmRange());
        P->g_m2l_wide.assign(kM2LGroups, GemmRange());
        P->m2l_targets.assign(kM2LGroups, {});
        if ((int64_t)nv * R >= (int64_t)INT32_MAX) throw Error(PKIFMM_ERR_INVALID_ARG, "too many V-list columns");
        g.in = std::move(in_c);
        g.out = std::move(out_c);
        g.scale = std::move(sc_c);
        int max_slots = 1;
        std::vector<int> all_targets;
        for (int q = 0; q < kM2LGroups; ++q) {
            P->g_m2l[q] = range([&] {
                for (int d = 0; d < kNumM2L; ++d) {
                    if (d * kM2LGroups / kNumM2L != q || per_idx[d + 1] == per_idx[d]) continue;
                    const int64_t c0 = per_idx[d] * R, c1 = per_idx[d + 1] * R;   // expanded columns
                    for (int64_t j = c0; j < c1; j += 64)
                        for (int r0 = 0; r0 < kn; r0 += 64)
                            g.tiles.push_back(Tile{d, (int)j, (int)std::min<int64_t>(64, c1 - j), r0});
                }
            });
            if (mixed)     // the int8 GEMM's 128-row tiles: operator, row block, column block
                P->g_m2l_wide[q] = range([&] {
                    for (int d = 0; d < kNumM2L; ++d) {
                        if (d * kM2LGroups / kNumM2L != q || per_idx[d + 1] == per_idx[d]) continue;
                        const int64_t c0 = per_idx[d] * R, c1 = per_idx[d + 1] * R;
                        for (int r0 = 0; r0 < kn; r0 += kOzRows)
                            for (int64_t j = c0; j < c1; j += 64)
                                g.tiles.push_back(Tile{d, (int)j, (int)std::min<int64_t>(64, c1 - j), r0});
                    }
                });
            P->m2l_targets[q] = {(int)all_targets.size(), (int)gtarg[q].size()};
            all_targets.insert(all_targets.end(), gtarg[q].begin(), gtarg[q].end());
            max_slots = std::max(max_slots, slot_count[q]);
        }
        P->v_goff.upload(goff, s);
        P->v_gtargets.upload(all_targets, s);
        P->m2l_slots = max_slots;
    }
    GemmSet& G = P->gsets[1];
    G.tiles.upload(g.tiles, s);
    G.col_in.upload(g.in, s);
    G.col_out.upload(g.out, s);
    G.col_scale.upload(g.scale, s);
    P->m2l_tmp.ensure(std::max<size_t>(1, (size_t)P->m2l_slots * R * kn));
    PK_HIP(hipStreamSynchronize(s));
}

void build_work(pkifmm_plan* P, int R) {
    build_stage_tree(P, R);
    build_stage_x(P);
    build_stage_near(P, R);
    build_stage_m2l(P, R);
    P->R_built = R;
}

void run_gemm(pkifmm_plan* P, const Workspace& w, const GemmRange& gr, const double* ops, int64_t op_stride, int M,
              int K, const double* B, int64_t ldb, double* C, int64_t ldc, bool acc, hipStream_t s, int nkb = 1,
              bool allow_split = true, int rhs = 0) {
    if (gr.ntile == 0) return;
    GemmArgs a{};
    a.ops = ops;
    a.op_stride = op_stride;
    a.M = M;
    a.K = K;
    a.B = B;
    a.ldb = ldb;
    a.C = C;
    a.ldc = ldc;
    const GemmSet& G = P->gsets[gr.set];
    a.tiles = G.tiles.p + gr.tile0;
    a.n_tiles = gr.ntile;
    a.in_col = G.col_in.p;
    a.in_stride = nkb;
    a.kblock = K / nkb;
    a.out_col = G.col_out.p;
    a.scale = G.col_scale.p;
    a.accumulate = acc ? 1 : 0;
    a.rhs = rhs;
    // the per-level launches split K (latency-bound, few tiles); M2L never does
    if (allow_split) launch_gemm(a, s, w.split_tmp, w.split_cap);
    else launch_gemm(a, s);
}

// M2L of the mixed form: the same tiles and column lists on the int8 slices of the operators
// and of the upward densities (sliced once per evaluation, all nbox*R columns)
void run_gemm_oz(pkifmm_plan* P, const Workspace& w, const GemmRange& gr, int R, double* C, int64_t ldc,
                 hipStream_t s, int rows) {
    if (gr.ntile == 0) return;
    const int kp = oz_padded(P->kn);
    OzArgs a{};
    a.a_sl = P->m2l_oz.p;
    a.a_exp = P->m2l_oz_e.p;
    a.Mp = oz_rows_padded(P->kn);
    a.Kp = kp;
    a.M = P->kn;
    a.b_sl = w.phi_oz;
    a.b_exp = w.phi_oz_e;
    a.b_slice_stride = (int64_t)P->tree.nbox() * R * kp;
    a.C = C;
    a.ldc = ldc;
    const GemmSet& G = P->gsets[gr.set];
    a.tiles = G.tiles.p + gr.tile0;
    a.n_tiles = gr.ntile;
    a.in_col = G.col_in.p;
    a.out_col = G.col_out.p;
    a.scale = G.col_scale.p;
    a.rhs = R;
    a.accumulate = 0;
    launch_gemm_oz(a, rows, s);
}

void run_p2p(pkifmm_plan* P, const Workspace& ws, const SegRange& w, double* out_pts, double* out_surf, int R, bool f32,
             bool acc_pts, hipStream_t s, bool to_surface = false, int grid_cap = 0) {
    if (w.nwork == 0) return;
    P2PArgs a{};
    a.kernel = P->cfg.kernel;
    a.n_surf = P->n_surf;
    a.R = R;
    a.n = P->n;
    a.xs = P->xs.p;
    a.ioff = P->ioff.p;
    a.ds = ws.ds;
    a.ds32 = ws.ds32;
    a.phi_u = ws.phi_u;
    a.phi_d = ws.phi_d;
    a.box_level = P->b_level.p;
    a.box_ix = P->b_ix.p;
    a.box_iy = P->b_iy.p;
    a.box_iz = P->b_iz.p;
    a.box_begin = P->b_begin.p;
    a.box_end = P->b_end.p;
    a.box_send = P->b_send.p;
    a.usurf = P->usurf.p;
    a.segs = P->segs[w.set].p;
    a.work = P->work[w.set].p + w.work0;
    a.n_work = w.nwork;
    a.out_pts = out_pts;
    a.out_surf = out_surf;
    a.accumulate_pts = acc_pts ? 1 : 0;
    a.mpart = ws.mpart;
    a.n_slots = P->n_slots;
    a.grid_cap = grid_cap;
    a.rb_max = to_surface ? P->tune.rb_s2m : P->tune.rb_near;
    a.guard_all = P->guard_all ? 1 : 0;
    a.work_counter = nullptr;
    if (grid_cap > 0 && grid_cap < w.nwork)     // cleared before each launch (launch_p2p)
        a.work_counter = reinterpret_cast<unsigned long long*>(ws.counter);
    if (to_surface) launch_p2s(a, s);
    else launch_p2p(a, f32, s);
}

}  // namespace

namespace {

// Point a plan-backed workspace at the plan's buffers, part by part: the M2L temporary and the
// near-field partial slots are sized by the build stages on other host threads, and are read
// only after those threads have been joined.
enum WsPart { kWsTree, kWsM2L, kWsNear };
void bind_plan_workspace(pkifmm_plan* P, Workspace& w, WsPart part) {
    if (!w.from_plan) return;
    if (part == kWsM2L) {
        w.m2l_tmp = P->m2l_tmp.p;
        return;
    }
    if (part == kWsNear) {
        w.mpart = P->mpart.p;
        return;
    }
    w.ds = P->ds.p;
    w.ds32 = P->ds32.p;
    w.pot = P->pot.p;
    w.q_u = P->q_u.p;
    w.phi_u = P->phi_u.p;
    w.q_d = P->q_d.p;
    w.q_x = P->q_x.p;
    w.phi_d = P->phi_d.p;
    w.tmp = P->tmp.p;
    w.split_tmp = P->split_tmp.p;
    w.split_cap = (int64_t)P->split_tmp.n;
    w.sums = P->sums.p;
    w.counter = P->counter.p;
    w.phi_oz = P->phi_oz.p;
    w.phi_oz_e = P->phi_oz_e.p;
}

// The same workspace as regions of one array at `base` (each 256-byte aligned), sized exactly as
// the plan's buffers for the current work lists and n_rhs R, so that every kernel takes the same
// path (split-K factors included) and the results are the same bits.  Returns the bytes needed;
// with base == nullptr only counts them.  The neutrality sums are not placed (no checks there).
size_t carve_workspace(const pkifmm_plan* P, int R, char* base, Workspace& w) {
    const bool mixed = P->cfg.precision == PKIFMM_MIXED;
    const size_t cols = (size_t)P->tree.nbox() * R, kn = (size_t)P->kn;
    const size_t npts = (size_t)R * P->k * std::max<int64_t>(P->n, 1);
    const int n_roots = P->tree.level_start[1] - P->tree.level_start[0];
    size_t off = 0;
    auto take = [&](auto*& ptr, size_t count) {
        using T = std::remove_pointer_t<std::remove_reference_t<decltype(ptr)>>;
        const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
        ptr = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += (bytes + 255) / 256 * 256;
    };
    w.from_plan = false;
    take(w.ds, npts);
    if (mixed) take(w.ds32, npts);
    else w.ds32 = nullptr;
    take(w.pot, npts);
    take(w.q_u, cols * kn);
    take(w.phi_u, cols * kn);
    take(w.q_d, cols * kn);
    take(w.q_x, cols * kn);
    take(w.phi_d, (cols + (far_step_d(P) ? (size_t)n_roots * R : 0)) * kn);
    take(w.tmp, cols * kn);
    take(w.m2l_tmp, (size_t)P->m2l_slots * R * kn);
    take(w.split_tmp, (size_t)P->split_need);
    w.split_cap = P->split_need;
    if (P->mutual) take(w.mpart, (size_t)P->k * std::max<int64_t>(P->n_slots, 1));
    else w.mpart = nullptr;
    take(w.counter, 1);
    if (mixed) {
        take(w.phi_oz, (size_t)kOzSlices * cols * oz_padded(P->kn));
        take(w.phi_oz_e, cols);
    } else {
        w.phi_oz = nullptr;
        w.phi_oz_e = nullptr;
    }
    w.sums = nullptr;
    return off;
}

// Tuning files: one record per line, "arch kernel mask p precision n_rhs near_wpc rb_near rb_s2m
// m2l_rows" (a record without m2l_rows takes 64); '#' starts a comment.  A missing file is empty;
// a malformed line is skipped.
struct TuneLine {
    std::string arch;
    int kernel = 0;
    unsigned mask = 0;
    int p = 0, precision = 0, R = 0;
    Tuning t;
};

std::vector<TuneLine> read_tuning_file(const char* path) {
    std::vector<TuneLine> out;
    FILE* f = std::fopen(path, "r");
    if (!f) return out;
    char line[512];
    while (std::fgets(line, sizeof(line), f)) {
        if (char* c = std::strchr(line, '#')) *c = 0;
        char arch[64];
        TuneLine l;
        const int nf = std::sscanf(line, "%63s %d %u %d %d %d %d %d %d %d", arch, &l.kernel, &l.mask, &l.p,
                                   &l.precision, &l.R, &l.t.near_wpc, &l.t.rb_near, &l.t.rb_s2m, &l.t.m2l_rows);
        if ((nf == 9 || nf == 10) && l.R >= 1 && l.t.near_wpc >= 1 && l.t.near_wpc <= 16 && l.t.rb_near >= 0 &&
            l.t.rb_s2m >= 0 && (l.t.m2l_rows == 64 || l.t.m2l_rows == kOzRows)) {
            l.arch = arch;
            out.push_back(l);
        }
    }
    std::fclose(f);
    return out;
}

// replaces the record of the same key (arch, kernel, mask, p, precision, n_rhs) or adds it
bool write_tuning_record(const char* path, const TuneLine& rec) {
    std::vector<TuneLine> lines = read_tuning_file(path);
    bool done = false;
    for (TuneLine& l : lines)
        if (l.arch == rec.arch && l.kernel == rec.kernel && l.mask == rec.mask && l.p == rec.p &&
            l.precision == rec.precision && l.R == rec.R) {
            l = rec;
            done = true;
        }
    if (!done) lines.push_back(rec);
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "w");
    if (!f) return false;
    std::fprintf(f, "# arch kernel mask p precision n_rhs near_wpc rb_near rb_s2m m2l_rows (pkifmm_autotune)\n");
    for (const TuneLine& l : lines)
        std::fprintf(f, "%s %d %u %d %d %d %d %d %d %d\n", l.arch.c_str(), l.kernel, l.mask, l.p, l.precision, l.R,
                     l.t.near_wpc, l.t.rb_near, l.t.rb_s2m, l.t.m2l_rows);
    const bool ok = std::fclose(f) == 0;
    return ok && std::rename(tmp.c_str(), path) == 0;
}

// Wait until the last evaluation enqueued (on any stream) has finished: work lists, workspace and
// point buffers are rewritten or reallocated only after that.
void wait_idle(pkifmm_plan* P) { PK_HIP(hipEventSynchronize(P->ev_done)); }

void drop_graph(pkifmm_plan* P) {
    if (P->gexec) (void)hipGraphExecDestroy(P->gexec);
    if (P->graph) (void)hipGraphDestroy(P->graph);
    P->gexec = nullptr;
    P->graph = nullptr;
}

// A host thread building one stage's work lists on the caller's device.  join() rethrows what
// the stage threw; the destructor joins (errors then dropped), so an exception elsewhere never
// leaves the thread running.
class StageThread {
  public:
    template <class F>
    void start(F f) {
        int dev = 0;
        PK_HIP(hipGetDevice(&dev));
        const Allocator* al = g_alloc;
        th_ = std::thread([this, f, dev, al] {
            AllocScope scope(al);      // buffers sized here come from the caller's allocator too
            try {
                PK_HIP(hipSetDevice(dev));
                f();
            } catch (...) {
                err_ = std::current_exception();
            }
        });
    }
    void join() {
        if (th_.joinable()) th_.join();
        if (err_) {
            std::exception_ptr e = err_;
            err_ = nullptr;
            std::rethrow_exception(e);
        }
    }
    ~StageThread() {
        if (th_.joinable()) th_.join();
    }

  private:
    std::thread th_;
    std::exception_ptr err_;
};

// Enqueue one evaluation on stream s (no host synchronisation unless `checks`).
// The workspace comes from the plan (w.from_plan: its buffers, bound after each build stage that
// sizes them) or is given (the static array).
void enqueue_evaluate(pkifmm_plan* P, Workspace& w, int R, const double* density, double* potential, hipStream_t s,
                      bool checks, bool allow_timing, bool build = false) {
        if (!P->tune_fixed) {   // the tuned choices for this n_rhs, else the defaults
            P->tune = Tuning();
            for (const TuneRec& rec : P->tune_table)
                if (rec.R == R) P->tune = rec.t;
        }
        const int64_t n = P->n;
        const int k = P->k, kn = P->kn;
        const HostTree& t = P->tree;
        const bool mixed = P->cfg.precision == PKIFMM_MIXED;
        const bool timing = allow_timing && (P->cfg.flags & PKIFMM_PHASE_TIMING) != 0;
        std::vector<hipEvent_t> ev;
        auto mark_on = [&](hipStream_t st) {
            if (!timing) return;
            hipEvent_t e;
            PK_HIP(hipEventCreate(&e));
            PK_HIP(hipEventRecord(e, st));
            ev.push_back(e);
        };
        auto mark = [&]() { mark_on(s); };
        // first evaluation on new points: the M2L and near-field work lists are built on two
        // host threads (their own upload streams) while this thread builds the tree-pass lists
        // and enqueues the upward pass; each is joined just before its kernels are enqueued.  The
        // upward pass needs the tree alone, so it is enqueued before the host lists (still being
        // built by the thread set_points started) are waited for.
        StageThread th_m2l, th_near;
        if (build) {
            th_m2l.start([P, R] { build_stage_m2l(P, R); });
            th_near.start([P, R] { build_stage_near(P, R); });
            build_stage_tree(P, R);
        }
        bind_plan_workspace(P, w, kWsTree);
        if (!build) {
            bind_plan_workspace(P, w, kWsM2L);
            bind_plan_workspace(P, w, kWsNear);
        }
        launch_permute_density(density, P->perm.p, n, P->n_src, R, k, w.ds, mixed ? w.ds32 : nullptr, s);
        const int naxes = __builtin_popcount(P->cfg.periodic_mask);
        if (checks && (naxes == 1 || naxes == 2) && !(P->cfg.flags & PKIFMM_SKIP_CHECKS)) {
            // zero net density (Section 2, the compatibility condition), relative to the density's
            // magnitude so that the test does not depend on its scale: |sum phi| <= 1e-12 sum |phi|
            // per problem, right-hand side and component
            const int np = P->n_problems;
            std::vector<double> sums((size_t)np * R * k * 2);
            launch_density_sums(w.ds, n, R, k, P->prob_off.p, np, w.sums, s);
            PK_HIP(hipMemcpyAsync(sums.data(), w.sums, sizeof(double) * sums.size(), hipMemcpyDeviceToHost, s));
            PK_HIP(hipStreamSynchronize(s));
            for (size_t i = 0; i < sums.size(); i += 2)
                if (!(std::fabs(sums[i]) <= kNeutralRel * sums[i + 1]))
                    throw Error(PKIFMM_ERR_INCOMPATIBLE, "singly and doubly periodic input needs a zero net density");
        }
        const size_t cols = (size_t)t.nbox() * R;
        const int64_t kk = (int64_t)kn * kn;
        // Schedule.  Matrix-core GEMMs slow down many times over when they share compute units
        // with the direct sums, so the GEMM passes are placed where the chip is otherwise idle:
        // the upward pass and M2L run first (while the host builds the near-field lists), the
        // near field then starts on a second stream and M2L finishes in its tail, and the
        // downward pass runs after both.  The X list (a few long, latency-bound work items) runs
        // on a third stream into its own buffer.
        // 2. S2M and the upward pass; X list beside them
        mark();
        launch_fill_zero(w.q_u, (int64_t)cols * kn, s);     // kernels, not memset nodes (graph-safe)
        launch_fill_zero(w.q_d, (int64_t)cols * kn, s);
        launch_fill_zero(w.q_x, (int64_t)cols * kn, s);
        if (far_step_d(P))   // the roots hand no far field down the tree
            launch_fill_zero(w.phi_d + (size_t)t.level_start[0] * R * kn,
                             (int64_t)(t.level_start[1] - t.level_start[0]) * R * kn, s);
        run_p2p(P, w, P->w_s2m, nullptr, w.q_u, R, false, false, s, true);
        hipStream_t sx = P->x_stream, sn = P->near_stream;
        PK_HIP(hipEventRecord(P->ev_fork, s));
        for (int lv = t.depth; lv >= 0; --lv) {
            const bool split = lv <= kSplitLevels;
            run_gemm(P, w, P->g_m2m[lv], P->m2m.p, 0, kn, 8 * kn, w.phi_u, kn, w.q_u, kn, true, s, 8, split);
            run_gemm(P, w, P->g_up1[lv], P->up_Ut.p, 0, P->r_up, kn, w.q_u, kn, w.tmp, kn, false, s, 1, split);
            run_gemm(P, w, P->g_up2[lv], P->up_VS.p, 0, kn, P->r_up, w.tmp, kn, w.phi_u, kn, false, s, 1, split);
        }
        mark();
        if (build) build_stage_x(P);
        PK_HIP(hipStreamWaitEvent(sx, P->ev_fork, 0));
        run_p2p(P, w, P->w_x, nullptr, w.q_x, R, false, false, sx, true);
        PK_HIP(hipEventRecord(P->ev_xjoin, sx));
        // 3. root far field and V-list M2L into the downward check potentials
        th_m2l.join();                          // built while the upward pass was enqueued and ran
        bind_plan_workspace(P, w, kWsM2L);
        run_gemm(P, w, P->g_root, P->mroot.p, 0, kn, kn, w.phi_u, kn, w.q_d, kn, true, s);
        if (mixed) launch_oz_slice_columns(w.phi_u, kn, kn, (int64_t)cols, w.phi_oz, w.phi_oz_e, s);
        for (int q = 0; q < kM2LGroups; ++q) {
            if (P->g_m2l[q].ntile == 0) continue;
            if (mixed)
                run_gemm_oz(P, w, P->tune.m2l_rows == kOzRows ? P->g_m2l_wide[q] : P->g_m2l[q], R, w.m2l_tmp, kn, s,
                            P->tune.m2l_rows == kOzRows ? kOzRows : 64);
            else
                run_gemm(P, w, P->g_m2l[q], P->m2l.p, kk, kn, kn, w.phi_u, kn, w.m2l_tmp, kn, false, s, 1, false, R);
            launch_segment_reduce(w.m2l_tmp, P->v_goff.p + (size_t)q * (t.nbox() + 1),
                                  P->v_gtargets.p + P->m2l_targets[q].first, P->m2l_targets[q].second, R, kn,
                                  w.q_d, s);
        }
        mark();
        // 4. near field (U lists and the direct W/X entries) on the second stream; it needs only
        // the permuted densities
        th_near.join();
        bind_plan_workspace(P, w, kWsNear);
        PK_HIP(hipStreamWaitEvent(sn, P->ev_fork, 0));
        mark_on(sn);
        run_p2p(P, w, P->w_leaf_u, w.pot, nullptr, R, mixed, false, sn, false, P->tune.near_wpc * P->n_cu);
        if (P->mutual)
            launch_mutual_gather(w.mpart, P->n_slots, k, P->in_box.p, P->in_off.p, P->in_slot.p, P->n_in,
                                 P->b_begin.p, P->b_end.p, n, w.pot, sn);
        mark_on(sn);
        PK_HIP(hipEventRecord(P->ev_join, sn));
        // 5. after the near field and the X list: X-list check potentials join, then the
        // downward pass with the whole chip
        PK_HIP(hipStreamWaitEvent(s, P->ev_join, 0));
        PK_HIP(hipStreamWaitEvent(s, P->ev_xjoin, 0));
        launch_add_into(w.q_d, w.q_x, (int64_t)cols * kn, s);
        for (int lv = 0; lv <= t.depth; ++lv) {
            const bool split = lv <= kSplitLevels;
            if (lv >= 1)
                run_gemm(P, w, P->g_l2l[lv], P->l2l.p, kk, kn, kn, w.phi_d, kn, w.q_d, kn, true, s, 1, split);
            run_gemm(P, w, P->g_dn1[lv], P->dn_Ut.p, 0, P->r_dn, kn, w.q_d, kn, w.tmp, kn, false, s, 1, split);
            run_gemm(P, w, P->g_dn2[lv], P->dn_VS.p, 0, kn, P->r_dn, w.tmp, kn, w.phi_d, kn, false, s, 1, split);
        }
        mark();
        // 6. W list and L2T (float64: they consume equivalent densities)
        run_p2p(P, w, P->w_leaf_far, w.pot, nullptr, R, false, true, s);
        if (P->cfg.kernel == PKIFMM_LAPLACE && P->cfg.periodic_mask == 7u)   // the zero-mean sum's background
            launch_tp_background(w.ds, P->xs.p, n, P->prob_off.p, P->n_problems, w.phi_u, R, P->usurf.p, P->n_surf,
                                 w.pot, s);
        // 7. output
        const double c = (P->cfg.kernel == PKIFMM_LAPLACE ? 1.0 / (4.0 * M_PI) : 1.0 / (8.0 * M_PI)) / P->cfg.box_length;
        launch_unpermute(w.pot, P->perm.p, n, P->t_first, P->n_out, R, k, c, potential, s);
        mark();
        if (!P->capturing) PK_HIP(hipEventRecord(P->ev_done, s));
        if (timing) P->pending_events.push_back(ev);
        if (build) P->R_built = R;
}

}  // namespace

extern "C" {

int pkifmm_config_default(pkifmm_config* c) {
    if (!c) return PKIFMM_ERR_INVALID_ARG;
    std::memset(c, 0, sizeof(*c));
    c->kernel = PKIFMM_LAPLACE;
    c->periodic_mask = 0;
    c->p = 8;
    c->max_pts_per_leaf = 64;
    c->precision = PKIFMM_FP64;
    c->box_length = 1.0;
    c->svd_rel_threshold = 0.0;
    c->flags = 0;
    return PKIFMM_OK;
}

int pkifmm_plan_create(const pkifmm_config* cfg, pkifmm_plan** out) {
    if (!cfg || !out) return PKIFMM_ERR_INVALID_ARG;
    *out = nullptr;
    std::unique_ptr<pkifmm_plan> P(new pkifmm_plan());
    rocblas_handle h = nullptr;
    P->allocator.ctx = cfg->alloc_ctx;
    P->allocator.alloc = cfg->alloc;
    P->allocator.free = cfg->free;
    AllocScope scope(&P->allocator);
    try {
        check_config(*cfg);
        P->cfg = *cfg;
        P->cfg.operator_cache_dir = nullptr;   // the caller's string is read here only
        P->k = cfg->kernel == PKIFMM_LAPLACE ? 1 : 3;
        const int p = cfg->p;
        std::vector<double> u = unit_surface(p);
        P->n_surf = (int)u.size() / 3;
        P->kn = P->k * P->n_surf;
        const int kn = P->kn, ns = P->n_surf;
        // non-blocking: the uploads of one stage must not wait for the kernels of the previous
        // stage on the caller's stream (a legacy default stream would otherwise order them)
        PK_HIP(hipStreamCreateWithFlags(&P->setup_stream, hipStreamNonBlocking));
        PK_HIP(hipStreamCreateWithFlags(&P->setup_stream2, hipStreamNonBlocking));
        PK_HIP(hipStreamCreateWithFlags(&P->setup_stream3, hipStreamNonBlocking));
        // non-blocking: no implicit synchronisation with the legacy null stream; default priority
        PK_HIP(hipStreamCreateWithFlags(&P->near_stream, hipStreamNonBlocking));
        PK_HIP(hipStreamCreateWithFlags(&P->x_stream, hipStreamNonBlocking));
        PK_HIP(hipStreamCreateWithFlags(&P->capture_stream, hipStreamNonBlocking));
        PK_HIP(hipEventCreateWithFlags(&P->ev_fork, hipEventDisableTiming));
        PK_HIP(hipEventCreateWithFlags(&P->ev_join, hipEventDisableTiming));
        PK_HIP(hipEventCreateWithFlags(&P->ev_xjoin, hipEventDisableTiming));
        PK_HIP(hipEventCreateWithFlags(&P->ev_done, hipEventDisableTiming));
        hipStream_t s = P->setup_stream;
        {
            int dev = 0;
            PK_HIP(hipGetDevice(&dev));
            PK_HIP(hipDeviceGetAttribute(&P->n_cu, hipDeviceAttributeMultiprocessorCount, dev));
            P->dev = dev;
            P->scratch_base = scratch_address(dev);   // once per device, this device current
            // near field: a few workgroups per compute unit (Tuning::near_wpc) take items from a
            // counter in list (longest-first) order
            P->counter.ensure(1);
            hipDeviceProp_t prop;
            PK_HIP(hipGetDeviceProperties(&prop, dev));
            P->arch = prop.gcnArchName;
            P->arch = P->arch.substr(0, P->arch.find(':'));
        }
        if (rocblas_create_handle(&h) != rocblas_status_success) throw Error(PKIFMM_ERR_HIP, "rocblas handle");
        rocblas_set_stream(h, s);
        P->usurf.upload(u, s);
        const auto inner = scaled(u, kInnerHalf, 0, 0, 0), outer = scaled(u, kOuterHalf, 0, 0, 0);
        DBuf<double> d_in, d_out, d_tmp, A;
        d_in.upload(inner, s);
        d_out.upload(outer, s);
        A.ensure((size_t)kn * kn);
        double thr = cfg->svd_rel_threshold;
        if (thr == 0.0) thr = kDefaultSvdCut;
        // the solve factors and the root operator from the operator cache, when one is given and
        // holds them; a file that fails its checks is an error, not silently rebuilt
        std::string cache_file;
        OpBlob blob;
        bool cached = false;
        if (cfg->operator_cache_dir && cfg->operator_cache_dir[0]) {
            cache_file = opcache_path(cfg->operator_cache_dir, cfg->kernel, cfg->periodic_mask, p, thr,
                                      near_layers(*cfg));
            const int st = opcache_read(cache_file, &blob);
            if (st == PKIFMM_ERR_CACHE_CORRUPT ||
                (st == PKIFMM_OK && (blob.kernel != cfg->kernel || blob.mask != cfg->periodic_mask || blob.p != p ||
                                     blob.kn != kn || blob.cutoff != thr || blob.near_layers != near_layers(*cfg))))
                throw Error(PKIFMM_ERR_CACHE_CORRUPT, "operator cache file failed its checks: " + cache_file);
            cached = st == PKIFMM_OK;
        }
        double smax_up = 0.0, smax_dn = 0.0;
        // upward: check = outer, equivalent = inner;  downward: check = inner, equivalent = outer
        launch_kmat(cfg->kernel, d_out.p, ns, d_in.p, ns, A.p, kn, s);
        if (cached) {
            P->r_up = blob.r_up;
            P->f_up_Ut = blob.up_Ut;
            P->f_up_VS = blob.up_VS;
            P->up_Ut.upload(P->f_up_Ut, s);
            P->up_VS.upload(P->f_up_VS, s);
            PK_HIP(hipStreamSynchronize(s));
            check_solve(A.p, kn, P->r_up, P->f_up_Ut, P->f_up_VS, blob.smax_up);
        } else {
            P->r_up = pinv_build(h, s, A.p, kn, thr, P->up_Ut, P->up_VS, P->f_up_Ut, P->f_up_VS, &smax_up);
        }
        launch_kmat(cfg->kernel, d_in.p, ns, d_out.p, ns, A.p, kn, s);
        if (cached) {
            P->r_dn = blob.r_dn;
            P->f_dn_Ut = blob.dn_Ut;
            P->f_dn_VS = blob.dn_VS;
            P->dn_Ut.upload(P->f_dn_Ut, s);
            P->dn_VS.upload(P->f_dn_VS, s);
            PK_HIP(hipStreamSynchronize(s));
            check_solve(A.p, kn, P->r_dn, P->f_dn_Ut, P->f_dn_VS, blob.smax_dn);
        } else {
            P->r_dn = pinv_build(h, s, A.p, kn, thr, P->dn_Ut, P->dn_VS, P->f_dn_Ut, P->f_dn_VS, &smax_dn);
        }
        // M2M / L2L: parent edge 1 centred at 0, child o centred at +-1/4
        P->m2m.ensure((size_t)8 * kn * kn);
        P->l2l.ensure((size_t)8 * kn * kn);
        for (int o = 0; o < 8; ++o) {
            double cx = ((o >> 2) & 1) ? 0.25 : -0.25, cy = ((o >> 1) & 1) ? 0.25 : -0.25, cz = (o & 1) ? 0.25 : -0.25;
            d_tmp.upload(scaled(u, 0.5 * kInnerHalf, cx, cy, cz), s);
            launch_kmat(cfg->kernel, d_out.p, ns, d_tmp.p, ns, P->m2m.p + (size_t)o * kn * kn, kn, s);
            launch_kmat(cfg->kernel, d_tmp.p, ns, d_out.p, ns, P->l2l.p + (size_t)o * kn * kn, kn, s);
            PK_HIP(hipStreamSynchronize(s));
        }
        // M2L: target box centred at 0, source box centred at delta, both edge 1
        P->m2l.ensure((size_t)kNumM2L * kn * kn);
        for (int d = 0; d < kNumM2L; ++d) {
            int dx, dy, dz;
            m2l_offset_vector(d, dx, dy, dz);
            d_tmp.upload(scaled(u, kInnerHalf, dx, dy, dz), s);
            launch_kmat(cfg->kernel, d_in.p, ns, d_tmp.p, ns, P->m2l.p + (size_t)d * kn * kn, kn, s);
            PK_HIP(hipStreamSynchronize(s));
        }
        // root far field: K^{P,F}(x^{B0,d}, y^{B0,u}), both the 1.05 cube of the unit box
        P->mroot.ensure((size_t)kn * kn);
        if (cached) {
            P->mroot.upload(blob.mroot, s);
        } else if (cfg->periodic_mask == 0) {
            PK_HIP(hipMemsetAsync(P->mroot.p, 0, sizeof(double) * kn * kn, s));
        } else {
            d_tmp.upload(scaled(u, kInnerHalf, 0.5, 0.5, 0.5), s);
            launch_far_kmat(cfg->kernel, cfg->periodic_mask, d_tmp.p, ns, d_tmp.p, ns, P->mroot.p, kn,
                            near_layers(P->cfg), s);
        }
        if (!cache_file.empty() && !cached) {   // store what was built (a failed write leaves no file)
            OpBlob b;
            b.kernel = cfg->kernel;
            b.mask = cfg->periodic_mask;
            b.p = p;
            b.kn = kn;
            b.r_up = P->r_up;
            b.r_dn = P->r_dn;
            b.cutoff = thr;
            b.near_layers = near_layers(*cfg);
            b.smax_up = smax_up;
            b.smax_dn = smax_dn;
            b.up_Ut = P->f_up_Ut;
            b.up_VS = P->f_up_VS;
            b.dn_Ut = P->f_dn_Ut;
            b.dn_VS = P->f_dn_VS;
            b.mroot.resize((size_t)kn * kn);
            PK_HIP(hipMemcpyAsync(b.mroot.data(), P->mroot.p, sizeof(double) * kn * kn, hipMemcpyDeviceToHost, s));
            PK_HIP(hipStreamSynchronize(s));
            opcache_write(cache_file, b);
        }
        if (cfg->precision == PKIFMM_MIXED) {   // M2L of the mixed form runs on int8 slices
            const int kp = oz_padded(kn), mp = oz_rows_padded(kn);
            P->m2l_oz.ensure((size_t)kNumM2L * kOzSlices * mp * kp);
            P->m2l_oz_e.ensure((size_t)kNumM2L * mp);
            launch_oz_slice_operators(P->m2l.p, kNumM2L, kn, kn, P->m2l_oz.p, P->m2l_oz_e.p, s);
        }
        P->err_flag.ensure(2);
        if (cfg->tuning_file && cfg->tuning_file[0])
            for (const TuneLine& l : read_tuning_file(cfg->tuning_file))
                if (l.arch == P->arch && l.kernel == cfg->kernel && l.mask == cfg->periodic_mask && l.p == p &&
                    l.precision == cfg->precision)
                    P->tune_table.push_back(TuneRec{l.R, l.t});
        P->cfg.tuning_file = nullptr;
        PK_HIP(hipStreamSynchronize(s));
        rocblas_destroy_handle(h);
        h = nullptr;
        P->stats.svd_rank_up = P->r_up;
        P->stats.svd_rank_down = P->r_dn;
    } catch (const Error& e) {
        if (h) rocblas_destroy_handle(h);
        if (P->setup_stream) (void)hipStreamDestroy(P->setup_stream);
        if (P->setup_stream2) (void)hipStreamDestroy(P->setup_stream2);
        if (P->setup_stream3) (void)hipStreamDestroy(P->setup_stream3);
        if (P->near_stream) (void)hipStreamDestroy(P->near_stream);
        if (P->x_stream) (void)hipStreamDestroy(P->x_stream);
        if (P->capture_stream) (void)hipStreamDestroy(P->capture_stream);
        if (P->ev_fork) (void)hipEventDestroy(P->ev_fork);
        if (P->ev_join) (void)hipEventDestroy(P->ev_join);
        if (P->ev_xjoin) (void)hipEventDestroy(P->ev_xjoin);
        if (P->ev_done) (void)hipEventDestroy(P->ev_done);
        return e.code;
    } catch (const std::bad_alloc&) {
        if (h) rocblas_destroy_handle(h);
        return PKIFMM_ERR_OOM;
    }
    *out = P.release();
    return PKIFMM_OK;
}

}  // extern "C"

namespace {

// Point set-up of one problem (with separate targets when trg != nullptr) or of a batch.
int set_points_impl(pkifmm_plan* P, int n_problems, const int64_t* counts, const double* xyz, int64_t n_trg,
                    const double* trg, void* stream) {
    if (!P) return PKIFMM_ERR_INVALID_ARG;
    if (n_problems < 1 || !counts) return fail(P, Error(PKIFMM_ERR_INVALID_ARG, "n_problems or counts"));
    std::vector<int64_t> poff(n_problems + 1, 0);
    for (int i = 0; i < n_problems; ++i) {
        if (counts[i] < 0) return fail(P, Error(PKIFMM_ERR_INVALID_ARG, "negative count"));
        poff[i + 1] = poff[i] + counts[i];
    }
    const bool separate = trg != nullptr;
    if (n_trg < 0 || (!separate && n_trg != 0) || (separate && n_problems != 1))
        return fail(P, Error(PKIFMM_ERR_INVALID_ARG, "n_trg or trg_xyz"));
    const int64_t n_src = poff[n_problems];
    if (separate) poff[1] += n_trg;      // one problem: the union of sources and targets
    const int64_t n = poff[n_problems];
    if (n > (int64_t)INT32_MAX || (n_src > 0 && !xyz)) return fail(P, Error(PKIFMM_ERR_INVALID_ARG, "n or xyz"));
    auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = (hipStream_t)stream;
    P->allocator.stream = stream;
    AllocScope scope(&P->allocator);
    try {
        lists_settle(P);
        wait_idle(P);   // an evaluation in flight still reads the current points and lists
        P->have_points = false;
        P->R_built = -1;
        ++P->generation;
        drop_graph(P);
        P->separate = separate;
        P->n_src = n_src;
        P->t_first = separate ? n_src : 0;
        P->n_out = separate ? n_trg : n;
        if (separate && n > 0) {   // the union, sources first (input indices [0, n_src))
            P->xyz_union.ensure((size_t)3 * n);
            if (n_src) PK_HIP(hipMemcpyAsync(P->xyz_union.p, xyz, sizeof(double) * 3 * n_src, hipMemcpyDeviceToDevice, s));
            if (n_trg)
                PK_HIP(hipMemcpyAsync(P->xyz_union.p + 3 * n_src, trg, sizeof(double) * 3 * n_trg,
                                      hipMemcpyDeviceToDevice, s));
            xyz = P->xyz_union.p;
        }
        P->n = n;
        P->n_problems = n_problems;
        P->prob_off_h = poff;
        P->prob_off.upload(poff, s);
        const size_t m = std::max<int64_t>(n, 1);
        P->keys_a.ensure(m);
        P->keys_b.ensure(m);
        P->vals_a.ensure(m);
        P->perm.ensure(m);
        P->u_wrapped.ensure(3 * m);
        P->xs.ensure(3 * m);
        PK_HIP(hipMemsetAsync(P->err_flag.p, 0, 2 * sizeof(int), s));
        launch_keys(xyz, n, P->cfg.box_length, P->cfg.periodic_mask, P->keys_a.p, P->vals_a.p, P->u_wrapped.p,
                    P->err_flag.p, s);
        // each problem's points are sorted on their own (segmented sort for a batch)
        radix_sort_pairs(P->keys_a.p, P->keys_b.p, P->vals_a.p, P->perm.p, n, P->sort_temp, s, n_problems,
                         P->prob_off.p);
        launch_gather_points(P->u_wrapped.p, P->perm.p, n, P->xs.p, s);
        if (P->cfg.precision == PKIFMM_MIXED)   // are zero separations possible outside a leaf's own segment?
            launch_close_pairs(P->keys_b.p, P->xs.p, n, P->prob_off.p, n_problems, P->cfg.periodic_mask, kCloseDelta,
                               P->err_flag.p + 1, s);
        int err[2] = {0, 0};
        PK_HIP(hipMemcpyAsync(err, P->err_flag.p, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
        const uint64_t* keys = nullptr;
        if (n_problems > 1) {   // the forest is built on the host, one problem per thread
            P->keys_host.ensure(m);
            keys = P->keys_host.p;
            if (n) PK_HIP(hipMemcpyAsync(P->keys_host.p, P->keys_b.p, sizeof(uint64_t) * n, hipMemcpyDeviceToHost, s));
        }
        PK_HIP(hipStreamSynchronize(s));
        if (err[0]) throw Error(PKIFMM_ERR_OUT_OF_BOX, "coordinate outside the box on a non-periodic axis, or not finite");
        P->guard_all = err[1] != 0;
        P->stats.close_points = P->guard_all ? 1 : 0;
        if (n_problems == 1) {
            build_tree_device(P, P->keys_b.p, n, P->cfg.max_pts_per_leaf, P->tree, s);
            P->box_prob.assign(P->tree.nbox(), 0);     // the lists follow below, on a host thread
        } else {
            std::vector<HostTree> trees;
            std::vector<HostLists> lists;
            build_forest_host(keys, poff, P->cfg.max_pts_per_leaf, P->cfg.periodic_mask, near_layers(P->cfg), trees,
                              lists);
            merge_forest(trees, lists, poff, P->tree, P->lists, P->box_prob);
        }
        const HostTree& t = P->tree;
        P->box_send = t.end;
        P->box_tbeg = t.begin;
        if (separate && n > 0) {
            // every leaf's sources first, then its targets, each in (key, index) order: a stable sort
            // of the sorted points by (leaf begin, is target); then the leaves' source counts
            const int nl = (int)t.leaves.size();
            P->leaf_boxes.upload(t.leaves, s);
            P->b_begin.upload(t.begin, s);
            P->b_end.upload(t.end, s);
            P->leaf_nsrc.ensure(nl);
            P->leaf_nsrc_host.ensure(nl);
            launch_role_keys(P->leaf_boxes.p, nl, P->b_begin.p, P->b_end.p, P->perm.p, n_src, P->keys_a.p,
                             P->leaf_nsrc.p, s);
            radix_sort_pairs(P->keys_a.p, P->keys_b.p, P->perm.p, P->vals_a.p, n, P->sort_temp, s, 1, nullptr, 33);
            P->perm.swap(P->vals_a);
            launch_gather_points(P->u_wrapped.p, P->perm.p, n, P->xs.p, s);
            PK_HIP(hipMemcpyAsync(P->leaf_nsrc_host.p, P->leaf_nsrc.p, sizeof(int) * nl, hipMemcpyDeviceToHost, s));
            PK_HIP(hipStreamSynchronize(s));
            for (int i = 0; i < nl; ++i) {
                const int b = t.leaves[i];
                P->box_send[b] = P->box_tbeg[b] = t.begin[b] + P->leaf_nsrc_host.p[i];
            }
        }
        // one problem: its interaction lists are built on a host thread from here on, beside the
        // uploads below and the first evaluation's upward pass; every reader waits (lists_wait)
        if (n_problems == 1) {
            auto job = [P] {
                build_lists_host(P->tree, P->cfg.periodic_mask, P->lists);
                add_root_ring(P->tree, P->cfg.periodic_mask, near_layers(P->cfg), P->lists);
                list_stats(P);
            };
            try {
                P->lists_ready = std::async(std::launch::async, job).share();
            } catch (const std::system_error&) {   // no thread to be had: build them here
                job();
            }
        } else {
            list_stats(P);
        }
        P->b_send.upload(P->box_send, s);
        P->b_level.upload(t.level, s);
        P->b_ix.upload(t.ix, s);
        P->b_iy.upload(t.iy, s);
        P->b_iz.upload(t.iz, s);
        P->b_begin.upload(t.begin, s);
        P->b_end.upload(t.end, s);
        P->leaf_boxes.upload(t.leaves, s);
        if (P->cfg.precision == PKIFMM_MIXED) {
            P->ioff.ensure(3 * m);
            launch_leaf_offsets(P->xs.p, n, P->leaf_boxes.p, (int)t.leaves.size(), P->b_begin.p, P->b_end.p, P->b_level.p,
                                P->b_ix.p, P->b_iy.p, P->b_iz.p, P->ioff.p, s);
        }
        PK_HIP(hipStreamSynchronize(s));
        P->have_points = true;
        auto& st = P->stats;
        st.n_points = n;
        st.n_problems = n_problems;
        st.n_boxes = t.nbox();
        st.n_leaves = (int)t.leaves.size();
        st.depth = t.depth;
    } catch (const Error& e) {
        return fail(P, e);
    } catch (const std::bad_alloc&) {
        return fail(P, Error(PKIFMM_ERR_OOM, "host allocation"));
    }
    P->stats.ms_set_points = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return PKIFMM_OK;
}

}  // namespace

extern "C" {

int pkifmm_set_points(pkifmm_plan* P, int64_t n_src, const double* src_xyz, int64_t n_trg, const double* trg_xyz,
                      void* stream) {
    if (n_src < 0) return P ? fail(P, Error(PKIFMM_ERR_INVALID_ARG, "n_src")) : PKIFMM_ERR_INVALID_ARG;
    return set_points_impl(P, 1, &n_src, src_xyz, n_trg, trg_xyz, stream);
}

int pkifmm_set_points_batch(pkifmm_plan* P, int n_problems, const int64_t* counts, const double* xyz, void* stream) {
    return set_points_impl(P, n_problems, counts, xyz, 0, nullptr, stream);
}

int pkifmm_evaluate(pkifmm_plan* P, int R, const double* density, double* potential, void* stream) {
    if (!P) return PKIFMM_ERR_INVALID_ARG;
    if (!P->have_points) return fail(P, Error(PKIFMM_ERR_NO_POINTS, "set_points has not succeeded"));
    if (R < 1 || (P->n_src > 0 && !density) || (P->n_out > 0 && !potential))
        return fail(P, Error(PKIFMM_ERR_INVALID_ARG, "n_rhs or pointers"));
    auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = (hipStream_t)stream;
    P->allocator.stream = stream;
    AllocScope scope(&P->allocator);
    try {
        if (P->n == 0 || P->n_out == 0) return PKIFMM_OK;
        // new work lists (another n_rhs) overwrite lists and workspace that an evaluation still in
        // flight may read: wait for it first.  Otherwise the stream is ordered after the previous
        // evaluation on the device, whichever stream that ran on.
        if (P->R_built != R) wait_idle(P);
        PK_HIP(hipStreamWaitEvent(s, P->ev_done, 0));
        if (!(P->cfg.flags & PKIFMM_GRAPH)) {
            // a first evaluation on new points builds its work lists stage by stage, each
            // while the kernels of the previous stage run
            Workspace w;
            enqueue_evaluate(P, w, R, density, potential, s, true, true, P->R_built != R);
        } else {
            if (P->R_built != R) build_work(P, R);
            // captured once per (tree, R, buffers) on a library stream, replayed on the caller's
            const bool same = P->gexec && P->g_key_R == R && P->g_key_in == density && P->g_key_out == potential &&
                              P->g_key_gen == P->generation;
            if (!same) {
                wait_idle(P);   // the previous graph may still be running
                drop_graph(P);
                hipStream_t cs = P->capture_stream;
                PK_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed));
                P->capturing = true;
                try {
                    Workspace w;
                    enqueue_evaluate(P, w, R, density, potential, cs, false, false);
                } catch (...) {
                    P->capturing = false;
                    hipGraph_t g = nullptr;
                    (void)hipStreamEndCapture(cs, &g);
                    if (g) (void)hipGraphDestroy(g);
                    throw;
                }
                P->capturing = false;
                PK_HIP(hipStreamEndCapture(cs, &P->graph));
                PK_HIP(hipGraphInstantiate(&P->gexec, P->graph, nullptr, nullptr, 0));
                P->g_key_R = R;
                P->g_key_in = density;
                P->g_key_out = potential;
                P->g_key_gen = P->generation;
            }
            PK_HIP(hipGraphLaunch(P->gexec, s));
            PK_HIP(hipEventRecord(P->ev_done, s));
        }
    } catch (const Error& e) {
        return fail(P, e);
    } catch (const std::bad_alloc&) {
        return fail(P, Error(PKIFMM_ERR_OOM, "host allocation"));
    }
    P->stats.ms_evaluate = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return PKIFMM_OK;
}

int pkifmm_evaluate_noalloc(pkifmm_plan* P, int R, const double* density, double* potential, void* stream) {
    if (!P) return PKIFMM_ERR_INVALID_ARG;
    if (!P->have_points) return fail(P, Error(PKIFMM_ERR_NO_POINTS, "set_points has not succeeded"));
    if (R < 1 || (P->n_src > 0 && !density) || (P->n_out > 0 && !potential))
        return fail(P, Error(PKIFMM_ERR_INVALID_ARG, "n_rhs or pointers"));
    hipStream_t s = (hipStream_t)stream;
    try {
        if (P->n == 0 || P->n_out == 0) return PKIFMM_OK;
        // the work lists live in plan buffers, made by pkifmm_evaluate for this n_rhs
        if (P->R_built != R)
            throw Error(PKIFMM_ERR_INVALID_ARG, "no work lists for this n_rhs on these points: call pkifmm_evaluate "
                                                "with it once first");
        Workspace w;
        const size_t need = carve_workspace(P, R, nullptr, w);
        if (need > kScratchBytes)
            throw Error(PKIFMM_ERR_CAPACITY, "workspace of " + std::to_string(need) + " bytes exceeds the " +
                                                 std::to_string(kScratchBytes) + "-byte static array");
        carve_workspace(P, R, static_cast<char*>(P->scratch_base), w);
        // ordered after the plan's previous evaluation, unless the caller is capturing `stream`
        // into a graph (an event recorded outside the capture cannot be waited on inside it)
        hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
        PK_HIP(hipStreamIsCapturing(s, &cap));
        const bool capturing = cap != hipStreamCaptureStatusNone;
        if (!capturing) PK_HIP(hipStreamWaitEvent(s, P->ev_done, 0));
        P->capturing = capturing;
        try {
            enqueue_evaluate(P, w, R, density, potential, s, false, false);
        } catch (...) {
            P->capturing = false;
            throw;
        }
        P->capturing = false;
    } catch (const Error& e) {
        return fail(P, e);
    }
    return PKIFMM_OK;
}

int pkifmm_autotune(pkifmm_plan* P, int R, const double* density, double* potential, void* stream,
                    const char* tuning_file) {
    if (!P) return PKIFMM_ERR_INVALID_ARG;
    if (!P->have_points) return fail(P, Error(PKIFMM_ERR_NO_POINTS, "set_points has not succeeded"));
    if (R < 1 || (P->n_src > 0 && !density) || (P->n_out > 0 && !potential))
        return fail(P, Error(PKIFMM_ERR_INVALID_ARG, "n_rhs or pointers"));
    hipStream_t s = (hipStream_t)stream;
    P->allocator.stream = stream;
    AllocScope scope(&P->allocator);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    try {
        if (P->n == 0 || P->n_out == 0) return PKIFMM_OK;
        wait_idle(P);
        PK_HIP(hipEventCreate(&e0));
        PK_HIP(hipEventCreate(&e1));
        Tuning start;
        for (const TuneRec& rec : P->tune_table)
            if (rec.R == R) start = rec.t;
        P->tune_fixed = true;
        // median of 5 timed evaluations (after one untimed) with the choices t
        auto timed = [&](const Tuning& t) {
            P->tune = t;
            std::vector<float> ms;
            for (int rep = 0; rep < 6; ++rep) {
                Workspace w;
                PK_HIP(hipEventRecord(e0, s));
                enqueue_evaluate(P, w, R, density, potential, s, false, false, P->R_built != R);
                PK_HIP(hipEventRecord(e1, s));
                PK_HIP(hipEventSynchronize(e1));
                float m = 0.f;
                PK_HIP(hipEventElapsedTime(&m, e0, e1));
                if (rep > 0) ms.push_back(m);
            }
            std::sort(ms.begin(), ms.end());
            return (double)ms[ms.size() / 2];
        };
        Tuning best = start;
        double t_best = timed(best);
        auto descend = [&](int Tuning::*field, std::initializer_list<int> values) {
            for (int v : values) {
                if (v == best.*field) continue;
                Tuning t = best;
                t.*field = v;
                const double tt = timed(t);
                if (tt < 0.98 * t_best) {   // a change must win by more than the timing noise (~1-2 %)
                    best = t;
                    t_best = tt;
                }
            }
        };
        descend(&Tuning::near_wpc, {2, 3, 4, 6});
        if (P->cfg.precision == PKIFMM_MIXED) descend(&Tuning::m2l_rows, {64, kOzRows});
        if (R > 1) {
            if (P->k == 1) {
                descend(&Tuning::rb_near, {2, 4, 8, 16});
                descend(&Tuning::rb_s2m, {2, 4, 8});
            } else {
                descend(&Tuning::rb_near, {2, 4});
                descend(&Tuning::rb_s2m, {2, 4});
            }
        }
        P->tune_fixed = false;
        P->tune = best;
        bool found = false;
        for (TuneRec& rec : P->tune_table)
            if (rec.R == R) {
                rec.t = best;
                found = true;
            }
        if (!found) P->tune_table.push_back(TuneRec{R, best});
        ++P->generation;              // a captured graph of the old choices is recaptured
        P->stats.tune_ms = t_best;
        if (tuning_file && tuning_file[0]) {
            TuneLine l;
            l.arch = P->arch;
            l.kernel = P->cfg.kernel;
            l.mask = P->cfg.periodic_mask;
            l.p = P->cfg.p;
            l.precision = P->cfg.precision;
            l.R = R;
            l.t = best;
            if (!write_tuning_record(tuning_file, l)) throw Error(PKIFMM_ERR_INVALID_ARG, "tuning file not writable");
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    } catch (const Error& e) {
        P->tune_fixed = false;
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        return fail(P, e);
    }
    return PKIFMM_OK;
}

int pkifmm_get_stats(pkifmm_plan* P, pkifmm_stats* out) {
    if (!P || !out) return PKIFMM_ERR_INVALID_ARG;
    try {
        lists_wait(P);   // the list sizes
    } catch (const Error& e) {
        return fail(P, e);
    } catch (const std::bad_alloc&) {
        return fail(P, Error(PKIFMM_ERR_OOM, "host allocation"));
    }
    if (!P->pending_events.empty()) {
        double sum[PKIFMM_NUM_PHASES] = {0};
        int cnt = 0;
        hipError_t bad = hipSuccess;
        for (auto& ev : P->pending_events) {
            if (ev.size() == PKIFMM_NUM_PHASES + 2) {
                if (hipEventSynchronize(ev.back()) != hipSuccess) bad = hipErrorUnknown;
                // ev[0]: start; ev[1], ev[2]: ends of the up and M2L phases; ev[3], ev[4]: near field
                // on its own stream; ev[5], ev[6]: ends of the down and leaf phases
                const int a[PKIFMM_NUM_PHASES] = {3, 0, 1, 2, 5}, b[PKIFMM_NUM_PHASES] = {4, 1, 2, 5, 6};
                for (int i = 0; i < PKIFMM_NUM_PHASES && bad == hipSuccess; ++i) {
                    float ms = 0.f;
                    if (hipEventElapsedTime(&ms, ev[a[i]], ev[b[i]]) != hipSuccess) bad = hipErrorUnknown;
                    sum[i] += ms;
                }
                ++cnt;
            }
            for (hipEvent_t e : ev) (void)hipEventDestroy(e);
        }
        P->pending_events.clear();
        if (bad != hipSuccess) return fail(P, Error(PKIFMM_ERR_HIP, "phase timing events"));
        P->stats.n_timed = cnt;
        for (int i = 0; i < PKIFMM_NUM_PHASES; ++i) P->stats.ms_phase[i] = cnt ? sum[i] / cnt : 0.0;
    }
    P->stats.tune_near_wpc = P->tune.near_wpc;
    P->stats.tune_rb_near = P->tune.rb_near;
    P->stats.tune_rb_s2m = P->tune.rb_s2m;
    P->stats.tune_m2l_rows = P->tune.m2l_rows;
    *out = P->stats;
    return PKIFMM_OK;
}

int pkifmm_get_solve_factors(const pkifmm_plan* P, int which, int* rank, double* Ut, double* VS) {
    if (!P || !rank || (which != 0 && which != 1)) return PKIFMM_ERR_INVALID_ARG;
    const std::vector<double>& u = which == 0 ? P->f_up_Ut : P->f_dn_Ut;
    const std::vector<double>& v = which == 0 ? P->f_up_VS : P->f_dn_VS;
    *rank = which == 0 ? P->r_up : P->r_dn;
    if (Ut) std::memcpy(Ut, u.data(), sizeof(double) * u.size());
    if (VS) std::memcpy(VS, v.data(), sizeof(double) * v.size());
    return PKIFMM_OK;
}

int pkifmm_get_tree(const pkifmm_plan* P, int64_t* perm, int32_t* boxes) {
    if (!P) return PKIFMM_ERR_INVALID_ARG;
    if (!P->have_points) return PKIFMM_ERR_NO_POINTS;
    const HostTree& t = P->tree;
    if (perm && P->n > 0) {
        std::vector<uint32_t> h(P->n);
        if (hipMemcpy(h.data(), P->perm.p, sizeof(uint32_t) * P->n, hipMemcpyDeviceToHost) != hipSuccess)
            return PKIFMM_ERR_HIP;
        for (int64_t i = 0; i < P->n; ++i) perm[i] = h[i];
    }
    if (boxes)
        for (int b = 0; b < t.nbox(); ++b) {
            int fc = -1;
            for (int o = 0; o < 8 && fc < 0; ++o) fc = t.child[8 * b + o];
            int32_t row[8] = {t.level[b], t.ix[b], t.iy[b], t.iz[b], t.begin[b], t.end[b], t.parent[b], fc};
            std::memcpy(boxes + 8 * b, row, sizeof(row));
        }
    return PKIFMM_OK;
}

int pkifmm_get_list(const pkifmm_plan* P, char which, int64_t* offsets, int32_t* entries) {
    if (!P || !offsets) return PKIFMM_ERR_INVALID_ARG;
    if (!P->have_points) return PKIFMM_ERR_NO_POINTS;
    try {
        lists_wait(P);
    } catch (const Error& e) {
        return e.code;
    } catch (const std::bad_alloc&) {
        return PKIFMM_ERR_OOM;
    }
    const HostLists& L = P->lists;
    const std::vector<int64_t>* off;
    const std::vector<Entry>* ent;
    switch (which) {
        case 'U': off = &L.u_off; ent = &L.u; break;
        case 'V': off = &L.v_off; ent = &L.v; break;
        case 'W': off = &L.w_off; ent = &L.w; break;
        case 'X': off = &L.x_off; ent = &L.x; break;
        default: return PKIFMM_ERR_INVALID_ARG;
    }
    std::memcpy(offsets, off->data(), sizeof(int64_t) * off->size());
    if (entries)
        for (size_t e = 0; e < ent->size(); ++e) {
            const Entry& x = (*ent)[e];
            entries[4 * e] = x.src;
            entries[4 * e + 1] = x.sx;
            entries[4 * e + 2] = x.sy;
            entries[4 * e + 3] = x.sz;
        }
    return PKIFMM_OK;
}

int pkifmm_plan_destroy(pkifmm_plan* P) {
    if (!P) return PKIFMM_OK;
    lists_settle(P);
    if (P->ev_done) (void)hipEventSynchronize(P->ev_done);   // no evaluation may still read plan buffers
    for (auto& ev : P->pending_events)
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    drop_graph(P);
    if (P->setup_stream) (void)hipStreamDestroy(P->setup_stream);
    if (P->setup_stream2) (void)hipStreamDestroy(P->setup_stream2);
    if (P->setup_stream3) (void)hipStreamDestroy(P->setup_stream3);
    if (P->near_stream) (void)hipStreamDestroy(P->near_stream);
    if (P->x_stream) (void)hipStreamDestroy(P->x_stream);
    if (P->capture_stream) (void)hipStreamDestroy(P->capture_stream);
    if (P->ev_fork) (void)hipEventDestroy(P->ev_fork);
    if (P->ev_join) (void)hipEventDestroy(P->ev_join);
    if (P->ev_xjoin) (void)hipEventDestroy(P->ev_xjoin);
    if (P->ev_done) (void)hipEventDestroy(P->ev_done);
    delete P;
    return PKIFMM_OK;
}

const char* pkifmm_status_string(int s) {
    switch (s) {
        case PKIFMM_OK: return "ok";
        case PKIFMM_ERR_INVALID_ARG: return "invalid argument";
        case PKIFMM_ERR_OUT_OF_BOX: return "coordinate outside the box";
        case PKIFMM_ERR_INCOMPATIBLE: return "density violates the compatibility condition";
        case PKIFMM_ERR_UNSUPPORTED: return "unsupported kernel/periodicity";
        case PKIFMM_ERR_OOM: return "out of memory";
        case PKIFMM_ERR_HIP: return "HIP runtime error";
        case PKIFMM_ERR_NO_POINTS: return "no points set";
        case PKIFMM_ERR_NUMERICS: return "operator construction failed its self-check";
        case PKIFMM_ERR_CAPACITY: return "workspace exceeds the static array";
        case PKIFMM_ERR_CACHE_CORRUPT: return "operator cache file fails its checks";
        default: return "unknown status";
    }
}

const char* pkifmm_last_error(const pkifmm_plan* P) { return P ? P->last_error.c_str() : ""; }

}  // extern "C"
