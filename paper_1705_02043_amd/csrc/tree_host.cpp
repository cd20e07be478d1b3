// Octree topology and periodic interaction lists, built on the host from the
// Morton keys the device has already sorted.  The topology is small (a few
// thousand boxes for a million points), so it is cheaper to build here than
// to launch a dependent kernel per level.
//
// Tree rule (the paper's notation table: at most s points per leaf): a box is
// split into its non-empty octants while it holds more than s points, up to
// level 21.  Boxes are numbered level by level and in Morton order within a
// level.
//
// Lists (Section 2: the near field of a box is its same-level adjacent boxes;
// adaptive KIFMM U/V/W/X lists), with adjacency taken through the periodic
// wrap on periodic axes and every entry carrying its image shift p in
// {-1,0,1}^3 (the source box is translated by +p):
//   U(B)  B leaf: all leaves A with A+p adjacent to B (B itself included)
//   V(B)  children of the colleagues of parent(B) not adjacent to B
//   W(B)  B leaf: descendants A of B's colleagues, not adjacent to B, whose
//         parent is adjacent to B
//   X(B)  all (A, p) with (B, -p) in W(A)
// The root has no V list; its far field is the periodic root operator.
#include <algorithm>
#include <exception>
#include <cstdlib>
#include <unordered_map>

#include "pkifmm.h"
#include "topology.h"

namespace pk {

namespace {

inline uint64_t spread3(uint32_t v) {
    uint64_t x = v & 0x1fffff;
    x = (x | (x << 32)) & 0x1f00000000ffffull;
    x = (x | (x << 16)) & 0x1f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

inline uint64_t morton3(uint32_t x, uint32_t y, uint32_t z) {
    return (spread3(x) << 2) | (spread3(y) << 1) | spread3(z);
}

}  // namespace

void build_tree_host(const uint64_t* keys, int64_t n, int s, HostTree& t) {
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
    std::vector<int> frontier{0};
    while (!frontier.empty() && lv < kMaxLevel) {
        std::vector<int> next;
        const int sh = 3 * (kMaxLevel - (lv + 1));
        for (int b : frontier) {
            if (t.end[b] - t.begin[b] <= s) continue;
            const uint64_t* lo_ptr = keys + t.begin[b];
            const uint64_t* hi_ptr = keys + t.end[b];
            for (int o = 0; o < 8; ++o) {
                int cx = 2 * t.ix[b] + ((o >> 2) & 1);
                int cy = 2 * t.iy[b] + ((o >> 1) & 1);
                int cz = 2 * t.iz[b] + (o & 1);
                uint64_t prefix = morton3(cx, cy, cz);
                uint64_t klo = prefix << sh;
                uint64_t khi = ((prefix + 1) << sh) - 1;
                const uint64_t* a = std::lower_bound(lo_ptr, hi_ptr, klo);
                const uint64_t* e = std::upper_bound(a, hi_ptr, khi);
                if (e <= a) continue;
                int c = add(lv + 1, cx, cy, cz, (int)(a - keys), (int)(e - keys), b);
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

namespace {
struct OffsetTable {
    int idx[7][7][7];
    int vec[kNumM2L][3];
    OffsetTable() {
        int i = 0;
        for (int a = -3; a <= 3; ++a)
            for (int b = -3; b <= 3; ++b)
                for (int c = -3; c <= 3; ++c) {
                    if (std::max(std::abs(a), std::max(std::abs(b), std::abs(c))) < 2) {
                        idx[a + 3][b + 3][c + 3] = -1;
                        continue;
                    }
                    idx[a + 3][b + 3][c + 3] = i;
                    vec[i][0] = a; vec[i][1] = b; vec[i][2] = c;
                    ++i;
                }
    }
};
const OffsetTable& offsets() {
    static const OffsetTable t;
    return t;
}
}  // namespace

// offsets in [-3,3]^3 with |delta|_inf >= 2, numbered in lexicographic order (x slowest)
int m2l_offset_index(int dx, int dy, int dz) {
    if (dx < -3 || dx > 3 || dy < -3 || dy > 3 || dz < -3 || dz > 3) return -1;
    return offsets().idx[dx + 3][dy + 3][dz + 3];
}

void m2l_offset_vector(int idx, int& dx, int& dy, int& dz) {
    const OffsetTable& o = offsets();
    dx = o.vec[idx][0]; dy = o.vec[idx][1]; dz = o.vec[idx][2];
}

void build_lists_host(const HostTree& t, unsigned mask, HostLists& L) {
    const int nb = t.nbox();
    // (level, ix, iy, iz) -> box.  The boxes of a level are numbered in Morton order, so the
    // lookup is a binary search over the level's keys; a tree not in that order (none is built
    // here) would fall back to hash maps
    std::vector<uint64_t> key(nb);
    for (int b = 0; b < nb; ++b) key[b] = morton3(t.ix[b], t.iy[b], t.iz[b]);
    const int nlev = (int)t.level_start.size() - 1;
    bool ordered = nlev >= 0 && t.level_start.back() == nb;
    for (int lv = 0; ordered && lv < nlev; ++lv)
        for (int b = t.level_start[lv]; b < t.level_start[lv + 1]; ++b)
            if (t.level[b] != lv || (b > t.level_start[lv] && key[b] <= key[b - 1])) {
                ordered = false;
                break;
            }
    std::vector<std::unordered_map<uint64_t, int>> at(ordered ? 0 : t.depth + 1);
    if (!ordered)
        for (int b = 0; b < nb; ++b) at[t.level[b]][key[b]] = b;
    auto find = [&](int lv, uint64_t k) -> int {
        if (!ordered) {
            auto it = at[lv].find(k);
            return it == at[lv].end() ? -1 : it->second;
        }
        if (lv >= nlev) return -1;
        const auto lo = key.begin() + t.level_start[lv], hi = key.begin() + t.level_start[lv + 1];
        const auto it = std::lower_bound(lo, hi, k);
        return it != hi && *it == k ? (int)(it - key.begin()) : -1;
    };

    auto coord = [&](int b, int c) { return c == 0 ? t.ix[b] : (c == 1 ? t.iy[b] : t.iz[b]); };
    // closed boxes A+p and B touch or overlap
    auto adjacent = [&](int a, const int p[3], int b) {
        int la = t.level[a], lb = t.level[b];
        int m = std::max(la, lb);
        int64_t sa = int64_t(1) << (m - la), sb = int64_t(1) << (m - lb), per = int64_t(1) << m;
        for (int c = 0; c < 3; ++c) {
            int64_t alo = coord(a, c) * sa + p[c] * per, ahi = alo + sa;
            int64_t blo = coord(b, c) * sb, bhi = blo + sb;
            if (alo > bhi || blo > ahi) return false;
        }
        return true;
    };
    struct Col { int box; int p[3]; };
    std::vector<std::vector<Col>> coll(nb);
#pragma omp parallel for schedule(dynamic, 16)
    for (int b = 0; b < nb; ++b) {
        const int lv = t.level[b];
        const int side = 1 << lv;
        coll[b].reserve(27);
        for (int ox = -1; ox <= 1; ++ox)
            for (int oy = -1; oy <= 1; ++oy)
                for (int oz = -1; oz <= 1; ++oz) {
                    int g[3] = {t.ix[b] + ox, t.iy[b] + oy, t.iz[b] + oz};
                    int p[3] = {0, 0, 0};
                    bool ok = true;
                    for (int c = 0; c < 3; ++c) {
                        if (g[c] >= 0 && g[c] < side) continue;
                        if (mask & (1u << c)) {
                            p[c] = g[c] < 0 ? -1 : 1;
                            g[c] -= p[c] * side;
                        } else {
                            ok = false;
                        }
                    }
                    if (!ok) continue;
                    const int a = find(lv, morton3(g[0], g[1], g[2]));
                    if (a >= 0) coll[b].push_back({a, {p[0], p[1], p[2]}});
                }
        // ordered by (box, shift code): the V lists built from them then come out ordered
        // (children are numbered in their parents' order), and need no sort below
        std::sort(coll[b].begin(), coll[b].end(), [](const Col& x, const Col& y) {
            if (x.box != y.box) return x.box < y.box;
            return (x.p[0] + 1) * 9 + (x.p[1] + 1) * 3 + (x.p[2] + 1) < (y.p[0] + 1) * 9 + (y.p[1] + 1) * 3 + (y.p[2] + 1);
        });
    }
    auto mk = [](int a, const int p[3]) { return Entry{a, (int8_t)p[0], (int8_t)p[1], (int8_t)p[2]}; };
    // sort by (source, shift) through a packed 64-bit key (the shift code is lexicographic)
    // n entries at v in place: returns the count left after removing duplicates
    auto sort_span = [](Entry* v, size_t n) -> size_t {
        thread_local std::vector<int64_t> sk;    // reused: no allocation per list
        sk.resize(n);
        bool inc = true;   // strictly increasing: already sorted, no duplicates
        for (size_t i = 0; i < n; ++i) {
            sk[i] = ((int64_t)v[i].src << 8) | ((v[i].sx + 1) * 9 + (v[i].sy + 1) * 3 + (v[i].sz + 1));
            if (i > 0 && sk[i] <= sk[i - 1]) inc = false;
        }
        if (inc) return n;
        std::sort(sk.begin(), sk.end());
        sk.erase(std::unique(sk.begin(), sk.end()), sk.end());
        for (size_t i = 0; i < sk.size(); ++i) {
            int code = (int)(sk[i] & 0xff);
            v[i] = Entry{(int)(sk[i] >> 8), (int8_t)(code / 9 - 1), (int8_t)((code / 3) % 3 - 1), (int8_t)(code % 3 - 1)};
        }
        return sk.size();
    };
    auto sort_entries = [&](std::vector<Entry>& v) { v.resize(sort_span(v.data(), v.size())); };
    std::vector<std::vector<Entry>> U(nb), V(nb), Wl(nb);
#pragma omp parallel for schedule(dynamic, 8)
    for (int b = 0; b < nb; ++b) {
        if (t.level[b] >= 1) {
            // same-level boxes: A + p is adjacent to B iff every integer offset is in [-1, 1]
            const int side = 1 << t.level[b];
            V[b].reserve(189);
            for (const Col& pc : coll[t.parent[b]])
                for (int o = 0; o < 8; ++o) {
                    int a = t.child[8 * pc.box + o];
                    if (a < 0) continue;
                    int dx = t.ix[a] + pc.p[0] * side - t.ix[b];
                    int dy = t.iy[a] + pc.p[1] * side - t.iy[b];
                    int dz = t.iz[a] + pc.p[2] * side - t.iz[b];
                    if (std::abs(dx) > 1 || std::abs(dy) > 1 || std::abs(dz) > 1) V[b].push_back(mk(a, pc.p));
                }
            sort_entries(V[b]);
        }
        if (!t.is_leaf(b)) continue;
        thread_local std::vector<Col> stack;
        stack.assign(coll[b].begin(), coll[b].end());
        while (!stack.empty()) {
            Col c = stack.back();
            stack.pop_back();
            if (t.is_leaf(c.box)) {
                U[b].push_back(mk(c.box, c.p));
                continue;
            }
            for (int o = 0; o < 8; ++o) {
                int d = t.child[8 * c.box + o];
                if (d < 0) continue;
                if (adjacent(d, c.p, b)) stack.push_back({d, {c.p[0], c.p[1], c.p[2]}});
                else Wl[b].push_back(mk(d, c.p));
            }
        }
        for (int anc = t.parent[b]; anc >= 0; anc = t.parent[anc])
            for (const Col& c : coll[anc])
                if (t.is_leaf(c.box) && adjacent(c.box, c.p, b)) U[b].push_back(mk(c.box, c.p));
        sort_entries(U[b]);
        sort_entries(Wl[b]);
    }
    auto flatten = [nb](std::vector<std::vector<Entry>>& in, std::vector<int64_t>& off, std::vector<Entry>& out) {
        off.assign(nb + 1, 0);
        for (int b = 0; b < nb; ++b) off[b + 1] = off[b] + (int64_t)in[b].size();
        out.resize(off[nb]);
#pragma omp parallel for schedule(static)
        for (int b = 0; b < nb; ++b) std::copy(in[b].begin(), in[b].end(), out.begin() + off[b]);
    };
    flatten(U, L.u_off, L.u);
    flatten(V, L.v_off, L.v);
    flatten(Wl, L.w_off, L.w);
    // X lists: the W entries reversed, placed by counting (sources in increasing order), then
    // each list put in (source, shift) order
    L.x_off.assign(nb + 1, 0);
    for (const Entry& e : L.w) ++L.x_off[e.src + 1];
    for (int b = 0; b < nb; ++b) L.x_off[b + 1] += L.x_off[b];
    L.x.resize(L.x_off[nb]);
    {
        std::vector<int64_t> at_x(L.x_off.begin(), L.x_off.end() - 1);
        for (int a = 0; a < nb; ++a)
            for (int64_t i = L.w_off[a]; i < L.w_off[a + 1]; ++i) {
                const Entry& e = L.w[i];
                L.x[at_x[e.src]++] = Entry{a, (int8_t)-e.sx, (int8_t)-e.sy, (int8_t)-e.sz};
            }
    }
    std::vector<int64_t> xn(nb);   // entries kept per list (a W list has no duplicates, so all)
#pragma omp parallel for schedule(dynamic, 64)
    for (int b = 0; b < nb; ++b)
        xn[b] = (int64_t)sort_span(L.x.data() + L.x_off[b], (size_t)(L.x_off[b + 1] - L.x_off[b]));
    int64_t kept = 0;
    for (int b = 0; b < nb; ++b) {
        const int64_t o = L.x_off[b];
        L.x_off[b] = kept;
        std::copy(L.x.begin() + o, L.x.begin() + o + xn[b], L.x.begin() + kept);   // moves left or stays
        kept += xn[b];
    }
    L.x_off[nb] = kept;
    L.x.resize(kept);
}

}  // namespace pk

extern "C" int pkifmm_host_topology(const uint64_t* keys, int64_t n, int s, unsigned mask, char which,
                                    int64_t* n_boxes, int32_t* boxes, int64_t* offsets, int32_t* entries) {
    using namespace pk;
    if (!n_boxes || n < 0 || s < 1 || (n > 0 && !keys) || (mask & ~7u)) return PKIFMM_ERR_INVALID_ARG;
    try {
        HostTree t;
        build_tree_host(keys, n, s, t);
        *n_boxes = t.nbox();
        if (boxes)
            for (int b = 0; b < t.nbox(); ++b) {
                int fc = -1;
                for (int o = 0; o < 8 && fc < 0; ++o) fc = t.child[8 * b + o];
                int32_t row[8] = {t.level[b], t.ix[b], t.iy[b], t.iz[b], t.begin[b], t.end[b], t.parent[b], fc};
                for (int c = 0; c < 8; ++c) boxes[8 * b + c] = row[c];
            }
        if (!offsets) return PKIFMM_OK;
        HostLists L;
        build_lists_host(t, mask, L);
        const std::vector<int64_t>* off;
        const std::vector<Entry>* ent;
        switch (which) {
            case 'U': off = &L.u_off; ent = &L.u; break;
            case 'V': off = &L.v_off; ent = &L.v; break;
            case 'W': off = &L.w_off; ent = &L.w; break;
            case 'X': off = &L.x_off; ent = &L.x; break;
            default: return PKIFMM_ERR_INVALID_ARG;
        }
        for (size_t i = 0; i < off->size(); ++i) offsets[i] = (*off)[i];
        if (entries)
            for (size_t e = 0; e < ent->size(); ++e) {
                entries[4 * e] = (*ent)[e].src;
                entries[4 * e + 1] = (*ent)[e].sx;
                entries[4 * e + 2] = (*ent)[e].sy;
                entries[4 * e + 3] = (*ent)[e].sz;
            }
    } catch (const std::bad_alloc&) {
        return PKIFMM_ERR_OOM;
    }
    return PKIFMM_OK;
}

namespace pk {

// Near-field layer l > 1 (Section 3.6): the root's images with 2 <= |p|_inf <= l along the periodic
// axes act on the root through its upward equivalent density (M2L by the offset p at level 0),
// leaving the images |p|_inf > l to the far-field operator.  They become the root's V list, in
// (source, shift) order.
void add_root_ring(const HostTree& t, unsigned mask, int layers, HostLists& L) {
    if (layers <= 1 || mask == 0 || t.nbox() == 0) return;
    std::vector<Entry> ring;
    const int lim[3] = {mask & 1u ? layers : 0, mask & 2u ? layers : 0, mask & 4u ? layers : 0};
    for (int x = -lim[0]; x <= lim[0]; ++x)
        for (int y = -lim[1]; y <= lim[1]; ++y)
            for (int z = -lim[2]; z <= lim[2]; ++z)
                if (std::max(std::abs(x), std::max(std::abs(y), std::abs(z))) >= 2)
                    ring.push_back(Entry{0, (int8_t)x, (int8_t)y, (int8_t)z});
    std::sort(ring.begin(), ring.end());
    const int root = t.level_start[0];
    std::vector<Entry> v;
    v.reserve(L.v.size() + ring.size());
    v.insert(v.end(), L.v.begin(), L.v.begin() + L.v_off[root]);
    v.insert(v.end(), L.v.begin() + L.v_off[root], L.v.begin() + L.v_off[root + 1]);
    v.insert(v.end(), ring.begin(), ring.end());
    v.insert(v.end(), L.v.begin() + L.v_off[root + 1], L.v.end());
    for (size_t b = root + 1; b < L.v_off.size(); ++b) L.v_off[b] += (int64_t)ring.size();
    L.v.swap(v);
}

// One problem per host thread, the largest first (the OpenMP runtime runs the list builds'
// own parallel loops inside this one with one thread).
void build_forest_host(const uint64_t* sorted_keys, const std::vector<int64_t>& poff, int s, unsigned periodic_mask,
                       int near_layers, std::vector<HostTree>& trees, std::vector<HostLists>& lists) {
    const int np = (int)poff.size() - 1;
    trees.assign(np, HostTree());
    lists.assign(np, HostLists());
    std::vector<int> order(np);
    for (int q = 0; q < np; ++q) order[q] = q;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return poff[a + 1] - poff[a] > poff[b + 1] - poff[b]; });
    std::vector<std::exception_ptr> err(np);
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < np; ++i) {
        const int q = order[i];
        try {
            build_tree_host(sorted_keys + poff[q], poff[q + 1] - poff[q], s, trees[q]);
            build_lists_host(trees[q], periodic_mask, lists[q]);
            add_root_ring(trees[q], periodic_mask, near_layers, lists[q]);
        } catch (...) {
            err[q] = std::current_exception();
        }
    }
    for (const std::exception_ptr& e : err)
        if (e) std::rethrow_exception(e);
}

// Several independent trees as one forest: boxes renumbered level-major (all
// problems' level-0 boxes, then level 1, ...), problems in order within a
// level, each problem's own (level, Morton) order kept; point ranges shifted by
// the problem offsets.  Lists only ever connect boxes of one problem.
void merge_forest(const std::vector<HostTree>& trees, const std::vector<HostLists>& lists,
                  const std::vector<int64_t>& poff, HostTree& t, HostLists& L, std::vector<int>& box_prob) {
    const int np = (int)trees.size();
    int depth = 0;
    for (const HostTree& q : trees) depth = std::max(depth, q.depth);
    std::vector<std::vector<int>> gid(np);
    for (int q = 0; q < np; ++q) gid[q].assign(trees[q].nbox(), -1);
    t = HostTree();
    box_prob.clear();
    std::vector<std::pair<int, int>> src;   // global -> (problem, local)
    for (int lv = 0; lv <= depth; ++lv) {
        t.level_start.push_back((int)src.size());
        for (int q = 0; q < np; ++q) {
            const HostTree& a = trees[q];
            if (lv > a.depth) continue;
            for (int b = a.level_start[lv]; b < a.level_start[lv + 1]; ++b) {
                gid[q][b] = (int)src.size();
                src.push_back({q, b});
            }
        }
    }
    t.level_start.push_back((int)src.size());
    t.depth = depth;
    const int nb = (int)src.size();
    t.level.resize(nb); t.ix.resize(nb); t.iy.resize(nb); t.iz.resize(nb);
    t.begin.resize(nb); t.end.resize(nb); t.parent.resize(nb); t.child.assign(8 * (size_t)nb, -1);
    box_prob.resize(nb);
    for (int g = 0; g < nb; ++g) {
        const int q = src[g].first, b = src[g].second;
        const HostTree& a = trees[q];
        t.level[g] = a.level[b]; t.ix[g] = a.ix[b]; t.iy[g] = a.iy[b]; t.iz[g] = a.iz[b];
        t.begin[g] = (int)(a.begin[b] + poff[q]);
        t.end[g] = (int)(a.end[b] + poff[q]);
        t.parent[g] = a.parent[b] < 0 ? -1 : gid[q][a.parent[b]];
        for (int o = 0; o < 8; ++o) {
            int c = a.child[8 * b + o];
            t.child[8 * g + o] = c < 0 ? -1 : gid[q][c];
        }
        box_prob[g] = q;
    }
    t.leaf_id.assign(nb, -1);
    for (int g = 0; g < nb; ++g)
        if (t.is_leaf(g)) {
            t.leaf_id[g] = (int)t.leaves.size();
            t.leaves.push_back(g);
        }
    auto merge = [&](auto off_of, auto ent_of, std::vector<int64_t>& off, std::vector<Entry>& ent) {
        off.assign(nb + 1, 0);
        ent.clear();
        for (int g = 0; g < nb; ++g) {
            const int q = src[g].first, b = src[g].second;
            const std::vector<int64_t>& lo = off_of(lists[q]);
            const std::vector<Entry>& le = ent_of(lists[q]);
            for (int64_t e = lo[b]; e < lo[b + 1]; ++e) {
                Entry x = le[e];
                x.src = gid[q][x.src];
                ent.push_back(x);
            }
            off[g + 1] = (int64_t)ent.size();
        }
    };
    merge([](const HostLists& l) -> const std::vector<int64_t>& { return l.u_off; },
          [](const HostLists& l) -> const std::vector<Entry>& { return l.u; }, L.u_off, L.u);
    merge([](const HostLists& l) -> const std::vector<int64_t>& { return l.v_off; },
          [](const HostLists& l) -> const std::vector<Entry>& { return l.v; }, L.v_off, L.v);
    merge([](const HostLists& l) -> const std::vector<int64_t>& { return l.w_off; },
          [](const HostLists& l) -> const std::vector<Entry>& { return l.w; }, L.w_off, L.w);
    merge([](const HostLists& l) -> const std::vector<int64_t>& { return l.x_off; },
          [](const HostLists& l) -> const std::vector<Entry>& { return l.x; }, L.x_off, L.x);
}

}  // namespace pk
