// Host code of the library under AddressSanitizer and UndefinedBehaviorSanitizer (built by
// tests/test_sanitize_host.py with g++, no GPU code): the octree and U/V/W/X lists
// (pkifmm_host_topology) on uniform, graded, clustered, one-point, empty and face-touching
// inputs for every periodic mask, the forest of a batch (one problem per host thread) against
// each problem built alone, and the operator cache (write, read back, corrupt, truncate,
// check).  Exits non-zero on any mismatch; the sanitizers abort on any memory or UB error.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include <unistd.h>

#include "opcache.h"
#include "pkifmm.h"
#include "topology.h"

namespace {

uint64_t spread(uint64_t v) {     // 21 bits -> every third bit
    v &= 0x1fffff;
    v = (v | v << 32) & 0x1f00000000ffffULL;
    v = (v | v << 16) & 0x1f0000ff0000ffULL;
    v = (v | v << 8) & 0x100f00f00f00f00fULL;
    v = (v | v << 4) & 0x10c30c30c30c30c3ULL;
    v = (v | v << 2) & 0x1249249249249249ULL;
    return v;
}

uint64_t key_of(double x, double y, double z) {
    auto q = [](double u) { return (uint64_t)std::min(2097151.0, std::floor(u * 2097152.0)); };
    return spread(q(x)) << 2 | spread(q(y)) << 1 | spread(q(z));
}

int fails = 0;

void topology(const std::vector<uint64_t>& keys, int s, const char* name) {
    for (unsigned mask = 0; mask < 8; ++mask) {
        int64_t nb = 0;
        if (pkifmm_host_topology(keys.data(), (int64_t)keys.size(), s, mask, 'U', &nb, nullptr, nullptr, nullptr) !=
            PKIFMM_OK) {
            std::printf("%s: count failed\n", name);
            ++fails;
            return;
        }
        std::vector<int32_t> boxes((size_t)8 * std::max<int64_t>(nb, 1));
        std::vector<int64_t> off((size_t)nb + 1);
        for (char which : {'U', 'V', 'W', 'X'}) {
            int64_t nb2 = 0;
            int rc = pkifmm_host_topology(keys.data(), (int64_t)keys.size(), s, mask, which, &nb2, boxes.data(),
                                          off.data(), nullptr);
            if (rc != PKIFMM_OK || nb2 != nb || off[0] != 0) {
                std::printf("%s mask %u %c: rc %d\n", name, mask, which, rc);
                ++fails;
                continue;
            }
            std::vector<int32_t> ent((size_t)4 * std::max<int64_t>(off[nb], 1));
            rc = pkifmm_host_topology(keys.data(), (int64_t)keys.size(), s, mask, which, &nb2, boxes.data(), off.data(),
                                      ent.data());
            for (int64_t b = 0; b < nb && rc == PKIFMM_OK; ++b) {
                if (off[b + 1] < off[b]) { std::printf("%s: offsets decrease\n", name); ++fails; break; }
            }
            for (int64_t e = 0; e < off[nb]; ++e)
                if (ent[4 * e] < 0 || ent[4 * e] >= nb || std::abs(ent[4 * e + 1]) > 1 || std::abs(ent[4 * e + 2]) > 1 ||
                    std::abs(ent[4 * e + 3]) > 1) {
                    std::printf("%s mask %u %c: entry %lld out of range\n", name, mask, which, (long long)e);
                    ++fails;
                    break;
                }
        }
        // leaves partition the points
        int64_t covered = 0;
        for (int64_t b = 0; b < nb; ++b)
            if (boxes[8 * b + 7] < 0) covered += boxes[8 * b + 5] - boxes[8 * b + 4];
        if (covered != (int64_t)keys.size()) {
            std::printf("%s: leaves hold %lld of %zu points\n", name, (long long)covered, keys.size());
            ++fails;
        }
    }
}

std::vector<uint64_t> sorted_keys(const std::vector<double>& xyz) {
    std::vector<uint64_t> k(xyz.size() / 3);
    for (size_t i = 0; i < k.size(); ++i) k[i] = key_of(xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2]);
    std::sort(k.begin(), k.end());
    return k;
}

// A batch's forest (build_forest_host: several problems at a time on host threads, largest
// first) against every problem built alone: the same boxes and the same lists.
void forest(const std::vector<std::vector<uint64_t>>& probs, int s) {
    std::vector<uint64_t> keys;
    std::vector<int64_t> poff{0};
    for (const auto& p : probs) {
        keys.insert(keys.end(), p.begin(), p.end());
        poff.push_back(poff.back() + (int64_t)p.size());
    }
    for (unsigned mask : {0u, 1u, 3u, 7u}) {
        const int layers = mask == 7u ? 2 : 1;
        std::vector<pk::HostTree> trees;
        std::vector<pk::HostLists> lists;
        pk::build_forest_host(keys.data(), poff, s, mask, layers, trees, lists);
        if (trees.size() != probs.size() || lists.size() != probs.size()) {
            std::printf("forest mask %u: %zu problems\n", mask, trees.size());
            ++fails;
            continue;
        }
        for (size_t q = 0; q < probs.size(); ++q) {
            pk::HostTree t;
            pk::HostLists L;
            pk::build_tree_host(keys.data() + poff[q], poff[q + 1] - poff[q], s, t);
            pk::build_lists_host(t, mask, L);
            pk::add_root_ring(t, mask, layers, L);
            const pk::HostTree& f = trees[q];
            const pk::HostLists& g = lists[q];
            const bool same = t.level == f.level && t.ix == f.ix && t.iy == f.iy && t.iz == f.iz &&
                              t.begin == f.begin && t.end == f.end && t.parent == f.parent && t.child == f.child &&
                              t.leaves == f.leaves && t.level_start == f.level_start && t.depth == f.depth &&
                              L.u_off == g.u_off && L.v_off == g.v_off && L.w_off == g.w_off && L.x_off == g.x_off &&
                              L.u == g.u && L.v == g.v && L.w == g.w && L.x == g.x;
            if (!same) {
                std::printf("forest mask %u: problem %zu differs from its own build\n", mask, q);
                ++fails;
            }
        }
    }
}

void cache() {
    const std::string dir = "asan_cache_dir";
    std::string cmd = "mkdir -p " + dir;
    if (std::system(cmd.c_str()) != 0) { ++fails; return; }
    pk::OpBlob b;
    b.kernel = 2; b.mask = 7; b.p = 4; b.kn = 3 * 56; b.r_up = 150; b.r_dn = 149; b.near_layers = 2;
    b.cutoff = 1e-11; b.smax_up = 3.5; b.smax_dn = 2.5;
    std::mt19937 rng(5);
    std::uniform_real_distribution<double> u(-1, 1);
    auto fill = [&](std::vector<double>& v, size_t n) { v.resize(n); for (double& x : v) x = u(rng); };
    fill(b.up_Ut, (size_t)b.kn * b.r_up); fill(b.up_VS, (size_t)b.kn * b.r_up);
    fill(b.dn_Ut, (size_t)b.kn * b.r_dn); fill(b.dn_VS, (size_t)b.kn * b.r_dn);
    fill(b.mroot, (size_t)b.kn * b.kn);
    const std::string path = pk::opcache_path(dir.c_str(), b.kernel, b.mask, b.p, b.cutoff, b.near_layers);
    if (!pk::opcache_write(path, b)) { std::printf("cache write failed\n"); ++fails; return; }
    pk::OpBlob r;
    if (pk::opcache_read(path, &r) != PKIFMM_OK || r.up_Ut != b.up_Ut || r.mroot != b.mroot || r.r_dn != b.r_dn ||
        r.near_layers != 2) {
        std::printf("cache round trip failed\n");
        ++fails;
    }
    if (pkifmm_operator_cache_check(path.c_str()) != PKIFMM_OK) { std::printf("check of a good file failed\n"); ++fails; }
    // one flipped byte in the payload, then a truncated file, then a missing one
    FILE* f = std::fopen(path.c_str(), "r+b");
    std::fseek(f, 1000, SEEK_SET);
    int c = std::fgetc(f);
    std::fseek(f, 1000, SEEK_SET);
    std::fputc(c ^ 0x10, f);
    std::fclose(f);
    if (pk::opcache_read(path, &r) != PKIFMM_ERR_CACHE_CORRUPT) { std::printf("flip not detected\n"); ++fails; }
    if (pkifmm_operator_cache_check(path.c_str()) != PKIFMM_ERR_CACHE_CORRUPT) { ++fails; }
    if (truncate(path.c_str(), 40) != 0) { ++fails; }
    if (pk::opcache_read(path, &r) != PKIFMM_ERR_CACHE_CORRUPT) { std::printf("truncation not detected\n"); ++fails; }
    if (truncate(path.c_str(), 0) != 0) { ++fails; }
    if (pk::opcache_read(path, &r) != PKIFMM_ERR_CACHE_CORRUPT) { std::printf("empty file not detected\n"); ++fails; }
    if (pk::opcache_read(dir + "/absent.bin", &r) != pk::kOpcacheAbsent) { ++fails; }
    if (pkifmm_operator_cache_check((dir + "/absent.bin").c_str()) != PKIFMM_ERR_INVALID_ARG) { ++fails; }
    if (pkifmm_operator_cache_check(nullptr) != PKIFMM_ERR_INVALID_ARG) { ++fails; }
}

}  // namespace

int main() {
    std::mt19937 rng(1);
    std::uniform_real_distribution<double> u(0.0, 1.0);
    std::normal_distribution<double> g(0.0, 1.0);
    std::vector<double> xyz;
    for (int i = 0; i < 3 * 6000; ++i) xyz.push_back(u(rng));
    topology(sorted_keys(xyz), 40, "uniform");
    xyz.clear();
    for (int i = 0; i < 4000; ++i) {            // graded: a dense ball near a corner and a thin background
        const bool ball = i % 4 != 0;
        for (int a = 0; a < 3; ++a) {
            double v = ball ? 0.05 + 0.01 * g(rng) : u(rng);
            xyz.push_back(std::min(std::max(v, 0.0), std::nextafter(1.0, 0.0)));
        }
    }
    topology(sorted_keys(xyz), 20, "graded");
    xyz.clear();
    for (int i = 0; i < 2000; ++i) {            // points on the faces and corners
        const double c[3] = {i % 3 == 0 ? 0.0 : u(rng), i % 5 == 0 ? std::nextafter(1.0, 0.0) : u(rng), i % 7 == 0 ? 0.0 : u(rng)};
        for (double v : c) xyz.push_back(v);
    }
    topology(sorted_keys(xyz), 16, "faces");
    std::vector<uint64_t> same(500, key_of(0.3, 0.3, 0.3));   // coincident points: the depth limit
    topology(same, 8, "coincident");
    topology(std::vector<uint64_t>{key_of(0.5, 0.5, 0.5)}, 1, "one point");
    topology(std::vector<uint64_t>{}, 10, "empty");
    {   // a batch: uniform, graded, empty, one point, coincident, uniform again (sizes unordered)
        std::vector<std::vector<uint64_t>> probs;
        for (int n : {3000, 0, 1, 800}) {
            std::vector<double> p;
            for (int i = 0; i < 3 * n; ++i) p.push_back(n == 800 ? std::pow(u(rng), 3.0) : u(rng));
            probs.push_back(sorted_keys(p));
        }
        probs.push_back(same);
        probs.push_back(sorted_keys(xyz));      // the faces set
        forest(probs, 24);
    }
    int64_t nb = 0;
    if (pkifmm_host_topology(nullptr, 5, 10, 0, 'U', &nb, nullptr, nullptr, nullptr) != PKIFMM_ERR_INVALID_ARG) ++fails;
    std::vector<uint64_t> k1{1, 2, 3};
    if (pkifmm_host_topology(k1.data(), 3, 10, 8, 'U', &nb, nullptr, nullptr, nullptr) != PKIFMM_ERR_INVALID_ARG) ++fails;
    cache();
    std::printf("host code under the sanitizers: %s\n", fails ? "FAILED" : "ok");
    return fails ? 1 : 0;
}
