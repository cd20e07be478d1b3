// On-disk cache of the costly Stage-1 operators (Algorithm 2, Stage 1): the factors of the
// two check-to-equivalent solves (U^T and V S^+, Appendix B) and the periodic root operator
// M_root = K^{P,F}(x^{B0,d}, y^{B0,u}).  They depend on the kernel, the periodic axes, p and
// the solve cutoff alone (unit box, raw kernels), and the paper computes them once for all
// simulations (Section 2.2, after the M2L solve).  The translation operators (M2M, L2L,
// M2L) are plain kernel evaluations and are rebuilt on the device each time.
//
// File layout (little-endian, as written by this host):
//   char magic[8] = "PKIFMMOP"; uint32 version; int32 kernel; uint32 mask; int32 p;
//   int32 kn; int32 r_up; int32 r_dn; int32 near_layers; double cutoff; double s_max_up, s_max_dn;
//   double up_Ut[r_up*kn], up_VS[kn*r_up], dn_Ut[r_dn*kn], dn_VS[kn*r_dn], mroot[kn*kn];
//   uint64 fnv1a64 of every byte before it.
#include <cinttypes>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include <unistd.h>

#include "opcache.h"

namespace pk {

namespace {

constexpr char kMagic[8] = {'P', 'K', 'I', 'F', 'M', 'M', 'O', 'P'};
constexpr uint32_t kVersion = 1;

struct Header {
    char magic[8];
    uint32_t version;
    int32_t kernel;
    uint32_t mask;
    int32_t p, kn, r_up, r_dn, near_layers;
    double cutoff, smax_up, smax_dn;
};
static_assert(sizeof(Header) == 64, "cache header layout");

uint64_t fnv1a(const unsigned char* p, size_t n, uint64_t h = 1469598103934665603ull) {
    for (size_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 1099511628211ull;
    }
    return h;
}

size_t payload_doubles(const Header& h) {
    return 2 * (size_t)h.r_up * h.kn + 2 * (size_t)h.r_dn * h.kn + (size_t)h.kn * h.kn;
}

}  // namespace

std::string opcache_path(const char* dir, int kernel, unsigned mask, int p, double cutoff, int near_layers) {
    char name[160];
    std::snprintf(name, sizeof(name), "pkifmm_ops_k%d_m%u_p%d_l%d_c%a_v%u.bin", kernel, mask, p, near_layers, cutoff,
                  kVersion);
    std::string d(dir);
    if (!d.empty() && d.back() != '/') d += '/';
    return d + name;
}

int opcache_read(const std::string& path, OpBlob* out) {
    FILE* f = std::fopen(path.c_str(), "rb");
    if (!f) return kOpcacheAbsent;
    std::vector<unsigned char> buf;
    unsigned char chunk[1 << 16];
    size_t got;
    while ((got = std::fread(chunk, 1, sizeof(chunk), f)) > 0) buf.insert(buf.end(), chunk, chunk + got);
    std::fclose(f);
    Header h;
    if (buf.size() < sizeof(Header) + sizeof(uint64_t)) return PKIFMM_ERR_CACHE_CORRUPT;
    std::memcpy(&h, buf.data(), sizeof(h));
    if (std::memcmp(h.magic, kMagic, 8) != 0 || h.version != kVersion || h.kn <= 0 || h.r_up <= 0 ||
        h.r_dn <= 0 || h.r_up > h.kn || h.r_dn > h.kn)
        return PKIFMM_ERR_CACHE_CORRUPT;
    const size_t nd = payload_doubles(h);
    if (buf.size() != sizeof(Header) + nd * sizeof(double) + sizeof(uint64_t)) return PKIFMM_ERR_CACHE_CORRUPT;
    uint64_t sum;
    std::memcpy(&sum, buf.data() + buf.size() - sizeof(uint64_t), sizeof(sum));
    if (fnv1a(buf.data(), buf.size() - sizeof(uint64_t)) != sum) return PKIFMM_ERR_CACHE_CORRUPT;
    if (!out) return PKIFMM_OK;
    out->kernel = h.kernel;
    out->mask = h.mask;
    out->p = h.p;
    out->kn = h.kn;
    out->r_up = h.r_up;
    out->r_dn = h.r_dn;
    out->near_layers = h.near_layers;
    out->cutoff = h.cutoff;
    out->smax_up = h.smax_up;
    out->smax_dn = h.smax_dn;
    size_t at = sizeof(Header);
    auto take = [&](std::vector<double>& v, size_t n) {
        v.resize(n);
        std::memcpy(v.data(), buf.data() + at, n * sizeof(double));
        at += n * sizeof(double);
    };
    take(out->up_Ut, (size_t)h.r_up * h.kn);
    take(out->up_VS, (size_t)h.kn * h.r_up);
    take(out->dn_Ut, (size_t)h.r_dn * h.kn);
    take(out->dn_VS, (size_t)h.kn * h.r_dn);
    take(out->mroot, (size_t)h.kn * h.kn);
    return PKIFMM_OK;
}

bool opcache_write(const std::string& path, const OpBlob& b) {
    Header h;
    std::memcpy(h.magic, kMagic, 8);
    h.version = kVersion;
    h.kernel = b.kernel;
    h.mask = b.mask;
    h.p = b.p;
    h.kn = b.kn;
    h.r_up = b.r_up;
    h.r_dn = b.r_dn;
    h.near_layers = b.near_layers;
    h.cutoff = b.cutoff;
    h.smax_up = b.smax_up;
    h.smax_dn = b.smax_dn;
    std::vector<unsigned char> buf(sizeof(Header));
    std::memcpy(buf.data(), &h, sizeof(h));
    auto put = [&](const std::vector<double>& v) {
        const unsigned char* p = reinterpret_cast<const unsigned char*>(v.data());
        buf.insert(buf.end(), p, p + v.size() * sizeof(double));
    };
    put(b.up_Ut);
    put(b.up_VS);
    put(b.dn_Ut);
    put(b.dn_VS);
    put(b.mroot);
    const uint64_t sum = fnv1a(buf.data(), buf.size());
    const unsigned char* sp = reinterpret_cast<const unsigned char*>(&sum);
    buf.insert(buf.end(), sp, sp + sizeof(sum));
    // written under a temporary name and renamed: a reader never sees a partial file
    const std::string tmp = path + ".tmp" + std::to_string((long)getpid());
    FILE* f = std::fopen(tmp.c_str(), "wb");
    if (!f) return false;
    const bool ok = std::fwrite(buf.data(), 1, buf.size(), f) == buf.size();
    if (std::fclose(f) != 0 || !ok || std::rename(tmp.c_str(), path.c_str()) != 0) {
        std::remove(tmp.c_str());
        return false;
    }
    return true;
}

}  // namespace pk

extern "C" int pkifmm_operator_cache_check(const char* path) {
    if (!path) return PKIFMM_ERR_INVALID_ARG;
    const int st = pk::opcache_read(path, nullptr);
    return st == pk::kOpcacheAbsent ? PKIFMM_ERR_INVALID_ARG : st;
}
