// The operator cache on disk (opcache.cpp): host code only.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "pkifmm.h"

namespace pk {

struct OpBlob {                  // the cached Stage-1 operators of one (kernel, mask, p, cutoff)
    int kernel = 0;
    unsigned mask = 0;
    int p = 0, kn = 0, r_up = 0, r_dn = 0;
    int near_layers = 1;         // the root operator covers images |p|_inf > near_layers
    double cutoff = 0.0;
    double smax_up = 0.0, smax_dn = 0.0;   // largest singular values (the solves' self-check norm)
    std::vector<double> up_Ut, up_VS, dn_Ut, dn_VS, mroot;   // column-major, as the plan holds them
};

constexpr int kOpcacheAbsent = 1;

// file of (kernel, mask, p, cutoff) in dir
std::string opcache_path(const char* dir, int kernel, unsigned mask, int p, double cutoff, int near_layers);
// PKIFMM_OK (and *out filled unless NULL), kOpcacheAbsent, or PKIFMM_ERR_CACHE_CORRUPT (bad magic,
// version, sizes or checksum)
int opcache_read(const std::string& path, OpBlob* out);
// false if the file could not be written (the caller goes on without the cache)
bool opcache_write(const std::string& path, const OpBlob& b);

}  // namespace pk
