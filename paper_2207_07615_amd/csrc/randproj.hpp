// Randomized projection (fresh Gaussian sketch per iteration): device
// layout and launcher.
#pragma once

#include <algorithm>

#include "common.hpp"

namespace plss {

constexpr int kRpRows = 1024;  // rows per workgroup of the S_kᵀ r kernel

struct RpDesc {
  double* S;       // m x rp sketch S_k (row-major)
  double* Y;       // n x rp, Y = Aᵀ S_k (row-major)
  double* part_g;  // ngram x 256 partial Gram matrices (16 x 16)
  double* part_s;  // nsig x 16 partial S_kᵀ r
  double* c;       // 16 coefficients G^{-1} sigma (zero for columns left out)
  int r;           // sketch columns (1..16)
  int rp;          // r rounded up to 4 (one Philox block gives 4 normals)
  int ngram, nsig;
  unsigned k0, k1; // Philox key: the seed's low and high words
};

void launch_rp_step(const Desc* d, const RpDesc* rd, int rp, int m, int n, int AV, const int2* alist, int na,
                    bool striped, int ngram, int nsig, hipStream_t s);

}  // namespace plss
