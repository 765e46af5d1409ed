// Randomized projection (the paper's comparison method of Section 8): every
// iteration draws a fresh standard normal sketch S_k (m x r) and applies
// eq. (pkLong) with W = I:
//   Y = Aᵀ S_k, G = Yᵀ Y, sigma = S_kᵀ r, c = G^{-1} sigma (kept columns),
//   p = Y c, x += p, r -= A p.
// S_k is drawn on the device by Philox4x32-10 (Salmon et al., SC 2011) and
// Box-Muller: entry [i, 4q + t] is normal t of the counter (i, k, q, 0) with
// key (seed low word, seed high word).  G is a Gram product over the n rows
// of Y on the matrix cores (v_mfma_f64_16x16x4f64).
//
// Launch sequence of one iteration (every kernel returns early once the
// solve is done):
//   k_rp_sketch, k_rp_y, k_rp_gram, k_rp_sig, k_rp_solve, k_rp_p,
//   k_sspmv<RESID> or k_spmv<RESID> (r -= A p, partial rho), k_rp_fin
#include "kernels.hpp"
#include "randproj.hpp"

namespace plss {

namespace {
constexpr int kPB = 1024;
typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ double bsum(double v, double* s_tmp) {
  v = wsum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) s_tmp[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = s_tmp[0];
  for (int q = 1; q < kPB / 64; ++q) t += s_tmp[q];
  __syncthreads();
  return t;
}

__device__ double bsum_array(const double* __restrict__ a, int n, double* s_tmp) {
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += kPB) v += a[i];
  return bsum(v, s_tmp);
}

// Philox4x32-10: ten rounds of the multiply-xor mix, key bumped by the Weyl
// constants between rounds.
__device__ __forceinline__ void philox(unsigned c[4], unsigned k0, unsigned k1) {
#pragma unroll
  for (int rnd = 0; rnd < 10; ++rnd) {
    if (rnd) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const unsigned long long p0 = 0xD2511F53ull * c[0];
    const unsigned long long p1 = 0xCD9E8D57ull * c[2];
    const unsigned hi0 = (unsigned)(p0 >> 32), lo0 = (unsigned)p0;
    const unsigned hi1 = (unsigned)(p1 >> 32), lo1 = (unsigned)p1;
    c[0] = hi1 ^ c[1] ^ k0;
    c[1] = lo1;
    c[2] = hi0 ^ c[3] ^ k1;
    c[3] = lo0;
  }
}

__device__ __forceinline__ double unit(unsigned w) { return ((double)w + 0.5) * 0x1p-32; }
}  // namespace

// S_k (m x rp, row-major): one Philox block per (row, group of 4 columns).
__global__ __launch_bounds__(256) void k_rp_sketch(const Desc* __restrict__ d, const RpDesc* __restrict__ rd) {
  const State* st = d->st;
  if (st->final_done || st->done) return;
  const int m = d->m, rp = rd->rp, nq = rp / 4;
  const unsigned it = (unsigned)(st->k_total + 1);
  const long long total = (long long)m * nq;
  for (long long e = blockIdx.x * 256ll + threadIdx.x; e < total; e += (long long)gridDim.x * 256) {
    const int i = (int)(e / nq), q = (int)(e % nq);
    unsigned c[4] = {(unsigned)i, it, (unsigned)q, 0u};
    philox(c, rd->k0, rd->k1);
    const double u0 = unit(c[0]), u1 = unit(c[1]), u2 = unit(c[2]), u3 = unit(c[3]);
    const double ra = sqrt(-2.0 * log(u0)), rb = sqrt(-2.0 * log(u2));
    const double aa = 6.283185307179586 * u1, ab = 6.283185307179586 * u3;
    double* s = rd->S + (size_t)i * rp + 4 * q;
    s[0] = ra * cos(aa);
    s[1] = ra * sin(aa);
    s[2] = rb * cos(ab);
    s[3] = rb * sin(ab);
  }
}

// Y = Aᵀ S_k: LPR lanes per row of Aᵀ (a column of A), lane q = column q of S.
template <int LPR>
__global__ __launch_bounds__(256) void k_rp_y(const Desc* __restrict__ d, const RpDesc* __restrict__ rd) {
  const State* st = d->st;
  if (st->final_done || st->done) return;
  const int n = d->n, rp = rd->rp;
  const int q = threadIdx.x % LPR;
  const int j = blockIdx.x * (256 / LPR) + threadIdx.x / LPR;
  if (j >= n || q >= rp) return;
  const double* __restrict__ tv = static_cast<const double*>(d->t_val);
  const int* __restrict__ ti = d->t_idx;
  const double* __restrict__ S = rd->S;
  double acc = 0.0;
  const int e1 = d->t_ptr[j + 1];
  int e = d->t_ptr[j];
  // eight entries at a time: indices, values and gathered rows of S all in
  // flight before the first product (the sum keeps the entry order)
  for (; e + 8 <= e1; e += 8) {
    int c[8];
    double v[8], sv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      c[u] = ti[e + u];
      v[u] = tv[e + u];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) sv[u] = S[(size_t)c[u] * rp + q];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += v[u] * sv[u];
  }
  for (; e < e1; ++e) acc += tv[e] * S[(size_t)ti[e] * rp + q];
  rd->Y[(size_t)j * rp + q] = acc;
}

// Partial G = Yᵀ Y per workgroup: each wave feeds 4 rows of Y per
// v_mfma_f64_16x16x4f64 (operand A = Yᵀ: lane -> (column lane % 16, row
// lane / 16); operand B = Y: lane -> (row lane / 16, column lane % 16), the
// same element), the 4 waves' 16 x 16 sums added in wave order.
__global__ __launch_bounds__(256) void k_rp_gram(const Desc* __restrict__ d, const RpDesc* __restrict__ rd) {
  __shared__ double s_g[4][256];
  const State* st = d->st;
  if (st->final_done || st->done) return;
  const int n = d->n, rp = rd->rp;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int col = lane & 15, kr = lane >> 4;
  const int waves = gridDim.x * 4;
  const int wid = blockIdx.x * 4 + w;
  d4 acc = {0.0, 0.0, 0.0, 0.0};
  for (long long r0 = 4ll * wid; r0 < n; r0 += 4ll * waves) {
    const long long row = r0 + kr;
    const double v = (row < n && col < rp) ? rd->Y[(size_t)row * rp + col] : 0.0;
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(v, v, acc, 0, 0, 0);
  }
  // result: item i of a lane -> (row lane / 16 + 4 i, column lane % 16)
#pragma unroll
  for (int i = 0; i < 4; ++i) s_g[w][(kr + 4 * i) * 16 + col] = acc[i];
  __syncthreads();
  const int t = threadIdx.x;
  rd->part_g[(size_t)blockIdx.x * 256 + t] = (s_g[0][t] + s_g[1][t]) + (s_g[2][t] + s_g[3][t]);
}

// Partial sigma = S_kᵀ r over chunks of kRpRows rows (lanes over columns).
__global__ __launch_bounds__(256) void k_rp_sig(const Desc* __restrict__ d, const RpDesc* __restrict__ rd) {
  __shared__ double s_a[256];
  const State* st = d->st;
  if (st->final_done || st->done) return;
  const int m = d->m, rp = rd->rp;
  const int q = threadIdx.x % 16, slot = threadIdx.x / 16;
  const int r0 = blockIdx.x * kRpRows, r1 = min(r0 + kRpRows, m);
  const double* __restrict__ r = static_cast<const double*>(d->r);
  double acc = 0.0;
  if (q < rp)
    for (int i = r0 + slot; i < r1; i += 16) acc += rd->S[(size_t)i * rp + q] * r[i];
  s_a[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x < 16) {
    double a = s_a[threadIdx.x];
    for (int u = 1; u < 16; ++u) a += s_a[u * 16 + threadIdx.x];
    rd->part_s[(size_t)blockIdx.x * 16 + threadIdx.x] = a;
  }
}

// G and sigma from their partials (fixed order), columns kept by the pivot
// rule, c = G^{-1} sigma on them; breakdown if none is kept.
__global__ __launch_bounds__(kPB) void k_rp_solve(const Desc* __restrict__ d, const RpDesc* __restrict__ rd) {
  __shared__ double s_G[16][16];
  __shared__ double s_sig[16];
  State* st = d->st;
  if (st->final_done || st->done) return;
  const int r = rd->r;
  const int t = threadIdx.x;
  if (t < 256) {
    double a = 0.0;
    for (int b = 0; b < rd->ngram; ++b) a += rd->part_g[(size_t)b * 256 + t];
    s_G[t / 16][t % 16] = a;
  } else if (t < 256 + 16) {
    const int q = t - 256;
    double a = 0.0;
    for (int b = 0; b < rd->nsig; ++b) a += rd->part_s[(size_t)b * 16 + q];
    s_sig[q] = a;
  }
  __syncthreads();
  if (t != 0) return;
  double L[16][16];
  int keep[16];
  int nk = 0;
  for (int j = 0; j < r; ++j) {
    double z[16];
    double zz = 0.0;
    for (int a = 0; a < nk; ++a) {
      double v = s_G[keep[a]][j];
      for (int c = 0; c < a; ++c) v -= L[a][c] * z[c];
      z[a] = v / L[a][a];
      zz += z[a] * z[a];
    }
    const double piv = s_G[j][j] - zz;
    if (piv > 1e-14 * s_G[j][j]) {
      for (int c = 0; c < nk; ++c) L[nk][c] = z[c];
      L[nk][nk] = sqrt(piv);
      keep[nk++] = j;
    }
  }
  for (int q = 0; q < 16; ++q) rd->c[q] = 0.0;
  if (nk == 0) {
    st->status = ST_BREAKDOWN;
    st->done = 1;
    return;
  }
  double tv[16];
  for (int a = 0; a < nk; ++a) {
    double v = s_sig[keep[a]];
    for (int c = 0; c < a; ++c) v -= L[a][c] * tv[c];
    tv[a] = v / L[a][a];
  }
  for (int a = nk - 1; a >= 0; --a) {
    double v = tv[a];
    for (int c = a + 1; c < nk; ++c) v -= L[c][a] * tv[c];
    tv[a] = v / L[a][a];
  }
  for (int a = 0; a < nk; ++a) rd->c[keep[a]] = tv[a];
  // the update is applied by the next kernels: count it now (the product
  // r -= A p runs for k > 0)
  st->k += 1;
  st->k_total += 1;
}

// p = Y c, x += p
__global__ __launch_bounds__(256) void k_rp_p(const Desc* __restrict__ d, const RpDesc* __restrict__ rd) {
  const State* st = d->st;
  if (st->final_done || st->done) return;
  const int n = d->n, rp = rd->rp;
  double c[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) c[q] = rd->c[q];
  double* p = static_cast<double*>(d->p);
  for (int j = blockIdx.x * 256 + threadIdx.x; j < n; j += gridDim.x * 256) {
    const double* y = rd->Y + (size_t)j * rp;
    double v = 0.0;
    for (int q = 0; q < rp; ++q) v += y[q] * c[q];
    p[j] = v;
    d->x[j] += v;
  }
}

// rho from the product's partials; residual history; stop test.
__global__ __launch_bounds__(kPB) void k_rp_fin(const Desc* __restrict__ d, const RpDesc* __restrict__ rd) {
  __shared__ double s_red[kPB / 64];
  State* st = d->st;
  if (st->final_done || st->done) return;
  const double rho = bsum_array(d->part_rho, d->rho_cnt, s_red);
  if (threadIdx.x != 0) return;
  st->rho = rho;
  if (st->k_total < d->hist_len) d->hist[st->k_total] = sqrt(rho) * st->scale;
  if (sqrt(rho) <= st->thr) {
    st->status = ST_OK;
    st->done = 1;
    return;
  }
  if (st->k_total >= st->maxit) {
    st->status = ST_NOT_CONVERGED;
    st->done = 1;
  }
}

void launch_rp_step(const Desc* d, const RpDesc* rd, int rp, int m, int n, int AV, const int2* alist, int na,
                    bool striped, int ngram, int nsig, hipStream_t s) {
  const long long cnt = (long long)m * (rp / 4);
  const int gs = (int)std::min<long long>((cnt + 255) / 256, 16384);
  k_rp_sketch<<<gs, 256, 0, s>>>(d, rd);
  const int lpr = rp <= 4 ? 4 : (rp <= 8 ? 8 : 16);
  const int gy = (n + 256 / lpr - 1) / (256 / lpr);
  switch (lpr) {
    case 4: k_rp_y<4><<<gy, 256, 0, s>>>(d, rd); break;
    case 8: k_rp_y<8><<<gy, 256, 0, s>>>(d, rd); break;
    default: k_rp_y<16><<<gy, 256, 0, s>>>(d, rd); break;
  }
  k_rp_gram<<<ngram, 256, 0, s>>>(d, rd);
  k_rp_sig<<<nsig, 256, 0, s>>>(d, rd);
  k_rp_solve<<<1, kPB, 0, s>>>(d, rd);
  k_rp_p<<<std::min((n + 255) / 256, 8192), 256, 0, s>>>(d, rd);
  if (striped) launch_sspmv(MODE_RESID, false, d, alist, na, 0, s);
  else launch_spmv(MODE_RESID, false, AV, d, alist, na, 0, s);
  k_rp_fin<<<1, kPB, 0, s>>>(d, rd);
  PLSS_HIP(hipGetLastError());
}

}  // namespace plss
