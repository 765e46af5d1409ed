// Kernels of the one-column sketch step (identity and mixed sketches).
//
// A step appends one sketch column s (a residual r or an identity column
// e_i) and applies the minimum-norm update of eq. (pkLong).  With
// S_{k-1}ᵀ r_{k-1} = 0 (eq. orthSr) and the stored history P = [p_1..p_kh],
// AP = [A p_1..A p_kh], Θ = diag(p_jᵀp_j) (Section 7), the update is
//   y = Aᵀ s, w = (AP)ᵀ s (= Pᵀ y), c = w/Θ, q = y - P c,
//   delta = (||y|| - ||d||)(||y|| + ||d||), ||d||^2 = Σ w_l^2/Θ_l,
//   sigma = sᵀ r, p = (sigma/delta) q.
// For s = e_i: y = a_i (row i of A), w = row i of AP, sigma = r_i
// (eq. pkKacz).  Then A p is appended to AP, r <- r - A p, x <- x + p.
//
// Launch sequence of one step (all early-exit when the system is done):
//   residual column:  k_spmv<TRANS> (y, ||y||^2), k_gemvt (partial w),
//                     k_col_prep, k_gemv, k_spmv<AP>, k_col_fin
//   identity column:  k_col_prep, k_gemv, k_spmv<AP>, k_col_fin
#include "kernels.hpp"

namespace plss {

namespace {
constexpr int kPW = 1024;  // threads of the per-system kernels

template <class T>
__device__ __forceinline__ T wsum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// fixed-order sum over a 1024-thread workgroup (valid in every thread)
__device__ double bsum(double v, double* s_tmp) {
  v = wsum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) s_tmp[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = s_tmp[0];
  for (int q = 1; q < kPW / 64; ++q) t += s_tmp[q];
  return t;
}

__device__ double bsum_array(const double* __restrict__ a, int n, double* s_tmp) {
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += kPW) v += a[i];
  return bsum(v, s_tmp);
}

// identity column index of sketch column t, or -1 for a residual column
__device__ __forceinline__ long long ident_index(const Desc* d, long long t) {
  if (d->sketch == 2) return (t & 1) ? (t >> 1) : -1;
  return t;
}
}  // namespace

// Stop test on r_0 = b (x0 = 0) before any column.
__global__ __launch_bounds__(kPW) void k_col_init(const Desc* __restrict__ D, const int* __restrict__ sys) {
  __shared__ double s_red[kPW / 64];
  const Desc* d = D + sys[blockIdx.x];
  State* st = d->st;
  if (st->final_done || st->done || st->k != 0 || st->col != 0) return;
  const double rho = bsum_array(d->part_rho, d->rho_cnt, s_red);
  if (threadIdx.x != 0) return;
  st->thr = st->tol_abs ? st->tol : st->tol * st->nb_out;
  st->scale = (st->tol_abs || st->nb_out == 0.0) ? 1.0 : 1.0 / st->nb_out;
  st->rho = rho;
  if (d->hist_len > 0) d->hist[0] = sqrt(rho) * st->scale;
  if (sqrt(rho) <= st->thr) {
    st->status = ST_OK;
    st->done = 1;
  }
}

// w_l = (AP)ᵀ r, partial over a chunk of 1024 rows per workgroup (one row
// per thread, 16 waves): part_w[l * wblk + blk] for l < kh.  Four columns
// of AP are read per pass, so 4 loads per thread are in flight; each wave
// sums its 64 products per column, and the 16 wave sums are added in wave
// order.
__global__ __launch_bounds__(kPW) void k_gemvt(const Desc* __restrict__ D, const int2* __restrict__ list) {
  __shared__ double s_w[kPW / 64][256];
  const int2 ent = list[blockIdx.x];
  const Desc* d = D + ent.x;
  const State* st = d->st;
  if (st->final_done || st->done) return;
  const int kh = (int)st->kh;
  if (kh == 0) return;
  const int m = d->m, lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int blk = ent.y;
  const int ri = blk * 1024 + threadIdx.x;
  const bool in = ri < m;
  const double rv = in ? static_cast<const double*>(d->r)[ri] : 0.0;
  const double* __restrict__ ap = d->AP + (in ? ri : 0);
  int l = 0;
  for (; l + 4 <= kh; l += 4) {
    double a[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) a[k] = in ? ap[(size_t)(l + k) * m] * rv : 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) a[k] = wsum(a[k]);
    if (lane == 0) {
#pragma unroll
      for (int k = 0; k < 4; ++k) s_w[w][l + k] = a[k];
    }
  }
  for (; l < kh; ++l) {
    double a = in ? ap[(size_t)l * m] * rv : 0.0;
    a = wsum(a);
    if (lane == 0) s_w[w][l] = a;
  }
  __syncthreads();
  for (int q = threadIdx.x; q < kh; q += kPW) {
    double a = s_w[0][q];
    for (int v = 1; v < kPW / 64; ++v) a += s_w[v][q];
    d->part_w[(size_t)q * d->wblk + blk] = a;
  }
}

// Column scalars: w, c = w/Θ, delta, sigma, gamma (one workgroup per system).
__global__ __launch_bounds__(kPW) void k_col_prep(const Desc* __restrict__ D, const int* __restrict__ sys) {
  __shared__ double s_red[kPW / 64];
  const Desc* d = D + sys[blockIdx.x];
  State* st = d->st;
  if (st->final_done || st->done) return;
  const int kh = (int)st->kh;
  const long long t = st->col;
  const long long id = ident_index(d, t);
  double yy, sigma;
  double w = 0.0;  // w_l for l = threadIdx.x
  const int l = threadIdx.x;
  if (id < 0) {
    // residual column: y = Aᵀ r (already in d->y), w = (AP)ᵀ r
    yy = bsum_array(d->part_phi, d->t_ntiles, s_red);
    if (l < kh) {
      // the block partials in block order, eight loads in flight
      const double* pw = d->part_w + (size_t)l * d->wblk;
      const int nb = d->wblk;
      int b = 0;
      for (; b + 8 <= nb; b += 8) {
        double v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = pw[b + k];
#pragma unroll
        for (int k = 0; k < 8; ++k) w += v[k];
      }
      for (; b < nb; ++b) w += pw[b];
    }
    sigma = st->rho;
  } else {
    const int i = d->perm[id % d->m];
    const int b0 = d->a_ptr[i], b1 = d->a_ptr[i + 1];
    const double* av = static_cast<const double*>(d->a_val);
    double s2 = 0.0;
    for (int e = b0 + threadIdx.x; e < b1; e += kPW) {
      const double v = av[e];
      d->dense[d->a_idx[e]] = v;
      s2 += v * v;
    }
    yy = bsum(s2, s_red);
    if (l < kh) w = d->AP[(size_t)l * d->m + i];
    sigma = static_cast<const double*>(d->r)[i];
    if (threadIdx.x == 0) st->row = i;
  }
  double c = 0.0, w2 = 0.0;
  if (l < kh) {
    c = w / d->Th[l];
    w2 = w * c;  // w_l^2 / Θ_l
    d->cv[l] = c;
  }
  const double nd2 = bsum(w2, s_red);
  if (threadIdx.x != 0) return;
  const double na = sqrt(yy), nd = sqrt(nd2);
  const double delta = (na - nd) * (na + nd);
  const bool bad = sigma == 0.0 || !(delta > 1e-14 * yy);
  st->col_kind = id < 0 ? 0 : 1;
  st->sigma = sigma;
  st->delta = delta;
  if (bad) {
    if (id < 0) {
      st->status = ST_BREAKDOWN;
      st->done = 1;
    }
    st->skip = 1;
    return;
  }
  st->skip = 0;
  st->gamma = sigma / delta;
}

// p = gamma (y - P c) -> column kh of P; x <- x + p; partial pᵀp.
__global__ __launch_bounds__(kWG) void k_gemv(const Desc* __restrict__ D, const int2* __restrict__ list) {
  __shared__ double s_c[256];
  __shared__ double s_red[kWaves];
  const int2 ent = list[blockIdx.x];
  const Desc* d = D + ent.x;
  const State* st = d->st;
  if (st->final_done || st->done || st->skip) return;
  const int kh = (int)st->kh, n = d->n;
  const double gamma = st->gamma;
  const double* __restrict__ ysrc = st->col_kind == 0 ? static_cast<const double*>(d->y) : d->dense;
  for (int l = threadIdx.x; l < kh; l += kWG) s_c[l] = d->cv[l];
  __syncthreads();
  double part = 0.0;
  const int base = ent.y * (kWG * 4);
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int j = base + u * kWG + threadIdx.x;
    if (j < n) {
      double acc = 0.0;
      for (int q = 0; q < kh; ++q) acc += d->P[(size_t)q * n + j] * s_c[q];
      const double pj = gamma * (ysrc[j] - acc);
      d->P[(size_t)kh * n + j] = pj;
      d->x[j] += pj;
      part += pj * pj;
    }
  }
  part = wsum(part);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = part;
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = s_red[0];
    for (int q = 1; q < kWaves; ++q) a += s_red[q];
    d->part_theta[ent.y] = a;
  }
}

// Close the step: Θ, history bookkeeping, residual history, stop test.
__global__ __launch_bounds__(kPW) void k_col_fin(const Desc* __restrict__ D, const int* __restrict__ sys) {
  __shared__ double s_red[kPW / 64];
  const Desc* d = D + sys[blockIdx.x];
  State* st = d->st;
  if (st->final_done || st->done) return;
  const long long t = st->col;
  const long long id = ident_index(d, t);
  if (id >= 0) {
    // clear the dense copy of row i
    const int i = st->row;
    for (int e = d->a_ptr[i] + threadIdx.x; e < d->a_ptr[i + 1]; e += kPW) d->dense[d->a_idx[e]] = 0.0;
  }
  const bool skip = st->skip != 0;
  double theta = 0.0, rho = 0.0;
  if (!skip) {
    theta = bsum_array(d->part_theta, d->u_nblk, s_red);
    rho = bsum_array(d->part_rho, d->rho_cnt, s_red);
  }
  if (threadIdx.x != 0) return;
  st->col = t + 1;
  const bool pass_end = id >= 0 && (id % d->m) == d->m - 1;
  if (!skip) {
    d->Th[st->kh] = theta;
    st->kh += 1;
    st->k += 1;
    st->k_total += 1;
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
      return;
    }
  }
  if (st->col >= st->max_cols) {  // bound on columns examined (skips included)
    st->status = ST_NOT_CONVERGED;
    st->done = 1;
    return;
  }
  if (pass_end || st->kh >= st->hist_cap) st->kh = 0;
}

// ------------------------------------------------------------------ launchers

void launch_col_init(const Desc* d, const int* sys, int ns, hipStream_t s) {
  k_col_init<<<ns, kPW, 0, s>>>(d, sys);
}

void launch_sketch_step(const Desc* d, int V, const int2* alist, int na, const int2* tlist, int nt,
                        const int2* ulist, int nu, const int2* wlist, int nw, const int* sys, int ns,
                        bool residual_column, int VT, const int2* cblist, int ncb, int VB, hipStream_t s) {
  if (residual_column) {
    launch_spmv(MODE_TRANS, false, VT, d, tlist, nt, 1, s);
    k_gemvt<<<nw, kPW, 0, s>>>(d, wlist);
  }
  k_col_prep<<<ns, kPW, 0, s>>>(d, sys);
  k_gemv<<<nu, kWG, 0, s>>>(d, ulist);
  if (ncb > 0) {
    // column blocks: each XCD gathers its own slice of the new column of P
    launch_spmv(MODE_APB, false, VB, d, cblist, ncb, 0, s);
    launch_apcomb(d, alist, na, s);
  } else {
    launch_spmv(MODE_AP, false, V, d, alist, na, 0, s);
  }
  k_col_fin<<<ns, kPW, 0, s>>>(d, sys);
  PLSS_HIP(hipGetLastError());
}

}  // namespace plss
