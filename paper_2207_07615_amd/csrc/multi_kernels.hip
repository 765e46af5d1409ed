// Many right-hand sides on one matrix: s independent residual-sketch
// recurrences (Algorithm 1 per column) whose products with A and Aᵀ are
// sparse x dense block products.  Blocks are row-major (row i holds the s
// columns contiguously), so each stored entry of A is read once per
// iteration for all s columns and the gathered row of the dense block is
// one contiguous access.  Every column keeps its own scalars and stop test;
// a finished column keeps its x and is no longer updated.
#include "multi_kernels.hpp"

namespace plss {

namespace {
template <class T>
__device__ __forceinline__ T wsum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
constexpr int kMW = 1024;  // threads of the per-block scalar kernel
}  // namespace

// Block product over the rows of one direction (CSR of A, or of Aᵀ).
// W lanes per row (W >= s, a power of two), kMB/W rows in flight per
// workgroup, kRB rows per workgroup (larger workgroups leave fewer per-block
// partials for the one-workgroup scalar step to read).  Per-column partial sums of the
// epilogue's squares go to part[blk * s + c] in a fixed order.
template <class Val, class Vin, class Acc, int MODE, int W>
__global__ __launch_bounds__(kMB) void k_spmm(const MDesc* __restrict__ d) {
  constexpr int NS = kMB / W;
  __shared__ double s_p[2][NS][W];
  const MState* st = d->st;
  if (st->all_done) return;
  const bool tr = (MODE == MMODE_TRANS);
  const int* __restrict__ ptr = tr ? d->t_ptr : d->a_ptr;
  const int* __restrict__ idx = tr ? d->t_idx : d->a_idx;
  const Val* __restrict__ val = static_cast<const Val*>(tr ? d->t_val : d->a_val);
  const int nrows = tr ? d->n : d->m;
  const int s = d->s;
  const int slot = threadIdx.x / W, c = threadIdx.x % W;
  const bool col = c < s;
  bool live = col && !(MODE == MMODE_REFINE ? st->final_[c] : st->done[c]);
  if (MODE == MMODE_RESID) live = live && st->k[c] > 0;
  const Vin* __restrict__ xin;
  if (MODE == MMODE_RESID) xin = static_cast<const Vin*>(d->P);
  else if (MODE == MMODE_TRANS) xin = static_cast<const Vin*>(d->R);
  else xin = reinterpret_cast<const Vin*>(d->X);
  double part = 0.0, part2 = 0.0;
  const int row0 = blockIdx.x * kRB;
  const int row1 = min(row0 + kRB, nrows);
  for (int i = row0 + slot; i < row1; i += NS) {
    Acc acc = Acc(0);
    const int b0 = ptr[i], b1 = ptr[i + 1];
    if (live) {  // a finished column's sums are not used: no gathers for it
      // eight entries at a time: their indices, values and gathered rows
      // are all in flight before the first product (the sum keeps the
      // entry order)
      int e = b0;
      for (; e + 8 <= b1; e += 8) {
        int j[8];
        Val v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          j[u] = idx[e + u];
          v[u] = val[e + u];
        }
        Vin xv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) xv[u] = xin[(size_t)j[u] * s + c];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += Acc(v[u]) * Acc(xv[u]);
      }
      for (; e < b1; ++e) {
        const int j = idx[e];
        acc += Acc(val[e]) * Acc(xin[(size_t)j * s + c]);
      }
    }
    if (live) {
      const size_t o = (size_t)i * s + c;
      if (MODE == MMODE_RESID) {
        using Vec = Vin;
        Vec* R = static_cast<Vec*>(d->R);
        const Acc rn = Acc(R[o]) - acc;
        R[o] = Vec(rn);
        part += double(rn) * double(rn);
      } else if (MODE == MMODE_TRANS) {
        using Vec = Vin;
        static_cast<Vec*>(d->Y)[o] = Vec(acc);
        const double a = double(Vec(acc));
        part += a * a;
      } else {
        const double bi = d->B[o];
        const double ri = bi - double(acc);
        d->R64[o] = ri;
        part += ri * ri;
        part2 += bi * bi;
      }
    }
  }
  s_p[0][slot][c] = part;
  s_p[1][slot][c] = part2;
  __syncthreads();
  // thread c < s is lane c of slot 0: its `live` is column c's (a column
  // skipped by this launch keeps the partials another kernel wrote)
  if (threadIdx.x < s && live) {
    double a = 0.0, b2 = 0.0;
    for (int q = 0; q < NS; ++q) {
      a += s_p[0][q][threadIdx.x];
      b2 += s_p[1][q][threadIdx.x];
    }
    double* dst = (MODE == MMODE_TRANS) ? d->part_phi : d->part_rho;
    dst[(size_t)blockIdx.x * s + threadIdx.x] = a;
    if (MODE == MMODE_REFINE) d->part_b[(size_t)blockIdx.x * s + threadIdx.x] = b2;
  }
}

// Fixed-order per-column sums of part[blk * s + c], blk < nb: thread t
// handles column t % s over blocks t / s, t / s + kMW / s, ...
__device__ void col_sums(const double* __restrict__ part, int nb, int s, double* s_tmp, double* out) {
  const int sub = threadIdx.x / s, c = threadIdx.x % s, nsub = kMW / s;
  double v = 0.0;
  if (sub < nsub) {
    // 16 independent partial sums, their loads in flight together (one
    // workgroup reads all the partials, so its loads in flight set the
    // pace), combined in a fixed order
    constexpr int U = 16;
    double a[U];
#pragma unroll
    for (int u = 0; u < U; ++u) a[u] = 0.0;
    for (int b = sub; b < nb; b += U * nsub) {
      double t[U];
#pragma unroll
      for (int u = 0; u < U; ++u) t[u] = b + u * nsub < nb ? part[(size_t)(b + u * nsub) * s + c] : 0.0;
#pragma unroll
      for (int u = 0; u < U; ++u) a[u] += t[u];
    }
#pragma unroll
    for (int w = U / 2; w > 0; w >>= 1)
#pragma unroll
      for (int u = 0; u < w; ++u) a[u] = a[u] + a[u + w];
    v = a[0];
  }
  __syncthreads();
  if (sub < nsub) s_tmp[sub * s + c] = v;
  __syncthreads();
  if (threadIdx.x < s) {
    double a = 0.0;
    for (int q = 0; q < nsub; ++q) a += s_tmp[q * s + threadIdx.x];
    out[threadIdx.x] = a;
  }
  __syncthreads();
}

// Per-column scalars of Algorithm 1 (one workgroup).
// One workgroup per column: the column's block partials of rho, phi, theta
// (and of ||b||², needed only at an inner start) summed in a fixed order -
// thread t adds blocks t, t + kMS, ... in order, then a tree over the
// threads - with every load of the column issued together; then the
// column's step scalars.
constexpr int kMS = 256;

__device__ __forceinline__ double tree_sum(double v, double* s_buf) {
  s_buf[threadIdx.x] = v;
  __syncthreads();
  for (int w = kMS / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) s_buf[threadIdx.x] += s_buf[threadIdx.x + w];
    __syncthreads();
  }
  return s_buf[0];
}

__global__ __launch_bounds__(kMS) void k_mstep(const MDesc* __restrict__ d) {
  __shared__ double s_buf[4][kMS];
  MState* st = d->st;
  if (st->all_done) return;
  const int s = d->s, c = blockIdx.x;
  if (st->done[c]) return;  // the same for the whole workgroup
  const long long k = st->k[c];
  const bool want_b = k == 0;
  const int nmax = max(d->na_blk, max(d->nt_blk, d->nu_blk));
  double a_rho = 0.0, a_phi = 0.0, a_theta = 0.0, a_b = 0.0;
  for (int b = threadIdx.x; b < nmax; b += kMS) {
    const size_t o = (size_t)b * s + c;
    const double vr = b < d->na_blk ? d->part_rho[o] : 0.0;
    const double vp = b < d->nt_blk ? d->part_phi[o] : 0.0;
    const double vt = b < d->nu_blk ? d->part_theta[o] : 0.0;
    const double vb = want_b && b < d->na_blk ? d->part_b[o] : 0.0;
    a_rho += vr;
    a_phi += vp;
    a_theta += vt;
    a_b += vb;
  }
  const double rho = tree_sum(a_rho, s_buf[0]);
  const double phi = tree_sum(a_phi, s_buf[1]);
  const double theta_sum = tree_sum(a_theta, s_buf[2]);
  const double nb2 = want_b ? tree_sum(a_b, s_buf[3]) : 0.0;
  if (threadIdx.x != 0) return;
  if (k == 0) {
    const double nb = sqrt(nb2);
    st->nb[c] = nb;
    double eta = st->inner_tol;
    if (d->is_f32) {
      const double need = 0.5 * st->tol * (st->tol_abs ? 1.0 : st->nb_out[c]) / st->nu[c];
      if (need > eta) eta = need;
      st->thr[c] = eta * nb;
    } else {
      st->thr[c] = st->tol_abs ? st->tol : st->tol * st->nb_out[c];
    }
  }
  st->rho[c] = rho;
  if (sqrt(rho) <= st->thr[c]) {
    st->status[c] = ST_OK;
    st->done[c] = 1;
    st->beta[c] = st->gamma[c] = 0.0;
    return;
  }
  if (st->k_total[c] >= st->maxit) {
    st->status[c] = ST_NOT_CONVERGED;
    st->done[c] = 1;
    st->beta[c] = st->gamma[c] = 0.0;
    return;
  }
  double beta, gamma;
  if (k == 0) {
    if (!(phi > 0.0)) {
      st->status[c] = ST_BREAKDOWN;
      st->done[c] = 1;
      st->beta[c] = st->gamma[c] = 0.0;
      return;
    }
    beta = 0.0;
    gamma = rho / phi;
  } else {
    const double theta = theta_sum;
    const double sr = sqrt(theta * phi) / rho;
    if (!(sr > 1.0)) {
      st->status[c] = ST_BREAKDOWN;
      st->done[c] = 1;
      st->beta[c] = st->gamma[c] = 0.0;
      return;
    }
    beta = 1.0 / ((sr - 1.0) * (sr + 1.0));
    gamma = (theta / rho) * beta;
  }
  st->beta[c] = beta;
  st->gamma[c] = gamma;
  st->fresh[c] = (k == 0);
  st->k[c] = k + 1;
  st->k_total[c] += 1;
}

// P <- beta P + gamma Y ; X <- X + P (X: inner solution) ; partial theta per column.
template <class Vec>
__global__ __launch_bounds__(kMB) void k_mupdate(const MDesc* __restrict__ d) {
  __shared__ double s_p[kMB];
  const MState* st = d->st;
  if (st->all_done) return;
  const int s = d->s;
  const long long total = (long long)d->n * s;
  Vec* __restrict__ P = static_cast<Vec*>(d->P);
  const Vec* __restrict__ Y = static_cast<const Vec*>(d->Y);
  double* __restrict__ X = d->Xi;
  // kMB threads x 16 elements; s divides kMB (s a power of two here) so each
  // thread stays on one column.  In each of two passes, eight elements'
  // loads go out before any store (the three arrays are distinct), then the
  // elements are updated in order.
  const long long base = (long long)blockIdx.x * kUE;
  const int c = threadIdx.x % s;
  double part = 0.0;
  if (!st->done[c]) {
    const double beta = st->beta[c], gamma = st->gamma[c];
    const bool fresh = st->fresh[c] != 0;
    constexpr int U = 8;  // two passes of eight elements
    for (int h = 0; h < 2; ++h) {
      const long long hb = base + (long long)h * U * kMB + threadIdx.x;
      Vec pv[U], yv[U];
      double xv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const long long o = hb + (long long)u * kMB;
        const bool in = o < total;
        pv[u] = in ? P[o] : Vec(0);
        yv[u] = in ? Y[o] : Vec(0);
        xv[u] = in ? X[o] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const long long o = hb + (long long)u * kMB;
        if (o < total) {
          const double pn = fresh ? gamma * double(yv[u]) : beta * double(pv[u]) + gamma * double(yv[u]);
          const Vec pq = Vec(pn);
          P[o] = pq;
          X[o] = xv[u] + double(pq);
          part += double(pq) * double(pq);
        }
      }
    }
  }
  s_p[threadIdx.x] = part;
  __syncthreads();
  if (threadIdx.x < s) {
    double a = 0.0;
    for (int q = threadIdx.x; q < kMB; q += s) a += s_p[q];
    d->part_theta[(size_t)blockIdx.x * s + threadIdx.x] = a;
  }
}

// Outer step per column: nu = ||b - A x||, finish or (re)start the inner solve.
__global__ __launch_bounds__(kMW) void k_mouter(const MDesc* __restrict__ d) {
  __shared__ double s_tmp[kMW];
  __shared__ double s_rr[64], s_bb[64];
  MState* st = d->st;
  if (st->all_done) return;
  const int s = d->s;
  col_sums(d->part_rho, d->na_blk, s, s_tmp, s_rr);
  col_sums(d->part_b, d->na_blk, s, s_tmp, s_bb);
  const int c = threadIdx.x;
  if (c < s && !st->final_[c]) {
    const double nu = sqrt(s_rr[c]);
    if (st->outer == 0) st->nb_out[c] = sqrt(s_bb[c]);
    const double nbo = st->nb_out[c];
    const double rel = (st->tol_abs || nbo == 0.0) ? nu : nu / nbo;
    st->relres_true[c] = rel;
    bool fin = false;
    int fs = ST_OK;
    if (rel <= st->tol) {
      fin = true;
    } else if (st->outer > 0 && (!d->is_f32 || st->outer >= st->max_outer ||
                                 st->k_total[c] >= st->maxit || st->status[c] == ST_BREAKDOWN ||
                                 !(nu < st->nu[c]))) {
      fin = true;
      fs = !d->is_f32 ? st->status[c] : (st->status[c] == ST_BREAKDOWN ? ST_BREAKDOWN : ST_NOT_CONVERGED);
    }
    if (fin) {
      st->final_[c] = 1;
      st->final_status[c] = fs;
      st->done[c] = 1;
    } else {
      st->nu[c] = d->is_f32 ? nu : 1.0;
      st->k[c] = 0;
      st->done[c] = 0;
      st->status[c] = ST_OK;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int all = 1;
    for (int q = 0; q < s; ++q) all &= st->final_[q];
    st->all_done = all;
    st->outer += 1;
  }
}

// Inner start: R = C = R64 / nu (float32 storage) or R64, partial ||c||^2.
template <class Vec>
__global__ __launch_bounds__(kMB) void k_mstart(const MDesc* __restrict__ d) {
  __shared__ double s_p[kMB];
  const MState* st = d->st;
  if (st->all_done) return;
  const int s = d->s;
  const int W = d->W;
  const int NS = kMB / W, slot = threadIdx.x / W, c = threadIdx.x % W;
  double part = 0.0;
  const bool live = c < s && !st->done[c] && st->k[c] == 0;
  const int row0 = blockIdx.x * kRB, row1 = min(row0 + kRB, d->m);
  if (live) {
    const double inv = d->is_f32 ? 1.0 / st->nu[c] : 1.0;
    Vec* R = static_cast<Vec*>(d->R);
    for (int i = row0 + slot; i < row1; i += NS) {
      const size_t o = (size_t)i * s + c;
      const Vec v = Vec(d->R64[o] * inv);
      R[o] = v;
      part += double(v) * double(v);
    }
  }
  s_p[threadIdx.x] = part;
  __syncthreads();
  if (threadIdx.x < s && live) {
    double a = 0.0;
    for (int q = 0; q < NS; ++q) a += s_p[q * W + threadIdx.x];
    d->part_rho[(size_t)blockIdx.x * s + threadIdx.x] = a;
    d->part_b[(size_t)blockIdx.x * s + threadIdx.x] = a;
  }
}

// X_out += nu * X_inner for columns that just finished an inner solve;
// X_inner <- 0 (float32 storage only).
__global__ __launch_bounds__(256) void k_maxpy(const MDesc* __restrict__ d) {
  const MState* st = d->st;
  if (st->all_done || !d->is_f32) return;
  const int s = d->s;
  const long long total = (long long)d->n * s;
  for (long long o = blockIdx.x * 256LL + threadIdx.x; o < total; o += (long long)gridDim.x * 256) {
    const int c = (int)(o % s);
    if (st->done[c] && !st->final_[c] && st->outer > 0) {
      d->X[o] += st->nu[c] * d->Xi[o];
      d->Xi[o] = 0.0;
    }
  }
}

// column-major (m x ncols) -> row-major (m x s), padding columns zero
__global__ void k_tin(const double* __restrict__ src, int m, int ncols, int s, double* __restrict__ dst) {
  const long long total = (long long)m * s;
  for (long long o = blockIdx.x * 256LL + threadIdx.x; o < total; o += (long long)gridDim.x * 256) {
    const int i = (int)(o / s), c = (int)(o % s);
    dst[o] = c < ncols ? src[(size_t)c * m + i] : 0.0;
  }
}

// row-major (n x s) -> column-major (n x ncols)
__global__ void k_tout(const double* __restrict__ src, int n, int ncols, int s, double* __restrict__ dst) {
  const long long total = (long long)n * ncols;
  for (long long o = blockIdx.x * 256LL + threadIdx.x; o < total; o += (long long)gridDim.x * 256) {
    const int c = (int)(o / n), i = (int)(o % n);
    dst[o] = src[(size_t)i * s + c];
  }
}

// ------------------------------------------------------------------ launchers

static int g256(long long work) {
  long long g = (work + 1023) / 1024;
  return (int)(g < 1 ? 1 : (g > 65536 ? 65536 : g));
}
void launch_transpose_in(const double* src, int m, int ncols, int s, double* dst, hipStream_t st) {
  k_tin<<<g256((long long)m * s), 256, 0, st>>>(src, m, ncols, s, dst);
  PLSS_HIP(hipGetLastError());
}
void launch_transpose_out(const double* src, int n, int ncols, int s, double* dst, hipStream_t st) {
  k_tout<<<g256((long long)n * ncols), 256, 0, st>>>(src, n, ncols, s, dst);
  PLSS_HIP(hipGetLastError());
}

template <class Val, class Vin, class Acc, int MODE>
static void spmm_w(int W, const MDesc* d, int grid, hipStream_t s) {
  switch (W) {
    case 8: k_spmm<Val, Vin, Acc, MODE, 8><<<grid, kMB, 0, s>>>(d); break;
    case 16: k_spmm<Val, Vin, Acc, MODE, 16><<<grid, kMB, 0, s>>>(d); break;
    case 32: k_spmm<Val, Vin, Acc, MODE, 32><<<grid, kMB, 0, s>>>(d); break;
    case 64: k_spmm<Val, Vin, Acc, MODE, 64><<<grid, kMB, 0, s>>>(d); break;
    default: throw InvalidArg{"bad block width"};
  }
}

void launch_spmm(int mode, bool f32, int W, const MDesc* d, int grid, hipStream_t s) {
  if (!f32) {
    if (mode == MMODE_RESID) spmm_w<double, double, double, MMODE_RESID>(W, d, grid, s);
    else if (mode == MMODE_TRANS) spmm_w<double, double, double, MMODE_TRANS>(W, d, grid, s);
    else spmm_w<double, double, double, MMODE_REFINE>(W, d, grid, s);
  } else {
    if (mode == MMODE_RESID) spmm_w<float, float, float, MMODE_RESID>(W, d, grid, s);
    else if (mode == MMODE_TRANS) spmm_w<float, float, float, MMODE_TRANS>(W, d, grid, s);
    else spmm_w<float, double, double, MMODE_REFINE>(W, d, grid, s);
  }
  PLSS_HIP(hipGetLastError());
}

void launch_mstep(const MDesc* d, int ncols, hipStream_t s) { k_mstep<<<ncols, kMS, 0, s>>>(d); }
void launch_mouter(const MDesc* d, hipStream_t s) { k_mouter<<<1, kMW, 0, s>>>(d); }
void launch_mupdate(bool f32, const MDesc* d, int grid, hipStream_t s) {
  if (f32) k_mupdate<float><<<grid, kMB, 0, s>>>(d);
  else k_mupdate<double><<<grid, kMB, 0, s>>>(d);
}
void launch_mstart(bool f32, const MDesc* d, int grid, hipStream_t s) {
  if (f32) k_mstart<float><<<grid, kMB, 0, s>>>(d);
  else k_mstart<double><<<grid, kMB, 0, s>>>(d);
}
void launch_maxpy(const MDesc* d, int grid, hipStream_t s) { k_maxpy<<<grid, 256, 0, s>>>(d); }

}  // namespace plss
