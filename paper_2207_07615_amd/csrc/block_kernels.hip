// Kernels of the block sketch step.
//
// A step appends a block of w sketch columns S_new (the residual r_{k-1}
// and/or identity columns e_i) and applies eq. (pkLong) through the block
// form of the triangular update of Section 2.4.  The history is held as
// mutually orthogonal projected blocks Z_j with Delta_j = Z_jᵀ Z_j = L_j L_jᵀ
// and the products A Z_j (the block analogue of Section 7's P, AP, Θ), so
// with Y_new = Aᵀ S_new:
//   W = Zᵀ Y_new          identity column i: row i of A Z; residual: (A Z)ᵀ r
//   U = L^{-1} W, C = L^{-T} U                  (L block-diagonal)
//   Delta = Y_newᵀ Y_new - Uᵀ U                 (Schur complement, w x w)
//   keep the columns whose pivot in block order exceeds 1e-14 ||y_j||^2
//   c' = Delta^{-1} sigma, sigma = S_newᵀ r      (on the kept columns)
//   Z_new = Y_new - Z C                          (MFMA, the dense contraction)
//   x += Z_new c', A Z_new, r -= (A Z_new) c'
//
// Launch sequence of one step (every kernel returns early once the solve is
// done, and the update kernels when the block keeps no column):
//   [residual column: k_spmv<TRANS> (y = Aᵀ r, phi), k_bgemvt (partial (A Z)ᵀ r)]
//   k_blk_prep, k_blk_zgemm, k_blk_scatter, k_blk_spmm, k_blk_fin
#include "block.hpp"
#include "kernels.hpp"

namespace plss {

namespace {
constexpr int kPB = 1024;  // threads of the one-workgroup kernels
typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double wsum(double v) {
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
  for (int q = 1; q < kPB / 64; ++q) t += s_tmp[q];
  __syncthreads();
  return t;
}

__device__ double bsum_array(const double* __restrict__ a, int n, double* s_tmp) {
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += kPB) v += a[i];
  return bsum(v, s_tmp);
}

// a_iᵀ a_l of two sparse rows with ascending column indices: entries
// [p, pe) and [q, qe) of (idx, val)
__device__ double row_dot(const int* idx, const double* val, int p, int pe, int q, int qe) {
  double g = 0.0;
  while (p < pe && q < qe) {
    const int c1 = idx[p], c2 = idx[q];
    if (c1 == c2) {
      g += val[p] * val[q];
      ++p;
      ++q;
    } else if (c1 < c2) {
      ++p;
    } else {
      ++q;
    }
  }
  return g;
}
}  // namespace

// Partial (A Z)ᵀ r over a chunk of kBRows rows per workgroup: part_w[k * wblk
// + chunk] for the K history columns.  A thread takes one column of a row
// slot (consecutive threads read consecutive columns of a row of A Z); the
// slots are added in slot order.
__global__ __launch_bounds__(kPB) void k_bgemvt(const Desc* __restrict__ d, const BlkDesc* __restrict__ bd) {
  __shared__ double s_acc[kPB];
  const State* st = d->st;
  const BlkState* bs = bd->bs;
  if (st->final_done || st->done) return;
  const int K = (int)bs->K;
  if (K == 0) return;
  int kc = 64;
  while (kc < K) kc <<= 1;
  const int slots = kPB / kc;
  const int k = threadIdx.x % kc, slot = threadIdx.x / kc;
  const int r0 = blockIdx.x * kBRows;
  const int r1 = min(r0 + kBRows, d->m);
  const double* __restrict__ r = static_cast<const double*>(d->r);
  const int kcap = bd->kcap;
  double acc = 0.0;
  if (k < K)
    for (int row = r0 + slot; row < r1; row += slots) acc += bd->AZh[(size_t)row * kcap + k] * r[row];
  s_acc[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x < K) {
    double a = s_acc[threadIdx.x];
    for (int q = 1; q < slots; ++q) a += s_acc[q * kc + threadIdx.x];
    bd->part_w[(size_t)threadIdx.x * bd->wblk + blockIdx.x] = a;
  }
}

// Block scalars (one workgroup): the block's rows, history clear at the
// capacity, W, U, C, Y_newᵀ Y_new, Delta, the kept columns (pivoted Cholesky
// in block order), c' = Delta^{-1} sigma.
__global__ __launch_bounds__(kPB) void k_blk_prep(const Desc* __restrict__ d, const BlkDesc* __restrict__ bd) {
  __shared__ int s_rows[kBW];
  __shared__ double s_sig[kBW];
  __shared__ double s_G[kBW][kBW];
  __shared__ double s_D[kBW][kBW];
  __shared__ double s_L[kBW][kBW];
  __shared__ int s_keep[kBW];
  __shared__ int s_w, s_K, s_nblk, s_nk, s_stop;
  __shared__ double s_red[kPB / 64];
  // the block's rows of A, staged for the sparse Gram entries when they fit
  constexpr int kStage = 3072;
  __shared__ int s_ridx[kStage];
  __shared__ double s_rval[kStage];
  __shared__ int s_roff[kBW + 1];
  State* st = d->st;
  BlkState* bs = bd->bs;
  if (st->final_done || st->done) return;
  const int m = d->m, res = bd->residual, kcap = bd->kcap;
  if (threadIdx.x == 0) {
    const long long pos = bs->pos;
    const int nrow = (int)min((long long)bd->block, (long long)m - pos);
    const int w = res + nrow;
    long long K = bs->K, nb = bs->nblk;
    if (K + w > bs->cap) {
      K = 0;
      nb = 0;
    }
    bs->K = K;
    bs->nblk = nb;
    bs->nrow = nrow;
    bs->pass_end = (pos + nrow >= m) ? 1 : 0;
    s_w = w;
    s_K = (int)K;
    s_nblk = (int)nb;
    s_stop = 0;
  }
  __syncthreads();
  const int w = s_w, K = s_K, nblk = s_nblk;
  const double* __restrict__ r = static_cast<const double*>(d->r);
  const double* __restrict__ av = static_cast<const double*>(d->a_val);
  if (threadIdx.x < w) {
    const int l = threadIdx.x;
    if (l < res) {
      s_rows[l] = -1;
      s_sig[l] = st->rho;
    } else {
      const int i = bd->perm[bs->pos + l - res];
      s_rows[l] = i;
      s_sig[l] = r[i];
    }
  }
  const double phi = res ? bsum_array(d->part_phi, d->t_ntiles, s_red) : 0.0;  // y_rᵀ y_r
  __syncthreads();
  if (threadIdx.x == 0) {
    int o = 0;
    for (int l = 0; l < w; ++l) {
      s_roff[l] = o;
      if (l >= res) o += d->a_ptr[s_rows[l] + 1] - d->a_ptr[s_rows[l]];
    }
    s_roff[w] = o;
  }
  __syncthreads();
  const bool staged = s_roff[w] <= kStage;
  if (staged) {
    for (int l = res; l < w; ++l) {
      const int b0 = d->a_ptr[s_rows[l]], len = s_roff[l + 1] - s_roff[l];
      for (int e = threadIdx.x; e < len; e += kPB) {
        s_ridx[s_roff[l] + e] = d->a_idx[b0 + e];
        s_rval[s_roff[l] + e] = av[b0 + e];
      }
    }
  }
  __syncthreads();
  // W = Zᵀ Y_new into Ug (row k = history column k)
  for (int e = threadIdx.x; e < K * w; e += kPB) {
    const int k = e / w, l = e % w;
    double v = 0.0;
    if (l < res) {
      const double* pw = bd->part_w + (size_t)k * bd->wblk;
      const int nb = bd->wblk;
      double t[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      int b = 0;
      for (; b + 8 <= nb; b += 8) {
#pragma unroll
        for (int u = 0; u < 8; ++u) t[u] += pw[b + u];
      }
      for (; b < nb; ++b) t[0] += pw[b];
      v = ((t[0] + t[1]) + (t[2] + t[3])) + ((t[4] + t[5]) + (t[6] + t[7]));
    } else {
      v = bd->AZh[(size_t)s_rows[l] * kcap + k];
    }
    bd->Ug[(size_t)k * kBW + l] = v;
  }
  __syncthreads();
  // U = L^{-1} W and C = L^{-T} U, one (history block, column) per thread
  for (int e = threadIdx.x; e < nblk * w; e += kPB) {
    const int j = e / w, l = e % w;
    const int o = bd->bo[j], wj = bd->wh[j];
    const double* L = bd->Lh + (size_t)j * kBW * kBW;
    // loops over the full width with the block's width as a predicate keep
    // u in registers
    double u[kBW];
#pragma unroll
    for (int a = 0; a < kBW; ++a) {
      double v = a < wj ? bd->Ug[(size_t)(o + a) * kBW + l] : 0.0;
#pragma unroll
      for (int c = 0; c < a; ++c) v -= L[a * kBW + c] * u[c];
      u[a] = a < wj ? v / L[a * kBW + a] : 0.0;
    }
#pragma unroll
    for (int a = 0; a < kBW; ++a)
      if (a < wj) bd->Ug[(size_t)(o + a) * kBW + l] = u[a];
#pragma unroll
    for (int a = kBW - 1; a >= 0; --a) {
      double v = u[a];
#pragma unroll
      for (int c = a + 1; c < kBW; ++c) v -= L[c * kBW + a] * u[c];
      u[a] = a < wj ? v / L[a * kBW + a] : 0.0;
    }
#pragma unroll
    for (int a = 0; a < kBW; ++a)
      if (a < wj) bd->Cg[(size_t)(o + a) * kBW + l] = u[a];
  }
  // G0 = Y_newᵀ Y_new: phi, y_rᵀ a_i, a_iᵀ a_l (upper triangle)
  for (int e = threadIdx.x; e < w * w; e += kPB) {
    const int a = e / w, l = e % w;
    if (a > l) continue;
    double g;
    if (l < res) {
      g = phi;
    } else if (a < res) {
      const double* __restrict__ y = static_cast<const double*>(d->y);
      g = 0.0;
      if (staged) {
        for (int q = s_roff[l]; q < s_roff[l + 1]; ++q) g += y[s_ridx[q]] * s_rval[q];
      } else {
        const int i = s_rows[l];
        for (int q = d->a_ptr[i]; q < d->a_ptr[i + 1]; ++q) g += y[d->a_idx[q]] * av[q];
      }
    } else if (staged) {
      g = row_dot(s_ridx, s_rval, s_roff[a], s_roff[a + 1], s_roff[l], s_roff[l + 1]);
    } else {
      const int i = s_rows[a], k2 = s_rows[l];
      g = row_dot(d->a_idx, av, d->a_ptr[i], d->a_ptr[i + 1], d->a_ptr[k2], d->a_ptr[k2 + 1]);
    }
    s_G[a][l] = g;
    s_G[l][a] = g;
  }
  __syncthreads();
  // Delta = G0 - Uᵀ U: one wave per entry (upper triangle), its lanes over
  // the history columns, a fixed-order wave sum
  {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int e = wv; e < w * w; e += kPB / 64) {
      const int a = e / w, l = e % w;
      if (a > l) continue;
      double v = 0.0;
      for (int k = lane; k < K; k += 64) v += bd->Ug[(size_t)k * kBW + a] * bd->Ug[(size_t)k * kBW + l];
      v = wsum(v);
      if (lane == 0) {
        const double dd = s_G[a][l] - v;
        s_D[a][l] = dd;
        s_D[l][a] = dd;
      }
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int nk = 0;
    for (int j = 0; j < w; ++j) {
      double z[kBW];
      double zz = 0.0;
#pragma unroll
      for (int a = 0; a < kBW; ++a) {
        double v = a < nk ? s_D[s_keep[a]][j] : 0.0;
#pragma unroll
        for (int c = 0; c < a; ++c) v -= s_L[a][c] * z[c];
        z[a] = a < nk ? v / s_L[a][a] : 0.0;
        zz += z[a] * z[a];
      }
      const double piv = s_D[j][j] - zz;
      if (piv > 1e-14 * s_G[j][j]) {
#pragma unroll
        for (int c = 0; c < kBW; ++c)
          if (c < nk) s_L[nk][c] = z[c];
        s_L[nk][nk] = sqrt(piv);
        s_keep[nk++] = j;
      } else if (j < res) {
        st->status = ST_BREAKDOWN;
        st->done = 1;
        s_stop = 1;
        break;
      }
    }
    s_nk = nk;
    if (!s_stop) {
      bs->skip = nk == 0 ? 1 : 0;
      bs->wk = nk;
      bs->res_kept = (nk > 0 && res && s_keep[0] == 0) ? 1 : 0;
      // c' = (L Lᵀ)^{-1} sigma on the kept columns
      double t[kBW];
#pragma unroll
      for (int a = 0; a < kBW; ++a) {
        double v = a < nk ? s_sig[s_keep[a]] : 0.0;
#pragma unroll
        for (int c = 0; c < a; ++c) v -= s_L[a][c] * t[c];
        t[a] = a < nk ? v / s_L[a][a] : 0.0;
      }
#pragma unroll
      for (int a = kBW - 1; a >= 0; --a) {
        double v = t[a];
#pragma unroll
        for (int c = a + 1; c < kBW; ++c) v -= (c < nk ? s_L[c][a] : 0.0) * t[c];
        t[a] = a < nk ? v / s_L[a][a] : 0.0;
      }
      for (int q = 0; q < kBW; ++q) {
        bs->cp[q] = q < nk ? t[q] : 0.0;
        bs->rows[q] = q < nk ? s_rows[s_keep[q]] : -1;
      }
      if (nk > 0) {
        double* L = bd->Lh + (size_t)nblk * kBW * kBW;
        for (int a = 0; a < kBW; ++a)
          for (int c = 0; c < kBW; ++c) L[a * kBW + c] = (a < nk && c <= a) ? s_L[a][c] : 0.0;
        bd->bo[nblk] = K;
        bd->wh[nblk] = nk;
      }
    }
  }
  __syncthreads();
  if (s_stop || s_nk == 0) return;
  // C restricted to the kept columns (in order), zero elsewhere; rows up to
  // K rounded to 4 (the contraction's last chunk) zero past K
  const int nk = s_nk;
  const int K4 = (K + 3) & ~3;
  for (int k = threadIdx.x; k < K4; k += kPB) {
    double row[kBW];
    for (int l = 0; l < kBW; ++l) row[l] = (k < K && l < w) ? bd->Cg[(size_t)k * kBW + l] : 0.0;
    for (int q = 0; q < kBW; ++q) bd->Cg[(size_t)k * kBW + q] = q < nk ? row[s_keep[q]] : 0.0;
  }
}

// Z_new = Y_new - Z C for 16 rows per wave (v_mfma_f64_16x16x4f64 over the
// history columns, 4 per instruction): the dense part of Y_new is the
// residual column y_r; the identity columns' sparse rows are added by
// k_blk_scatter.  Epilogue: Z_new into the history, x += (dense part of
// Z_new) c'.
__global__ __launch_bounds__(256) void k_blk_zgemm(const Desc* __restrict__ d, const BlkDesc* __restrict__ bd) {
  const State* st = d->st;
  const BlkState* bs = bd->bs;
  if (st->final_done || st->done || bs->skip) return;
  const int lane = threadIdx.x & 63;
  const int n = d->n;
  const int n0 = (blockIdx.x * 4 + (threadIdx.x >> 6)) * 16;
  if (n0 >= n) return;
  const int K = (int)bs->K, kcap = bd->kcap, wk = bs->wk;
  // operands: A = Z (16 rows x 4 history columns): lane -> (row lane % 16,
  // column lane / 16); B = C (4 x 16): lane -> (row lane / 16, column lane % 16)
  const int ar = n0 + (lane & 15);
  const int ak = lane >> 4;
  const double* __restrict__ zrow = bd->Zh + (size_t)min(ar, n - 1) * kcap;
  const double* __restrict__ cg = bd->Cg + (lane & 15);
  d4 acc = {0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < K; k0 += 4) {
    const int k = k0 + ak;
    const double a = (ar < n && k < K) ? zrow[k] : 0.0;
    const double b = cg[(size_t)k * kBW];
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  }
  // result: item i of a lane -> (row lane / 16 + 4 i, column lane % 16)
  const int c = lane & 15;
  const int rbase = n0 + (lane >> 4);
  const bool res_col = bs->res_kept && c == 0;
  const double cpc = c < wk ? bs->cp[c] : 0.0;
  const double* __restrict__ y = static_cast<const double*>(d->y);
  double* zn = bd->Zh + K;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int row = rbase + 4 * i;
    const bool in = row < n && c < wk;
    const double z = in ? (res_col ? y[row] : 0.0) - acc[i] : 0.0;
    if (in) zn[(size_t)row * kcap + c] = z;
    double pd = z * cpc;
    pd += __shfl_xor(pd, 1, 64);
    pd += __shfl_xor(pd, 2, 64);
    pd += __shfl_xor(pd, 4, 64);
    pd += __shfl_xor(pd, 8, 64);
    if (c == 0 && row < n) d->x[row] += pd;
  }
}

// The identity columns' rows of A into Z_new (column q: row i of A, distinct
// columns j) and x += c'_q a_q, one kept column after the other (a barrier
// between them: two rows may share a column j).
__global__ __launch_bounds__(kPB) void k_blk_scatter(const Desc* __restrict__ d, const BlkDesc* __restrict__ bd) {
  const State* st = d->st;
  const BlkState* bs = bd->bs;
  if (st->final_done || st->done || bs->skip) return;
  const int K = (int)bs->K, kcap = bd->kcap, wk = bs->wk;
  const double* __restrict__ av = static_cast<const double*>(d->a_val);
  double* zn = bd->Zh + K;
  for (int q = bs->res_kept; q < wk; ++q) {
    const int i = bs->rows[q];
    const double cq = bs->cp[q];
    for (int e = d->a_ptr[i] + threadIdx.x; e < d->a_ptr[i + 1]; e += kPB) {
      const int j = d->a_idx[e];
      const double v = av[e];
      zn[(size_t)j * kcap + q] += v;
      d->x[j] += cq * v;
    }
    __syncthreads();
  }
}

// A Z_new (LPR lanes per row, lane q = column q: the row's entries gather
// rows of Z_new) into the history; r -= (A Z_new) c'; partial rho per
// workgroup.
template <int LPR>
__global__ __launch_bounds__(256) void k_blk_spmm(const Desc* __restrict__ d, const BlkDesc* __restrict__ bd) {
  __shared__ double s_red[4];
  const State* st = d->st;
  const BlkState* bs = bd->bs;
  if (st->final_done || st->done || bs->skip) return;
  const int m = d->m, K = (int)bs->K, kcap = bd->kcap, wk = bs->wk;
  const int q = threadIdx.x % LPR;
  const int i = blockIdx.x * (256 / LPR) + threadIdx.x / LPR;
  const double* __restrict__ zn = bd->Zh + K;
  const double* __restrict__ av = static_cast<const double*>(d->a_val);
  double acc = 0.0;
  if (i < m && q < wk) {
    const int e1 = d->a_ptr[i + 1];
    int e = d->a_ptr[i];
    // eight entries at a time: their indices, values and gathered rows in
    // flight before the first product (the sum keeps the entry order)
    for (; e + 8 <= e1; e += 8) {
      int c[8];
      double v[8], zv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        c[u] = d->a_idx[e + u];
        v[u] = av[e + u];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) zv[u] = zn[(size_t)c[u] * kcap + q];
#pragma unroll
      for (int u = 0; u < 8; ++u) acc += v[u] * zv[u];
    }
    for (; e < e1; ++e) acc += av[e] * zn[(size_t)d->a_idx[e] * kcap + q];
    bd->AZh[(size_t)i * kcap + K + q] = acc;
  }
  double rs = acc * (q < wk ? bs->cp[q] : 0.0);
#pragma unroll
  for (int off = 1; off < LPR; off <<= 1) rs += __shfl_xor(rs, off, 64);
  double part = 0.0;
  if (i < m && q == 0) {
    double* r = static_cast<double*>(d->r);
    const double rn = r[i] - rs;
    r[i] = rn;
    part = rn * rn;
  }
  part = wsum(part);
  if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = part;
  __syncthreads();
  if (threadIdx.x == 0) bd->part_r[blockIdx.x] = (s_red[0] + s_red[1]) + (s_red[2] + s_red[3]);
}

// Close the step: rho, history bookkeeping, residual history, stop test.
__global__ __launch_bounds__(kPB) void k_blk_fin(const Desc* __restrict__ d, const BlkDesc* __restrict__ bd) {
  __shared__ double s_red[kPB / 64];
  State* st = d->st;
  BlkState* bs = bd->bs;
  if (st->final_done || st->done) return;
  const bool skip = bs->skip != 0;
  const double rho = skip ? 0.0 : bsum_array(bd->part_r, bd->nparts, s_red);
  if (threadIdx.x != 0) return;
  bs->steps += 1;
  st->col = bs->steps;
  const int pass_end = bs->pass_end;
  bs->pos = pass_end ? 0 : bs->pos + bs->nrow;
  if (!skip) {
    bs->nblk += 1;
    bs->K += bs->wk;
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
  if (bs->steps >= bs->max_steps) {
    st->status = ST_NOT_CONVERGED;
    st->done = 1;
    return;
  }
  if (pass_end) {
    bs->nblk = 0;
    bs->K = 0;
  }
}

// ------------------------------------------------------------------ launchers

void launch_block_step(const Desc* d, const BlkDesc* bd, bool residual, int lpr, int VT, const int2* tlist,
                       int nt, int n, int wblk, int nparts, hipStream_t s) {
  if (residual) {
    launch_spmv(MODE_TRANS, false, VT, d, tlist, nt, 1, s);
    k_bgemvt<<<wblk, kPB, 0, s>>>(d, bd);
  }
  k_blk_prep<<<1, kPB, 0, s>>>(d, bd);
  k_blk_zgemm<<<(n + 63) / 64, 256, 0, s>>>(d, bd);
  k_blk_scatter<<<1, kPB, 0, s>>>(d, bd);
  switch (lpr) {
    case 4: k_blk_spmm<4><<<nparts, 256, 0, s>>>(d, bd); break;
    case 8: k_blk_spmm<8><<<nparts, 256, 0, s>>>(d, bd); break;
    default: k_blk_spmm<16><<<nparts, 256, 0, s>>>(d, bd); break;
  }
  k_blk_fin<<<1, kPB, 0, s>>>(d, bd);
  PLSS_HIP(hipGetLastError());
}

}  // namespace plss
