// Device kernels of the PLSS hot path for gfx950 (CDNA4, wave64).
//
// Per inner iteration of Algorithm 1 (W = diag(1/wi) or I):
//   k_spmv<RESID>  r <- r - A p, partial rho             (one workgroup per CSR tile)
//   k_spmv<TRANS>  y <- Aᵀ r,   partial phi             (one workgroup per CSC tile)
//   k_step         rho, phi, theta; stop test; beta, gamma (one workgroup per system)
//   k_update       p <- beta p + gamma W y; x <- x + p; partial theta
// Outer (refinement / start / finish) sequence:
//   k_axpy_out     x <- x + nu d (float32 storage only)
//   k_spmv<REFINE> r64 <- b - A x in float64
//   k_outer        nu = ||r64||; finish or (re)start the inner solve
//   k_start        r <- c = r64 / nu (or b), partial rho, partial ||c||^2
//
// Every reduction is a fixed-order tree over fixed tiles: results do not
// depend on scheduling or on which other systems share the launch.
#include "kernels.hpp"

#include <climits>

namespace plss {

// ------------------------------------------------------------------ reductions

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over the workgroup in a fixed order; the result is valid in every thread.
template <class T>
__device__ __forceinline__ T block_sum(T v, T* s_tmp) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) s_tmp[w] = v;
  __syncthreads();
  T t = s_tmp[0];
#pragma unroll
  for (int q = 1; q < kWaves; ++q) t += s_tmp[q];
  return t;
}

// Fixed-order sum of a[0..n) by one workgroup (valid in every thread).
__device__ double block_sum_array(const double* __restrict__ a, int n, double* s_tmp) {
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += kWG) v += a[i];
  return block_sum(v, s_tmp);
}

// Same with 1024 threads (16 waves), 4 independent loads per thread in flight.
constexpr int kRW = 1024;
__device__ double big_sum_array(const double* __restrict__ a, int n, double* s_tmp) {
  double v0 = 0.0, v1 = 0.0, v2 = 0.0, v3 = 0.0;
  int i = threadIdx.x;
  for (; i + 3 * kRW < n; i += 4 * kRW) {
    v0 += a[i];
    v1 += a[i + kRW];
    v2 += a[i + 2 * kRW];
    v3 += a[i + 3 * kRW];
  }
  for (; i < n; i += kRW) v0 += a[i];
  double v = (v0 + v1) + (v2 + v3);
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) s_tmp[w] = v;
  __syncthreads();
  double t = s_tmp[0];
  for (int q = 1; q < kRW / 64; ++q) t += s_tmp[q];
  return t;
}

// Fixed-order sums of four arrays by one workgroup of kRW threads, their
// loads issued together (valid in thread 0): thread t adds elements
// t, t + kRW, t + 2 kRW, ... of each array in turn, then the workgroup adds
// the threads' sums wave by wave.  s_tmp: 4 x 16 doubles.
__device__ double4 big_sums4(const double* __restrict__ a0, int n0, const double* __restrict__ a1, int n1,
                             const double* __restrict__ a2, int n2, const double* __restrict__ a3, int n3,
                             double* s_tmp) {
  const int nmax = max(max(n0, n1), max(n2, n3));
  double v0 = 0.0, v1 = 0.0, v2 = 0.0, v3 = 0.0;
  // a loop taken at least once, so the arrays' addresses are not waited
  // for behind a test of the counts
  int i = threadIdx.x;
  do {
    const double e0 = i < n0 ? a0[i] : 0.0;
    const double e1 = i < n1 ? a1[i] : 0.0;
    const double e2 = i < n2 ? a2[i] : 0.0;
    const double e3 = i < n3 ? a3[i] : 0.0;
    v0 += e0;
    v1 += e1;
    v2 += e2;
    v3 += e3;
    i += kRW;
  } while (i - (int)threadIdx.x < nmax);
  v0 = wave_sum(v0);
  v1 = wave_sum(v1);
  v2 = wave_sum(v2);
  v3 = wave_sum(v3);
  constexpr int W = kRW / 64;
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    s_tmp[w] = v0;
    s_tmp[W + w] = v1;
    s_tmp[2 * W + w] = v2;
    s_tmp[3 * W + w] = v3;
  }
  __syncthreads();
  // thread a adds array a's wave sums in wave order
  if (threadIdx.x < 4) {
    const double* t = s_tmp + threadIdx.x * W;
    double r = t[0];
    for (int q = 1; q < W; ++q) r += t[q];
    s_tmp[4 * W + threadIdx.x] = r;
  }
  __syncthreads();
  return make_double4(s_tmp[4 * W], s_tmp[4 * W + 1], s_tmp[4 * W + 2], s_tmp[4 * W + 3]);
}

// Exclusive segmented scan across the workgroup of (f, v) pairs, where a
// set flag starts a new segment after the element:
//   incl_j = f_j ? v_j : incl_{j-1} + v_j,  result_j = incl_{j-1} (0 for j = 0).
template <class T>
__device__ __forceinline__ T seg_scan_excl(int f, T v, T* s_v, int* s_f) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  T sv = v;
  int sf = f;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    T ov = __shfl_up(sv, off, 64);
    int of = __shfl_up(sf, off, 64);
    if (lane >= off) {
      if (!sf) sv = ov + sv;
      sf |= of;
    }
  }
  if (lane == 63) {
    s_v[w] = sv;
    s_f[w] = sf;
  }
  __syncthreads();
  T pv = T(0);
  for (int q = 0; q < w; ++q) pv = s_f[q] ? s_v[q] : pv + s_v[q];
  T incl = sf ? sv : pv + sv;
  T ex = __shfl_up(incl, 1, 64);
  if (lane == 0) ex = pv;
  return ex;
}

// ------------------------------------------------------------------ phase guards

// phase: the inner iteration runs while final_done == 0 and done == 0.
// The state's fields are all read before any is tested (no short-circuit),
// so their loads go out together.
template <int MODE>
__device__ __forceinline__ bool spmv_skip(const State* st) {
  if (MODE == MODE_PLAIN) return false;
  const int fd = st->final_done, dn = st->done;
  if (MODE == MODE_REFINE) return (fd | (dn == 0)) != 0;
  if (MODE == MODE_TRANSB || MODE == MODE_TRANS) return (fd | dn) != 0;
  if (MODE == MODE_RESID) {
    const long long k = st->k;
    return ((fd | dn) != 0) | (k == 0);
  }
  if (MODE == MODE_AP || MODE == MODE_APB) {
    const int sk = st->skip;
    return (fd | dn | sk) != 0;
  }
  return (fd | dn) != 0;
}

// ------------------------------------------------------------------ tile SpMV

// Wave-level segmented scan (exclusive) of (f, v) pairs over the 64 lanes,
// with the same combine rule as seg_scan_excl.
template <class T>
__device__ __forceinline__ T wave_seg_scan_excl(int f, T v) {
  const int lane = threadIdx.x & 63;
  T sv = v;
  int sf = f;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    T ov = __shfl_up(sv, off, 64);
    int of = __shfl_up(sf, off, 64);
    if (lane >= off) {
      if (!sf) sv = ov + sv;
      sf |= of;
    }
  }
  T ex = __shfl_up(sv, 1, 64);
  if (lane == 0) ex = T(0);
  return ex;
}

// wave maximum of an int (every lane gets it)
__device__ __forceinline__ int wave_max_i(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
  return v;
}

// rows of at most this many entries: a tile whose rows are all this short is
// summed one row per lane
constexpr int kShortRow = 16;

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One launch covers a list of (system, group) pairs; a group is 4
// consecutive wave tiles of one system, one per wave of the workgroup.  A
// wave tile holds at most 64*V stored entries and at most 64*V rows, or a
// single longer row.  Short-row tiles stage products in wave-private LDS
// and split them into rows with a segmented scan; long rows are summed in
// registers by the whole wave.  Each wave's tile sum order and each group's
// partial are fixed by the matrix alone.
template <class Val, class Vin, class Acc, int MODE, int V>
__global__ __launch_bounds__(kWG) void k_spmv(const Desc* __restrict__ D,
                                              const int2* __restrict__ list, int transpose) {
  constexpr int TW = 64 * V;
  __shared__ Acc s_prod[kWaves][TW];        // products, then row sums
  __shared__ int s_off[kWaves][TW + 1];     // row offsets of the tile
  __shared__ double s_wp[2][kWaves];

  constexpr bool kBlk = MODE == MODE_TRANSB || MODE == MODE_APB;  // one block of an XCD-interleaved list
  const int2 ent = list[blockIdx.x];
  if (kBlk && ent.y < 0) return;  // padding of the XCD-interleaved list
  const Desc* d = D + ent.x;
  const State* st = d->st;

  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const bool tr = (MODE == MODE_TRANS) || (MODE == MODE_PLAIN && transpose);
  const int blk = kBlk ? (ent.y >> 24) : 0;
  const int gi = kBlk ? (ent.y & 0xFFFFFF) : ent.y;
  const int* __restrict__ ptr =
      MODE == MODE_TRANSB ? d->tb_ptr[blk] : (MODE == MODE_APB ? d->cb_ptr[blk] : (tr ? d->t_ptr : d->a_ptr));
  const int* __restrict__ idx =
      MODE == MODE_TRANSB ? d->tb_idx[blk] : (MODE == MODE_APB ? d->cb_idx[blk] : (tr ? d->t_idx : d->a_idx));
  const Val* __restrict__ val = static_cast<const Val*>(
      MODE == MODE_TRANSB ? d->tb_val[blk] : (MODE == MODE_APB ? d->cb_val[blk] : (tr ? d->t_val : d->a_val)));
  const int4* __restrict__ wtd =
      MODE == MODE_TRANSB ? d->tb_wtd[blk] : (MODE == MODE_APB ? d->cb_wtd[blk] : (tr ? d->t_wtd : d->a_wtd));
  // this wave's tile, read beside the state's flags (both before either is used)
  const int4 wd = wtd[gi * kWaves + w];
  if (spmv_skip<MODE>(st)) return;

  const Vin* __restrict__ xin;
  if (MODE == MODE_RESID) xin = static_cast<const Vin*>(d->p);
  else if (MODE == MODE_TRANS || MODE == MODE_TRANSB) xin = static_cast<const Vin*>(d->r);
  else if (MODE == MODE_REFINE) xin = reinterpret_cast<const Vin*>(d->xo);
  else if (MODE == MODE_PLAIN) xin = static_cast<const Vin*>(d->p);
  else xin = reinterpret_cast<const Vin*>(d->P + (size_t)st->kh * d->n);  // AP, APB: the new column of P

  double part = 0.0, part2 = 0.0;

  // Row epilogue: the fused vector work of each mode.
  auto epi = [&](int i, Acc s) {
    if (MODE == MODE_RESID) {
      using Vec = Vin;
      Vec* r = static_cast<Vec*>(d->r);
      Acc rn = Acc(r[i]) - s;
      r[i] = Vec(rn);
      part += double(rn) * double(rn);
    } else if (MODE == MODE_AP) {
      double* r = static_cast<double*>(d->r);
      double rn = r[i] - double(s);
      r[i] = rn;
      d->AP[(size_t)st->kh * d->m + i] = double(s);
      part += rn * rn;
    } else if (MODE == MODE_TRANS) {
      using Vec = Vin;
      static_cast<Vec*>(d->y)[i] = Vec(s);
      double ds = double(Vec(s));
      part += d->wi ? ds * ds / d->wi[i] : ds * ds;
    } else if (MODE == MODE_TRANSB) {
      using Vec = Vin;
      static_cast<Vec*>(d->ypart)[(size_t)blk * d->n + i] = Vec(s);
    } else if (MODE == MODE_APB) {
      d->appart[(size_t)blk * d->m + i] = double(s);
    } else if (MODE == MODE_REFINE) {
      double bi = d->b[i];
      double ri = bi - double(s);
      d->r64[i] = ri;
      part += ri * ri;
      part2 += bi * bi;
    } else {
      d->r64[i] = double(s);
    }
  };

  if (wd.y > wd.x) {  // a wave past the group's last tile has none
    const int r0 = wd.x, r1 = wd.y;
    const int e0 = wd.z;
    const int nr = r1 - r0, ne = wd.w - wd.z;
    if (ne > TW) {
      // one long row: the wave strides over it, 8 entries per lane in flight
      constexpr int U = 8;
      Acc acc = Acc(0);
      int e = lane;
      for (; e + 64 * (U - 1) < ne; e += 64 * U) {
        int c[U];
        Val v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          c[u] = __builtin_nontemporal_load(&idx[e0 + e + 64 * u]);
          v[u] = __builtin_nontemporal_load(&val[e0 + e + 64 * u]);
        }
        Acc xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) xv[u] = Acc(xin[c[u]]);
#pragma unroll
        for (int u = 0; u < U; ++u) acc += Acc(v[u]) * xv[u];
      }
      for (; e < ne; e += 64)
        acc += Acc(__builtin_nontemporal_load(&val[e0 + e])) *
               Acc(xin[__builtin_nontemporal_load(&idx[e0 + e])]);
      acc = wave_sum(acc);
      if (lane == 0) epi(r0, acc);
    } else {
      Acc* sp = s_prod[w];
      int* so = s_off[w];
      for (int i = lane; i <= nr; i += 64) so[i] = ptr[r0 + i] - e0;
      if (ne > 0) {
        // all V index / value loads, then all V gathers, in flight together;
        // slots past the tile's end reload its last entry and store nothing
        int c[V];
        Val v[V];
#pragma unroll
        for (int u = 0; u < V; ++u) {
          const int e = min(u * 64 + lane, ne - 1);
          c[u] = __builtin_nontemporal_load(&idx[e0 + e]);
          v[u] = __builtin_nontemporal_load(&val[e0 + e]);
        }
        Acc xv[V];
#pragma unroll
        for (int u = 0; u < V; ++u) xv[u] = Acc(xin[c[u]]);
#pragma unroll
        for (int u = 0; u < V; ++u) {
          const int e = u * 64 + lane;
          if (e < ne) sp[e] = Acc(v[u]) * xv[u];
        }
      }
      wave_lds_sync();
      // the tile's longest row (the same value in every lane)
      int ml = 0;
      for (int i = lane; i < nr; i += 64) ml = max(ml, so[i + 1] - so[i]);
      ml = wave_max_i(ml);
      if (ml <= kShortRow) {
        // short rows: lane l sums rows l, l + 64, ... from their products, in
        // order; no search for the lane's first row and no scan across lanes
        for (int i = lane; i < nr; i += 64) {
          const int e1 = so[i + 1];
          Acc a = Acc(0);
          for (int e = so[i]; e < e1; ++e) a += sp[e];
          epi(r0 + i, a);
        }
      } else {
      // each lane sums V consecutive products, split at row ends
      const int c0 = lane * V;
      Acc acc = Acc(0);
      Acc endv[V];
      int endr[V];
#pragma unroll
      for (int q = 0; q < V; ++q) endr[q] = -1;
      if (c0 < ne) {
        int lo = 0, hi = nr;  // so[lo] <= c0 < so[hi]
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (so[mid] <= c0) lo = mid;
          else hi = mid;
        }
        int rr = lo;
        int rend = so[rr + 1];
#pragma unroll
        for (int q = 0; q < V; ++q) {
          const int e = c0 + q;
          if (e < ne) {
            acc += sp[e];
            if (e + 1 == rend) {
              endr[q] = rr;
              endv[q] = acc;
              acc = Acc(0);
              ++rr;
              while (rr < nr && so[rr + 1] == so[rr]) ++rr;
              rend = (rr < nr) ? so[rr + 1] : INT_MAX;
            }
          }
        }
      }
      int has_end = 0;
#pragma unroll
      for (int q = 0; q < V; ++q) has_end |= (endr[q] >= 0);
      const Acc carry = wave_seg_scan_excl<Acc>(has_end, acc);
      wave_lds_sync();  // every lane has read its products: the buffer now takes row sums
      bool first = true;
#pragma unroll
      for (int q = 0; q < V; ++q) {
        if (endr[q] >= 0) {
          sp[endr[q]] = first ? endv[q] + carry : endv[q];
          first = false;
        }
      }
      wave_lds_sync();
      for (int i = lane; i < nr; i += 64) epi(r0 + i, so[i] == so[i + 1] ? Acc(0) : sp[i]);
      }
    }
  }

  if (MODE == MODE_PLAIN || kBlk) return;
  part = wave_sum(part);
  if (MODE == MODE_REFINE) part2 = wave_sum(part2);
  if (lane == 0) {
    s_wp[0][w] = part;
    s_wp[1][w] = part2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = s_wp[0][0], b2 = s_wp[1][0];
#pragma unroll
    for (int q = 1; q < kWaves; ++q) {
      a += s_wp[0][q];
      b2 += s_wp[1][q];
    }
    const int t = ent.y;
    if (MODE == MODE_TRANS) d->part_phi[t] = a;
    else d->part_rho[t] = a;
    if (MODE == MODE_REFINE) d->part_b[t] = b2;
  }
}

// ------------------------------------------------------------------ outer sequence

// x <- x + nu d ; d <- 0   (float32 storage, after an inner solve)
__global__ __launch_bounds__(kWG) void k_axpy_out(const Desc* __restrict__ D,
                                                  const int2* __restrict__ list) {
  const int2 ent = list[blockIdx.x];
  const Desc* d = D + ent.x;
  const State* st = d->st;
  // only after an inner solve (outer >= 1): nu and d are defined from then on
  if (st->final_done || !st->done || !d->is_f32 || st->outer == 0) return;
  const double nu = st->nu;
  const int base = ent.y * (kWG * 4);
  for (int u = 0; u < 4; ++u) {
    const int j = base + u * kWG + threadIdx.x;
    if (j < d->n) {
      d->xo[j] += nu * d->x[j];
      d->x[j] = 0.0;
    }
  }
}

// nu = ||b - A x||; finish, or start a new inner solve.
__global__ __launch_bounds__(kRW) void k_outer(const Desc* __restrict__ D, const int* __restrict__ sys) {
  __shared__ double s_red[kRW / 64];
  const Desc* d = D + sys[blockIdx.x];
  State* st = d->st;
  if (st->final_done || !st->done) return;
  const double rr = big_sum_array(d->part_rho, d->rho_cnt, s_red);
  const double bb = big_sum_array(d->part_b, d->rho_cnt, s_red);
  if (threadIdx.x != 0) return;
  const double nu = sqrt(rr);
  if (st->outer == 0) st->nb_out = sqrt(bb);
  const double nbo = st->nb_out;
  const double rel = (st->tol_abs || nbo == 0.0) ? nu : nu / nbo;
  st->relres_true = rel;
  const bool converged = rel <= st->tol_out;
  if (st->outer == 0) {
    // before any inner solve: x0 may already satisfy the stop test
    if (converged) {
      st->final_status = ST_OK;
      st->final_done = 1;
      return;
    }
  } else if (!d->is_f32) {
    // float64 storage: one inner solve; its status stands (Algorithm 1 stops
    // on the recursively updated residual), the true residual is reported
    st->final_status = st->status;
    st->final_done = 1;
    return;
  } else if (converged) {
    st->final_status = ST_OK;
    st->final_done = 1;
    return;
  } else if (st->outer >= st->max_outer || st->k_total >= st->maxit ||
             st->status == ST_BREAKDOWN || !(nu < st->nu)) {
    st->final_status = (st->status == ST_BREAKDOWN) ? ST_BREAKDOWN : ST_NOT_CONVERGED;
    st->final_done = 1;
    return;
  }
  // (re)start the inner solve
  st->nu = d->is_f32 ? nu : 1.0;
  st->k = 0;
  st->done = 0;
  st->status = ST_OK;
  st->fresh = 1;
  st->outer += 1;
}

// r <- c (inner right-hand side), partial rho and ||c||^2, on the row
// partition of the partials: the CSR tiles, or the units of a striped store.
template <class Vec>
__global__ __launch_bounds__(kWG) void k_start(const Desc* __restrict__ D, const int2* __restrict__ list) {
  __shared__ double s_wp[kWaves];
  const int2 ent = list[blockIdx.x];
  const Desc* d = D + ent.x;
  const State* st = d->st;
  if (st->final_done || st->done || st->k != 0) return;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const double inv = d->is_f32 ? 1.0 / st->nu : 1.0;
  Vec* r = static_cast<Vec*>(d->r);
  Vec* c = static_cast<Vec*>(d->c);
  double part = 0.0;
  int r0 = 0, r1 = 0, i0 = lane, step = 64;
  if (d->a_striped) {
    r0 = d->sa.urow[ent.y];
    r1 = d->sa.urow[ent.y + 1];
    i0 = threadIdx.x;
    step = kWG;
  } else {
    const int wt = d->a_grp[ent.y * kWaves + w];
    if (wt >= 0) {
      r0 = d->a_tile[wt];
      r1 = d->a_tile[wt + 1];
    }
  }
  for (int i = r0 + i0; i < r1; i += step) {
    const Vec ci = Vec(d->r64[i] * inv);
    r[i] = ci;
    if (c) c[i] = ci;
    part += double(ci) * double(ci);
  }
  part = wave_sum(part);
  if (lane == 0) s_wp[w] = part;
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = s_wp[0];
    for (int q = 1; q < kWaves; ++q) a += s_wp[q];
    d->part_rho[ent.y] = a;
    d->part_b[ent.y] = a;
  }
}

// ------------------------------------------------------------------ inner step scalars

// Algorithm 1: rho, stop test, phi, theta, beta, gamma (one workgroup per system).
__global__ __launch_bounds__(kRW) void k_step(const Desc* __restrict__ D, const int* __restrict__ sys) {
  __shared__ double s_red[4 * (kRW / 64) + 4];
  const Desc* d = D + sys[blockIdx.x];
  State* st = d->st;
  // the state's flags and the four partial sums at once: theta's partials
  // are used only after the first update, those of ||c||^2 only before it
  // (the other one is summed for nothing)
  const int stopped = st->final_done | st->done;
  const long long k = st->k;
  const double4 sums = big_sums4(d->part_rho, d->rho_cnt, d->part_phi, d->phi_cnt, d->part_theta, d->u_nblk,
                                 d->part_b, d->rho_cnt, s_red);
  if (threadIdx.x != 0 || stopped) return;
  const double rho = sums.x, phi = sums.y;
  const double theta = k > 0 ? sums.z : 0.0;
  const double nbi = k == 0 ? sums.w : 0.0;

  if (k == 0) {
    // inner right-hand side norm and thresholds
    const double nb = sqrt(nbi);
    st->nb = nb;
    if (d->is_f32) {
      // inner target relative to ||c||; no tighter than the outer target needs
      double eta = st->inner_tol;
      const double need = 0.5 * st->tol_out * (st->tol_abs ? 1.0 : st->nb_out) / st->nu;
      if (need > eta) eta = need;
      st->thr = eta * nb;
    } else {
      st->thr = st->tol_abs ? st->tol : st->tol * st->nb_out;
    }
    st->scale = (st->tol_abs || st->nb_out == 0.0) ? st->nu : st->nu / st->nb_out;
  }
  const long long kt = st->k_total;
  if (kt < d->hist_len) d->hist[kt] = sqrt(rho) * st->scale;
  st->rho = rho;
  if (sqrt(rho) <= st->thr) {
    st->status = ST_OK;
    st->done = 1;
    return;
  }
  if (kt >= st->maxit) {
    st->status = ST_NOT_CONVERGED;
    st->done = 1;
    return;
  }
  st->phi = phi;
  double beta, gamma;
  if (k == 0) {
    if (!(phi > 0.0)) {
      st->status = ST_BREAKDOWN;
      st->done = 1;
      return;
    }
    beta = 0.0;
    gamma = rho / phi;
  } else {
    st->theta = theta;
    const double s = sqrt(theta * phi) / rho;
    if (!(s > 1.0)) {
      st->status = ST_BREAKDOWN;
      st->done = 1;
      return;
    }
    beta = 1.0 / ((s - 1.0) * (s + 1.0));
    gamma = (theta / rho) * beta;
  }
  st->beta = beta;
  st->gamma = gamma;
  st->fresh = (k == 0);
  st->k = k + 1;
  st->k_total = kt + 1;
}

// p <- beta p + gamma W y ; x <- x + p ; partial theta = p^T (WI p)
template <class Vec>
__global__ __launch_bounds__(kWG) void k_update(const Desc* __restrict__ D, const int2* __restrict__ list) {
  __shared__ double s_red[kWaves];
  const int2 ent = list[blockIdx.x];
  const Desc* d = D + ent.x;
  const State* st = d->st;
  Vec* __restrict__ p = static_cast<Vec*>(d->p);
  const Vec* __restrict__ y = static_cast<const Vec*>(d->y);
  double* __restrict__ x = d->x;
  const double* __restrict__ wi = d->wi;
  const int n = d->n;
  const int base = ent.y * (kWG * 4);
  // the vectors are loaded beside the state (whose flags and scalars they
  // do not depend on), so one round trip to memory precedes the arithmetic
  double yv[4], pv[4], xv[4], wv[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int j = base + u * kWG + threadIdx.x;
    const bool in = j < n;
    yv[u] = in ? double(y[j]) : 0.0;
    pv[u] = in ? double(p[j]) : 0.0;
    xv[u] = in ? x[j] : 0.0;
    wv[u] = (in && wi) ? wi[j] : 1.0;
  }
  if (st->final_done || st->done) return;
  const double beta = st->beta, gamma = st->gamma;
  const bool fresh = st->fresh != 0;
  double part = 0.0;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int j = base + u * kWG + threadIdx.x;
    if (j < n) {
      const double w = wv[u];
      const double wy = wi ? yv[u] / w : yv[u];
      const double pn = fresh ? gamma * wy : beta * pv[u] + gamma * wy;
      const Vec pr = Vec(pn);
      p[j] = pr;
      x[j] = xv[u] + double(pr);
      part += double(pr) * double(pr) * w;
    }
  }
  part = block_sum(part, s_red);
  if (threadIdx.x == 0) d->part_theta[ent.y] = part;
}

// ------------------------------------------------------------------ CSC builder

__global__ void k_csc_count(const int* __restrict__ idx, long long nnz, int* __restrict__ cnt) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nnz;
       e += (long long)gridDim.x * blockDim.x)
    atomicAdd(&cnt[idx[e]], 1);
}

// exclusive scan, stage 1: per-block sums of 1024-element chunks
__global__ __launch_bounds__(kWG) void k_scan_blocks(const int* __restrict__ in, int n,
                                                     long long* __restrict__ bsum) {
  __shared__ long long s_red[kWaves];
  long long v = 0;
  const int base = blockIdx.x * 1024;
  for (int u = 0; u < 4; ++u) {
    const int i = base + u * kWG + threadIdx.x;
    if (i < n) v += in[i];
  }
  v = block_sum(v, s_red);
  if (threadIdx.x == 0) bsum[blockIdx.x] = v;
}

// stage 2: serial exclusive scan of the block sums (single thread; <= a few thousand)
__global__ void k_scan_top(long long* bsum, int nb) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  long long s = 0;
  for (int i = 0; i < nb; ++i) {
    const long long v = bsum[i];
    bsum[i] = s;
    s += v;
  }
  bsum[nb] = s;
}

// stage 3: exclusive scan inside each chunk: out[i] = bsum[blk] + sum in[chunk start..i)
__global__ __launch_bounds__(kWG) void k_scan_apply(const int* __restrict__ in, int n,
                                                    const long long* __restrict__ bsum,
                                                    int* __restrict__ out) {
  __shared__ long long s_t[kWG];
  const int base = blockIdx.x * 1024 + threadIdx.x * 4;
  long long loc[4];
  long long s = 0;
  for (int u = 0; u < 4; ++u) {
    loc[u] = s;
    const int i = base + u;
    s += (i < n) ? in[i] : 0;
  }
  s_t[threadIdx.x] = s;
  __syncthreads();
  // Hillis-Steele inclusive scan over the 256 thread totals
  for (int off = 1; off < kWG; off <<= 1) {
    long long v = (threadIdx.x >= off) ? s_t[threadIdx.x - off] : 0;
    __syncthreads();
    s_t[threadIdx.x] += v;
    __syncthreads();
  }
  const long long pre = bsum[blockIdx.x] + s_t[threadIdx.x] - s;
  for (int u = 0; u < 4; ++u) {
    const int i = base + u;
    if (i < n) out[i] = (int)(pre + loc[u]);
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = (int)bsum[gridDim.x];
}

// scatter (row, position) of every entry into its column's segment; the order
// inside a segment is arbitrary and fixed afterwards by k_csc_sort
__global__ __launch_bounds__(kWG) void k_csc_scatter(const int* __restrict__ ptr,
                                                     const int* __restrict__ idx, int m,
                                                     int* __restrict__ cursor,
                                                     int* __restrict__ row_out,
                                                     int* __restrict__ pos_out) {
  const int lane = threadIdx.x & 63;
  const int wave = (blockIdx.x * kWG + threadIdx.x) >> 6;
  const int nwaves = (gridDim.x * kWG) >> 6;
  for (int i = wave; i < m; i += nwaves) {
    for (int e = ptr[i] + lane; e < ptr[i + 1]; e += 64) {
      const int slot = atomicAdd(&cursor[idx[e]], 1);
      row_out[slot] = i;
      pos_out[slot] = e;
    }
  }
}

// sort each column segment of at most kCscShort entries by row (rows are
// distinct inside a column, so the rank of an entry is the number of smaller
// rows): one wave per column, keys in LDS.  Longer columns are listed for
// k_csc_sort_long.
constexpr int kCscShort = 512;
__global__ __launch_bounds__(kWG) void k_csc_sort(const int* __restrict__ cptr, int n,
                                                  const int* __restrict__ row_in,
                                                  const int* __restrict__ pos_in,
                                                  int* __restrict__ row_out,
                                                  int* __restrict__ pos_out,
                                                  int* __restrict__ long_cols,
                                                  int* __restrict__ n_long) {
  __shared__ int s_key[kWaves][kCscShort];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wave = (blockIdx.x * kWG + threadIdx.x) >> 6;
  const int nwaves = (gridDim.x * kWG) >> 6;
  for (int j = wave; j < n; j += nwaves) {
    const int b = cptr[j], len = cptr[j + 1] - b;
    if (len > kCscShort) {
      if (lane == 0) long_cols[atomicAdd(n_long, 1)] = j;
      continue;
    }
    for (int q = lane; q < len; q += 64) s_key[w][q] = row_in[b + q];
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    for (int q = lane; q < len; q += 64) {
      const int key = s_key[w][q];
      int rank = 0;
      for (int o = 0; o < len; ++o) rank += s_key[w][o] < key;
      row_out[b + rank] = key;
      pos_out[b + rank] = pos_in[b + q];
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  }
}

// Columns longer than kCscShort: one workgroup per column, a least-
// significant-digit radix sort of the (row, position) pairs by row with
// 4-bit digits, linear in the column length per pass.  Each pass counts the
// column's digits, then walks the column in tiles of 4096 in order: a thread
// takes 4 consecutive entries, the (digit, thread) counts are scanned in
// digit-major order, and every entry goes to its digit's next free slot in
// entry order (stable).  Passes alternate between the two buffer pairs; an
// odd pass count ends in (row_b, pos_b).
constexpr int kSortT = 1024;
__global__ __launch_bounds__(kSortT) void k_csc_sort_long(const int* __restrict__ cptr,
                                                          const int* __restrict__ long_cols,
                                                          const int* __restrict__ n_long, int passes,
                                                          int* row_a, int* pos_a, int* row_b, int* pos_b) {
  __shared__ int s_cnt[16 * kSortT];
  __shared__ int s_sum[kSortT];
  __shared__ int s_base[16], s_tot[16], s_dstart[17];
  const int t = threadIdx.x;
  const int nl = *n_long;
  for (int ci = blockIdx.x; ci < nl; ci += gridDim.x) {
    const int j = long_cols[ci];
    const int b = cptr[j], len = cptr[j + 1] - b;
    int* rin = row_a + b;
    int* pin = pos_a + b;
    int* rout = row_b + b;
    int* pout = pos_b + b;
    for (int pass = 0; pass < passes; ++pass) {
      const int sh = 4 * pass;
      if (t < 16) s_tot[t] = 0;
      __syncthreads();
      for (int e = t; e < len; e += kSortT) atomicAdd(&s_tot[sh < 32 ? ((rin[e] >> sh) & 15) : 0], 1);
      __syncthreads();
      if (t == 0) {
        int acc = 0;
        for (int d = 0; d < 16; ++d) {
          s_base[d] = acc;
          acc += s_tot[d];
        }
      }
      __syncthreads();
      for (int t0 = 0; t0 < len; t0 += 4 * kSortT) {
        int key[4], pos[4], dig[4];
        int c[16];
#pragma unroll
        for (int d = 0; d < 16; ++d) c[d] = 0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int e = t0 + 4 * t + u;
          key[u] = e < len ? rin[e] : 0;
          pos[u] = e < len ? pin[e] : 0;
          dig[u] = e < len ? (sh < 32 ? ((key[u] >> sh) & 15) : 0) : -1;
#pragma unroll
          for (int d = 0; d < 16; ++d) c[d] += dig[u] == d;
        }
#pragma unroll
        for (int d = 0; d < 16; ++d) s_cnt[d * kSortT + t] = c[d];
        __syncthreads();
        // exclusive scan of s_cnt in digit-major order: thread t owns
        // entries [16 t, 16 t + 16)
        int loc[16];
        int run = 0;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          loc[q] = run;
          run += s_cnt[16 * t + q];
        }
        s_sum[t] = run;
        __syncthreads();
        for (int off = 1; off < kSortT; off <<= 1) {
          const int v = t >= off ? s_sum[t - off] : 0;
          __syncthreads();
          s_sum[t] += v;
          __syncthreads();
        }
        const int pre = s_sum[t] - run;
#pragma unroll
        for (int q = 0; q < 16; ++q) s_cnt[16 * t + q] = pre + loc[q];
        __syncthreads();
        if (t <= 16) s_dstart[t] = t < 16 ? s_cnt[t * kSortT] : s_sum[kSortT - 1];
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int d = dig[u];
          if (d < 0) continue;
          int before = 0;
#pragma unroll
          for (int v = 0; v < u; ++v) before += dig[v] == d;
          const int slot = s_base[d] + (s_cnt[d * kSortT + t] - s_dstart[d]) + before;
          rout[slot] = key[u];
          pout[slot] = pos[u];
        }
        __syncthreads();
        if (t < 16) s_base[t] += s_dstart[t + 1] - s_dstart[t];
        __syncthreads();
      }
      int* tr = rin; rin = rout; rout = tr;
      int* tp = pin; pin = pout; pout = tp;
      __syncthreads();
    }
  }
}

template <class Val>
__global__ void k_gather_vals(const int* __restrict__ pos, long long nnz, const double* __restrict__ src,
                              Val* __restrict__ dst) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nnz;
       e += (long long)gridDim.x * blockDim.x)
    dst[e] = Val(src[pos[e]]);
}

template <class Val>
__global__ void k_convert_vals(const double* __restrict__ src, long long nnz, Val* __restrict__ dst) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nnz;
       e += (long long)gridDim.x * blockDim.x)
    dst[e] = Val(src[e]);
}

__global__ void k_ptr64_to_32(const long long* __restrict__ src, int n1, int* __restrict__ dst) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n1; i += gridDim.x * blockDim.x)
    dst[i] = (int)src[i];
}

// ------------------------------------------------------------------ host wrappers

static int grid_for(long long work, int per_block = kWG * 4) {
  long long g = (work + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > 65536) g = 65536;
  return (int)g;
}

template <class Val, class Vin, class Acc, int MODE>
static void spmv_v(int V, const Desc* d, const int2* list, int n, int transpose, hipStream_t s) {
  switch (V) {
    case 4: k_spmv<Val, Vin, Acc, MODE, 4><<<n, kWG, 0, s>>>(d, list, transpose); break;
    case 8: k_spmv<Val, Vin, Acc, MODE, 8><<<n, kWG, 0, s>>>(d, list, transpose); break;
    case 16: k_spmv<Val, Vin, Acc, MODE, 16><<<n, kWG, 0, s>>>(d, list, transpose); break;
    default: throw InvalidArg{"unsupported tile width"};
  }
}

void launch_spmv(int mode, bool f32, int V, const Desc* d, const int2* list, int n, int transpose,
                 hipStream_t s) {
  if (n <= 0) return;
  if (!f32) {
    switch (mode) {
      case MODE_RESID: spmv_v<double, double, double, MODE_RESID>(V, d, list, n, 0, s); break;
      case MODE_TRANS: spmv_v<double, double, double, MODE_TRANS>(V, d, list, n, 1, s); break;
      case MODE_REFINE: spmv_v<double, double, double, MODE_REFINE>(V, d, list, n, 0, s); break;
      case MODE_PLAIN: spmv_v<double, double, double, MODE_PLAIN>(V, d, list, n, transpose, s); break;
      case MODE_AP: spmv_v<double, double, double, MODE_AP>(V, d, list, n, 0, s); break;
      case MODE_TRANSB: spmv_v<double, double, double, MODE_TRANSB>(V, d, list, n, 1, s); break;
      case MODE_APB: spmv_v<double, double, double, MODE_APB>(V, d, list, n, 0, s); break;
    }
  } else {
    switch (mode) {
      case MODE_RESID: spmv_v<float, float, float, MODE_RESID>(V, d, list, n, 0, s); break;
      case MODE_TRANS: spmv_v<float, float, float, MODE_TRANS>(V, d, list, n, 1, s); break;
      case MODE_REFINE: spmv_v<float, double, double, MODE_REFINE>(V, d, list, n, 0, s); break;
      case MODE_PLAIN: spmv_v<float, double, double, MODE_PLAIN>(V, d, list, n, transpose, s); break;
      case MODE_TRANSB: spmv_v<float, float, float, MODE_TRANSB>(V, d, list, n, 1, s); break;
      default: throw InvalidArg{"mode not available for float32 storage"};
    }
  }
  PLSS_HIP(hipGetLastError());
}

void launch_axpy_out(const Desc* d, const int2* ulist, int n, hipStream_t s) {
  if (n <= 0) return;
  k_axpy_out<<<n, kWG, 0, s>>>(d, ulist);
}
void launch_outer(const Desc* d, const int* sys, int n, hipStream_t s) {
  if (n <= 0) return;
  k_outer<<<n, kRW, 0, s>>>(d, sys);
}
void launch_start(bool f32, const Desc* d, const int2* alist, int n, hipStream_t s) {
  if (n <= 0) return;
  if (f32) k_start<float><<<n, kWG, 0, s>>>(d, alist);
  else k_start<double><<<n, kWG, 0, s>>>(d, alist);
}
void launch_step(const Desc* d, const int* sys, int n, hipStream_t s) {
  if (n <= 0) return;
  k_step<<<n, kRW, 0, s>>>(d, sys);
}
void launch_update(bool f32, const Desc* d, const int2* ulist, int n, hipStream_t s) {
  if (n <= 0) return;
  if (f32) k_update<float><<<n, kWG, 0, s>>>(d, ulist);
  else k_update<double><<<n, kWG, 0, s>>>(d, ulist);
}

void build_csc(const int* ptr, const int* idx, const double* vals64, int m, int n, long long nnz,
               bool f32, int* cptr, int* ridx, void* cvals, void* work, hipStream_t s) {
  // work layout: cnt[n] | cursor[n+1] | bsum[nb+1] (int64) | row_tmp[nnz] | pos_tmp[nnz] | pos[nnz] |
  // long_cols[n] | n_long
  char* w = static_cast<char*>(work);
  int* cnt = reinterpret_cast<int*>(w);
  w += sizeof(int) * ((size_t)n + 64);
  int* cursor = reinterpret_cast<int*>(w);
  w += sizeof(int) * ((size_t)n + 64);
  const int nb = (n + 1023) / 1024;
  long long* bsum = reinterpret_cast<long long*>(w);
  w += sizeof(long long) * ((size_t)nb + 64);
  int* row_tmp = reinterpret_cast<int*>(w);
  w += sizeof(int) * ((size_t)nnz + 64);
  int* pos_tmp = reinterpret_cast<int*>(w);
  w += sizeof(int) * ((size_t)nnz + 64);
  int* pos = reinterpret_cast<int*>(w);
  w += sizeof(int) * ((size_t)nnz + 64);
  int* long_cols = reinterpret_cast<int*>(w);
  w += sizeof(int) * ((size_t)n + 64);
  int* n_long = reinterpret_cast<int*>(w);

  PLSS_HIP(hipMemsetAsync(cnt, 0, sizeof(int) * (size_t)n, s));
  if (nnz > 0) k_csc_count<<<grid_for(nnz), kWG, 0, s>>>(idx, nnz, cnt);
  k_scan_blocks<<<nb, kWG, 0, s>>>(cnt, n, bsum);
  k_scan_top<<<1, 64, 0, s>>>(bsum, nb);
  k_scan_apply<<<nb, kWG, 0, s>>>(cnt, n, bsum, cptr);
  PLSS_HIP(hipMemcpyAsync(cursor, cptr, sizeof(int) * (size_t)n, hipMemcpyDeviceToDevice, s));
  if (nnz > 0) {
    k_csc_scatter<<<grid_for((long long)m * 64, kWG), kWG, 0, s>>>(ptr, idx, m, cursor, row_tmp, pos_tmp);
    PLSS_HIP(hipMemsetAsync(n_long, 0, sizeof(int), s));
    k_csc_sort<<<grid_for((long long)n * 64, kWG), kWG, 0, s>>>(cptr, n, row_tmp, pos_tmp, ridx, pos, long_cols,
                                                                n_long);
    // digit passes over the row indices (an odd count ends in ridx / pos)
    int bits = 1;
    while (bits < 31 && (1LL << bits) < (long long)m) ++bits;
    int passes = (bits + 3) / 4;
    if (passes % 2 == 0) ++passes;
    k_csc_sort_long<<<256, kSortT, 0, s>>>(cptr, long_cols, n_long, passes, row_tmp, pos_tmp, ridx, pos);
    if (f32) k_gather_vals<float><<<grid_for(nnz), kWG, 0, s>>>(pos, nnz, vals64, static_cast<float*>(cvals));
    else k_gather_vals<double><<<grid_for(nnz), kWG, 0, s>>>(pos, nnz, vals64, static_cast<double*>(cvals));
  }
  PLSS_HIP(hipGetLastError());
}

size_t csc_work_bytes(int n, long long nnz) {
  const int nb = (n + 1023) / 1024;
  return sizeof(int) * ((size_t)n + 64) * 3 + sizeof(long long) * ((size_t)nb + 64) +
         sizeof(int) * ((size_t)nnz + 64) * 3 + 256;
}

void convert_vals(const double* src, long long nnz, bool f32, void* dst, hipStream_t s) {
  if (nnz <= 0) return;
  if (f32) k_convert_vals<float><<<grid_for(nnz), kWG, 0, s>>>(src, nnz, static_cast<float*>(dst));
  else k_convert_vals<double><<<grid_for(nnz), kWG, 0, s>>>(src, nnz, static_cast<double*>(dst));
  PLSS_HIP(hipGetLastError());
}

void ptr64_to_32(const long long* src, int n1, int* dst, hipStream_t s) {
  k_ptr64_to_32<<<grid_for(n1, kWG), kWG, 0, s>>>(src, n1, dst);
  PLSS_HIP(hipGetLastError());
}

}  // namespace plss

namespace plss {

// CSR checks on the device: column indices in range, strictly ascending in a
// row, values finite.  flags bit 0: index out of range, bit 1: not ascending
// or duplicate, bit 2: non-finite value.
__global__ __launch_bounds__(kWG) void k_validate(const long long* __restrict__ ptr,
                                                  const int* __restrict__ idx,
                                                  const double* __restrict__ val, int m, int n,
                                                  int* __restrict__ flags) {
  const int lane = threadIdx.x & 63;
  const int wave = (blockIdx.x * kWG + threadIdx.x) >> 6;
  const int nwaves = (gridDim.x * kWG) >> 6;
  int f = 0;
  for (int i = wave; i < m; i += nwaves) {
    const long long b = ptr[i], e = ptr[i + 1];
    for (long long q = b + lane; q < e; q += 64) {
      const int c = idx[q];
      if (c < 0 || c >= n) f |= 1;
      if (q + 1 < e && idx[q + 1] <= c) f |= 2;
      if (!isfinite(val[q])) f |= 4;
    }
  }
  if (f) atomicOr(flags, f);
}

int validate_csr_device(const long long* ptr, const int* idx, const double* val, int m, int n,
                        int* dflag, hipStream_t s) {
  PLSS_HIP(hipMemsetAsync(dflag, 0, sizeof(int), s));
  k_validate<<<grid_for((long long)m * 64, kWG), kWG, 0, s>>>(ptr, idx, val, m, n, dflag);
  PLSS_HIP(hipGetLastError());
  int hf = 0;
  PLSS_HIP(hipMemcpyAsync(&hf, dflag, sizeof(int), hipMemcpyDeviceToHost, s));
  PLSS_HIP(hipStreamSynchronize(s));
  return hf;
}

}  // namespace plss

namespace plss {

// flag = 1 if any entry is not finite (or, with positive != 0, not > 0)
__global__ void k_check(const double* __restrict__ a, long long n, int positive, int* __restrict__ flag) {
  int f = 0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const double v = a[i];
    if (!isfinite(v) || (positive && !(v > 0.0))) f = 1;
  }
  if (f) atomicOr(flag, 1);
}

void launch_check(const double* a, long long n, int positive, int* flag, hipStream_t s) {
  if (n <= 0) return;
  k_check<<<grid_for(n), kWG, 0, s>>>(a, n, positive, flag);
  PLSS_HIP(hipGetLastError());
}

}  // namespace plss

namespace plss {

// ------------------------------------------------------------------ row-blocked transpose

// For every column j of the CSC and every row block b (rows [rb[b], rb[b+1])),
// the number of the column's entries in that block: rows are ascending inside
// a column, so block b's entries are one contiguous sub-segment.
__global__ void k_blk_count(const int* __restrict__ cp, const int* __restrict__ ri, int n,
                            const int* __restrict__ rb, int nblk, int* __restrict__ cnt) {
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
    const int b0 = cp[j], b1 = cp[j + 1];
    int prev = b0;
    for (int b = 0; b < nblk; ++b) {
      // first entry of the column with row >= rb[b + 1]
      const int lim = rb[b + 1];
      int lo = prev, hi = b1;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (ri[mid] < lim) lo = mid + 1;
        else hi = mid;
      }
      cnt[(size_t)b * n + j] = lo - prev;
      prev = lo;
    }
  }
}

// Copy block b's sub-segment of every column into that block's arrays:
// the sub-segment starts after the column's entries of blocks 0..b-1.
template <class Val>
__global__ void k_blk_copy(const int* __restrict__ cp, const int* __restrict__ ri, const Val* __restrict__ cv,
                           int n, int b, const int* __restrict__ bptr, int* __restrict__ oi,
                           Val* __restrict__ ov) {
  const int lane = threadIdx.x & 63;
  const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int nw = (gridDim.x * blockDim.x) >> 6;
  for (int j = wave; j < n; j += nw) {
    int src = cp[j];
    for (int q = 0; q < b; ++q) {
      const int* p = bptr + (size_t)q * (n + 1);
      src += p[j + 1] - p[j];
    }
    const int* p = bptr + (size_t)b * (n + 1);
    const int dst = p[j], len = p[j + 1] - p[j];
    for (int q = lane; q < len; q += 64) {
      oi[dst + q] = ri[src + q];
      ov[dst + q] = cv[src + q];
    }
  }
}

// y_j = sum over blocks of the block products (fixed block order); partial phi.
template <class Vec>
__global__ __launch_bounds__(kWG) void k_ycomb(const Desc* __restrict__ D, const int2* __restrict__ list) {
  __shared__ double s_red[kWaves];
  const int2 ent = list[blockIdx.x];
  const Desc* d = D + ent.x;
  const State* st = d->st;
  const int n = d->n, nb = d->nblk;
  if (nb <= 1) return;
  Vec* __restrict__ y = static_cast<Vec*>(d->y);
  const Vec* __restrict__ yp = static_cast<const Vec*>(d->ypart);
  const double* __restrict__ wi = d->wi;
  double part = 0.0;
  const int base = ent.y * (kWG * 4);
  // every block's partials loaded first (beside the state's flags, which
  // they do not depend on), then added in block order
  Vec v[4][kMaxBlk];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int j = base + u * kWG + threadIdx.x;
#pragma unroll
    for (int b = 0; b < kMaxBlk; ++b) v[u][b] = (b < nb && j < n) ? yp[(size_t)b * n + j] : Vec(0);
  }
  if (st->final_done || st->done) return;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int j = base + u * kWG + threadIdx.x;
    if (j < n) {
      Vec s = v[u][0];
#pragma unroll
      for (int b = 1; b < kMaxBlk; ++b) s = b < nb ? s + v[u][b] : s;
      y[j] = s;
      const double ds = double(s);
      part += wi ? ds * ds / wi[j] : ds * ds;
    }
  }
  part = block_sum(part, s_red);
  if (threadIdx.x == 0) d->part_phi[ent.y] = part;
}

// A p from its column-block products (identity and mixed sketches): for the
// rows of one CSR tile group, ap_i = sum over blocks of appart[b][i] in block
// order, then the step of MODE_AP: AP column kh <- ap, r <- r - ap, partial
// rho per group (the same partition as the unblocked product's partials).
__global__ __launch_bounds__(kWG) void k_apcomb(const Desc* __restrict__ D, const int2* __restrict__ list) {
  __shared__ double s_red[kWaves];
  const int2 ent = list[blockIdx.x];
  const Desc* d = D + ent.x;
  const State* st = d->st;
  if (st->final_done || st->done || st->skip) return;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int m = d->m, nb = d->cnblk;
  const double* __restrict__ ap = d->appart;
  double* __restrict__ r = static_cast<double*>(d->r);
  double* __restrict__ APk = d->AP + (size_t)st->kh * m;
  double part = 0.0;
  const int wt = d->a_grp[ent.y * kWaves + w];
  if (wt >= 0) {
    const int r0 = d->a_tile[wt], r1 = d->a_tile[wt + 1];
    for (int i = r0 + lane; i < r1; i += 64) {
      double v[kMaxBlk];
#pragma unroll
      for (int b = 0; b < kMaxBlk; ++b) v[b] = b < nb ? ap[(size_t)b * m + i] : 0.0;
      double sum = v[0];
#pragma unroll
      for (int b = 1; b < kMaxBlk; ++b) sum = b < nb ? sum + v[b] : sum;
      const double rn = r[i] - sum;
      r[i] = rn;
      APk[i] = sum;
      part += rn * rn;
    }
  }
  part = block_sum(part, s_red);
  if (threadIdx.x == 0) d->part_rho[ent.y] = part;
}

void launch_apcomb(const Desc* d, const int2* alist, int n, hipStream_t s) {
  if (n <= 0) return;
  k_apcomb<<<n, kWG, 0, s>>>(d, alist);
  PLSS_HIP(hipGetLastError());
}

// counts and per-block pointer arrays (bptr: nblk x (n+1), relative to each block)
void blk_build(const int* cp, const int* ri, int n, const int* d_rb, int nblk, int* d_cnt, int* d_bptr,
               void* scan_work, hipStream_t s) {
  k_blk_count<<<grid_for(n, kWG), kWG, 0, s>>>(cp, ri, n, d_rb, nblk, d_cnt);
  const int nbk = (n + 1023) / 1024;
  long long* bsum = static_cast<long long*>(scan_work);
  for (int b = 0; b < nblk; ++b) {
    k_scan_blocks<<<nbk, kWG, 0, s>>>(d_cnt + (size_t)b * n, n, bsum);
    k_scan_top<<<1, 64, 0, s>>>(bsum, nbk);
    k_scan_apply<<<nbk, kWG, 0, s>>>(d_cnt + (size_t)b * n, n, bsum, d_bptr + (size_t)b * (n + 1));
  }
  PLSS_HIP(hipGetLastError());
}

void blk_copy(const int* cp, const int* ri, const void* cv, bool f32, int n, int b, const int* d_bptr, int* oi,
              void* ov, hipStream_t s) {
  if (f32)
    k_blk_copy<float><<<grid_for((long long)n * 64, kWG), kWG, 0, s>>>(
        cp, ri, static_cast<const float*>(cv), n, b, d_bptr, oi, static_cast<float*>(ov));
  else
    k_blk_copy<double><<<grid_for((long long)n * 64, kWG), kWG, 0, s>>>(
        cp, ri, static_cast<const double*>(cv), n, b, d_bptr, oi, static_cast<double*>(ov));
  PLSS_HIP(hipGetLastError());
}

void launch_ycomb(bool f32, const Desc* d, const int2* ulist, int n, hipStream_t s) {
  if (n <= 0) return;
  if (f32) k_ycomb<float><<<n, kWG, 0, s>>>(d, ulist);
  else k_ycomb<double><<<n, kWG, 0, s>>>(d, ulist);
}

void scan_counts(const int* cnt, int n, int* out, void* work, hipStream_t s) {
  long long* bsum = static_cast<long long*>(work);
  if (n <= 0) {
    k_scan_top<<<1, 64, 0, s>>>(bsum, 0);
    k_ptr64_to_32<<<1, 64, 0, s>>>(bsum, 1, out);
    PLSS_HIP(hipGetLastError());
    return;
  }
  const int nbk = (n + 1023) / 1024;
  k_scan_blocks<<<nbk, kWG, 0, s>>>(cnt, n, bsum);
  k_scan_top<<<1, 64, 0, s>>>(bsum, nbk);
  k_scan_apply<<<nbk, kWG, 0, s>>>(cnt, n, bsum, out);
  PLSS_HIP(hipGetLastError());
}

}  // namespace plss
