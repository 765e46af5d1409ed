// Single-workgroup solve of a small system (Algorithm 1 with the outer
// refinement loop), one 1024-thread workgroup per system.
//
// For a system whose vectors fit in LDS the multi-kernel iteration spends
// its time in launches and host polls, not in the products (a 2000 x 1000
// system with 16,000 entries is a few microseconds of work per iteration).
// Here one workgroup runs the whole solve: x, r, p, y and both row-pointer
// arrays live in LDS, the matrix entries (CSR and CSC) are read from L2,
// every reduction is a fixed-order
// workgroup sum, and the phases are separated by workgroup barriers.  Rows
// of at most 64 entries are read from the matrix's slice layout (a wave's 64
// rows side by side, four entries per lane and load); the sum of each row
// keeps its entry order.  The
// decisions are those of the multi-kernel path (k_outer, k_start, k_step,
// k_update): the same stop test, breakdown and iteration-limit rules, the
// same refinement restarts and the same per-row arithmetic, so a system
// stops at the same iteration with the same status; only the order of the
// sums inside each product and reduction differs.  A launch covers any
// number of systems (one workgroup each), so a batch of small systems is one
// persistent launch whose systems finish independently.
#include "kernels.hpp"
#include "wave.hpp"

namespace plss {

namespace {

constexpr int kSmT = 1024;         // threads per system
constexpr int kSmWaves = kSmT / 64;
static_assert(kSmWaves == 16, "the workgroup sums add one wave sum per lane of a 16-lane row");
constexpr int kLongRow = 64;       // rows longer than this are summed by a whole wave

// v of lane l (l wave-uniform); the result is uniform
__device__ __forceinline__ double lane_value(double v, int l) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xFFFFFFFFLL), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}

// Inclusive sum over each row of 16 lanes (lane 15 of a row holds the row's
// total), by DPP row shifts in a fixed order.
__device__ __forceinline__ double row16_sum(double v) {
  v += dppv<kRowShr1, 0xF, true>(v);
  v += dppv<kRowShr2, 0xF, true>(v);
  v += dppv<kRowShr4, 0xF, true>(v);
  v += dppv<kRowShr8, 0xF, true>(v);
  return v;
}

// Fixed-order workgroup sums of one value (TWO = false) or two; the results
// are valid in every thread.  s_red holds two buffers of 2 x kSmWaves
// doubles used in turn (par flips every call), so one barrier per call
// suffices: a wave cannot write a buffer again before every wave has passed
// the next call's barrier, which it reaches only after reading this call's
// sums.  The barrier also publishes every LDS write made before the call.
template <bool TWO>
__device__ __forceinline__ void sm_sum2(double& a, double& b, double* s_red, int& par) {
  a = wave_sum_dpp(a);
  if (TWO) b = wave_sum_dpp(b);
  const int w = threadIdx.x >> 6;
  double* buf = s_red + par * (2 * kSmWaves);
  par ^= 1;
  if ((threadIdx.x & 63) == 0) {
    buf[w] = a;
    if (TWO) buf[kSmWaves + w] = b;
  }
  __syncthreads();
  // lanes 0..15 of every wave read the 16 wave sums, one each, and add them
  // within the first row of 16 lanes in a fixed order (shifts by 1, 2, 4, 8;
  // lane 15 ends with the total)
  const int l = threadIdx.x & 63;
  double ta = l < kSmWaves ? buf[l] : 0.0;
  double tb = TWO && l < kSmWaves ? buf[kSmWaves + l] : 0.0;
  ta = row16_sum(ta);
  a = lane_value(ta, kSmWaves - 1);
  if (TWO) {
    tb = row16_sum(tb);
    b = lane_value(tb, kSmWaves - 1);
  }
}

// Row products of a CSR direction (row pointers in LDS): rows of at most
// kLongRow entries one lane each (entries summed in order; four loads issued
// ahead), longer rows one wave each (lanes strided, then a wave sum);
// epi(i, s) runs once per row.
template <class Val, class Acc, class Vin, class Epi>
__device__ __forceinline__ void sm_rows(const int* __restrict__ ptr, const int* __restrict__ idx,
                                        const Val* __restrict__ val, int nrows, const int* __restrict__ lrows,
                                        int nlong, const Vin* __restrict__ v, const int* __restrict__ sl_base,
                                        const int* __restrict__ sl_idx, const Val* __restrict__ sl_val, Epi epi) {
  for (int i = threadIdx.x; i < nrows; i += kSmT) {
    const int len = ptr[i + 1] - ptr[i];
    if (len > kLongRow) continue;
    Acc s = Acc(0);
    const int sb = sl_base[i >> 6] + 4 * (i & 63);
    int k = 0;
    for (; k + 4 <= len; k += 4) {
      const int o = sb + (k >> 2) * 256;
      const int c0 = gload(&sl_idx[o]), c1 = gload(&sl_idx[o + 1]), c2 = gload(&sl_idx[o + 2]),
                c3 = gload(&sl_idx[o + 3]);
      const Val v0 = gload(&sl_val[o]), v1 = gload(&sl_val[o + 1]), v2 = gload(&sl_val[o + 2]),
                v3 = gload(&sl_val[o + 3]);
      s += Acc(v0) * Acc(v[c0]);
      s += Acc(v1) * Acc(v[c1]);
      s += Acc(v2) * Acc(v[c2]);
      s += Acc(v3) * Acc(v[c3]);
    }
    for (; k < len; ++k) {
      const int o = sb + (k >> 2) * 256 + (k & 3);
      s += Acc(gload(&sl_val[o])) * Acc(v[gload(&sl_idx[o])]);
    }
    epi(i, s);
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int q = w; q < nlong; q += kSmWaves) {
    const int i = gload(&lrows[q]);
    const int e0 = ptr[i], e1 = ptr[i + 1];
    Acc s = Acc(0);
    for (int e = e0 + lane; e < e1; e += 64) s += Acc(gload(&val[e])) * Acc(v[gload(&idx[e])]);
    s = wave_sum_dpp(s);
    if (lane == 0) epi(i, s);
  }
}

}  // namespace

// Val: stored value type; Vec: type of r, p, y (and of the products'
// accumulation), as in the multi-kernel path.
template <class Val, class Vec>
__global__ __launch_bounds__(kSmT) void k_small(const Desc* __restrict__ D, const int* __restrict__ sys) {
  __shared__ double s_mem[kSmallLds / sizeof(double)];
  __shared__ double s_red[4 * kSmWaves];
  int par = 0;  // buffer of the next workgroup sum
  const Desc* d = D + sys[blockIdx.x];
  State* st = d->st;
  const int m = d->m, n = d->n;
  const bool f32 = d->is_f32 != 0;
  // LDS: x (float64), r, p, y (Vec), then the row pointers and the slice
  // starts of both directions (the layout small_fits() checks)
  const int ma = (m + 31) & ~31, na = (n + 31) & ~31;
  double* xl = s_mem;
  Vec* r = reinterpret_cast<Vec*>(xl + na);
  Vec* p = r + ma;
  Vec* y = p + na;
  int* a_ptr_l = reinterpret_cast<int*>(y + na);
  int* t_ptr_l = a_ptr_l + ((m + 1 + 31) & ~31);
  const int nsa = (m + 63) / 64, nst = (n + 63) / 64;
  int* a_slb_l = t_ptr_l + ((n + 1 + 31) & ~31);
  int* t_slb_l = a_slb_l + ((nsa + 31) & ~31);
  // the descriptor's fields as restricted locals (stores to the vectors below
  // cannot then force the compiler to reread the descriptor)
  const int* __restrict__ a_ptr = d->a_ptr;
  const int* __restrict__ a_idx = d->a_idx;
  const int* __restrict__ t_ptr = d->t_ptr;
  const int* __restrict__ t_idx = d->t_idx;
  const int* __restrict__ a_long = d->a_long;
  const int* __restrict__ t_long = d->t_long;
  const int a_nlong = d->a_nlong, t_nlong = d->t_nlong;
  const Val* __restrict__ aval = static_cast<const Val*>(d->a_val);
  const Val* __restrict__ tval = static_cast<const Val*>(d->t_val);
  const int* __restrict__ a_slb = d->a_sl_base;
  const int* __restrict__ a_sli = d->a_sl_idx;
  const Val* __restrict__ a_slv = static_cast<const Val*>(d->a_sl_val);
  const int* __restrict__ t_slb = d->t_sl_base;
  const int* __restrict__ t_sli = d->t_sl_idx;
  const Val* __restrict__ t_slv = static_cast<const Val*>(d->t_sl_val);
  const double* __restrict__ bvec = d->b;
  double* __restrict__ r64 = d->r64;
  const double* __restrict__ wi = d->wi;
  double* __restrict__ xo = d->xo;
  double* __restrict__ xi = d->x;  // inner solution (== xo for float64 storage)
  Vec* __restrict__ cvec = static_cast<Vec*>(d->c);
  double* __restrict__ hist = d->hist;
  const long long hist_len = d->hist_len;
  for (int i = threadIdx.x; i <= m; i += kSmT) a_ptr_l[i] = gload(&a_ptr[i]);
  for (int i = threadIdx.x; i <= n; i += kSmT) t_ptr_l[i] = gload(&t_ptr[i]);
  for (int i = threadIdx.x; i < nsa; i += kSmT) a_slb_l[i] = gload(&a_slb[i]);
  for (int i = threadIdx.x; i < nst; i += kSmT) t_slb_l[i] = gload(&t_slb[i]);
  __syncthreads();

  const double tol = st->tol, tol_out = st->tol_out, inner_tol = st->inner_tol;
  const int tol_abs = st->tol_abs;
  const long long maxit = st->maxit, max_outer = st->max_outer;
  double nu = st->nu, nb_out = 0.0, relres_true = 0.0;
  double rho = 0.0, theta = 0.0, thr = 0.0, scale = 0.0;
  long long k_total = 0, outer = 0;
  int status = ST_OK, final_status = ST_OK;

  for (;;) {
    // ---- outer step (k_axpy_out, k_spmv<REFINE>, k_outer)
    if (f32 && outer > 0) {
      for (int j = threadIdx.x; j < n; j += kSmT) {
        gstore(&xo[j], gload(&xo[j]) + nu * gload(&xi[j]));
        gstore(&xi[j], 0.0);
      }
      __syncthreads();
    }
    double rr = 0.0, bb = 0.0;
    sm_rows<Val, double, double>(a_ptr_l, a_idx, aval, m, a_long, a_nlong, xo, a_slb_l, a_sli, a_slv, [&](int i, double s) {
      const double bi = gload(&bvec[i]);
      const double ri = bi - s;
      gstore(&r64[i], ri);
      rr += ri * ri;
      bb += bi * bi;
    });
    sm_sum2<true>(rr, bb, s_red, par);
    const double nu_new = sqrt(rr);
    if (outer == 0) nb_out = sqrt(bb);
    const double rel = (tol_abs || nb_out == 0.0) ? nu_new : nu_new / nb_out;
    relres_true = rel;
    const bool converged = rel <= tol_out;
    if (outer == 0) {
      if (converged) {
        final_status = ST_OK;
        break;
      }
    } else if (!f32) {
      final_status = status;
      break;
    } else if (converged) {
      final_status = ST_OK;
      break;
    } else if (outer >= max_outer || k_total >= maxit || status == ST_BREAKDOWN || !(nu_new < nu)) {
      final_status = status == ST_BREAKDOWN ? ST_BREAKDOWN : ST_NOT_CONVERGED;
      break;
    }
    nu = f32 ? nu_new : 1.0;
    status = ST_OK;
    outer += 1;

    // ---- inner start (k_start): r = c = r64 / nu
    const double inv = f32 ? 1.0 / nu : 1.0;
    double cc = 0.0, unused = 0.0;
    for (int i = threadIdx.x; i < m; i += kSmT) {
      const Vec ci = Vec(gload(&r64[i]) * inv);
      r[i] = ci;
      if (cvec) gstore(&cvec[i], ci);
      cc += double(ci) * double(ci);
    }
    sm_sum2<false>(cc, unused, s_red, par);  // its barrier also publishes r
    rho = cc;
    const double nb = sqrt(cc);
    if (f32) {
      double eta = inner_tol;
      const double need = 0.5 * tol_out * (tol_abs ? 1.0 : nb_out) / nu;
      if (need > eta) eta = need;
      thr = eta * nb;
    } else {
      thr = tol_abs ? tol : tol * nb_out;
    }
    scale = (tol_abs || nb_out == 0.0) ? nu : nu / nb_out;
    for (int j = threadIdx.x; j < n; j += kSmT) xl[j] = gload(&xi[j]);  // published by the next barrier

    // ---- inner iterations (k_spmv<RESID>, k_step, k_spmv<TRANS>, k_update)
    for (long long k = 0;; ++k) {
      if (k > 0) {
        double rp = 0.0, unused2 = 0.0;
        sm_rows<Val, Vec, Vec>(a_ptr_l, a_idx, aval, m, a_long, a_nlong, p, a_slb_l, a_sli, a_slv, [&](int i, Vec s) {
          const Vec rn = Vec(r[i] - s);
          r[i] = rn;
          rp += double(rn) * double(rn);
        });
        sm_sum2<false>(rp, unused2, s_red, par);
        rho = rp;
      }
      if (threadIdx.x == 0 && k_total < hist_len) gstore(&hist[k_total], sqrt(rho) * scale);
      if (sqrt(rho) <= thr) {
        status = ST_OK;
        break;
      }
      if (k_total >= maxit) {
        status = ST_NOT_CONVERGED;
        break;
      }
      double ph = 0.0, unused3 = 0.0;
      sm_rows<Val, Vec, Vec>(t_ptr_l, t_idx, tval, n, t_long, t_nlong, r, t_slb_l, t_sli, t_slv, [&](int i, Vec s) {
        y[i] = s;
        const double ds = double(s);
        ph += wi ? ds * ds / gload(&wi[i]) : ds * ds;
      });
      sm_sum2<false>(ph, unused3, s_red, par);
      double beta, gamma;
      if (k == 0) {
        if (!(ph > 0.0)) {
          status = ST_BREAKDOWN;
          break;
        }
        beta = 0.0;
        gamma = rho / ph;
      } else {
        const double s = sqrt(theta * ph) / rho;
        if (!(s > 1.0)) {
          status = ST_BREAKDOWN;
          break;
        }
        beta = 1.0 / ((s - 1.0) * (s + 1.0));
        gamma = (theta / rho) * beta;
      }
      const bool fresh = k == 0;
      k_total += 1;
      double th = 0.0, unused4 = 0.0;
      for (int j = threadIdx.x; j < n; j += kSmT) {
        const double w = wi ? gload(&wi[j]) : 1.0;
        const double wy = wi ? double(y[j]) / w : double(y[j]);
        const double pn = fresh ? gamma * wy : beta * double(p[j]) + gamma * wy;
        const Vec pv = Vec(pn);
        p[j] = pv;
        xl[j] += double(pv);
        th += double(pv) * double(pv) * w;
      }
      sm_sum2<false>(th, unused4, s_red, par);
      theta = th;
    }
    // the inner solution back to memory for the outer step
    for (int j = threadIdx.x; j < n; j += kSmT) gstore(&xi[j], xl[j]);
    __syncthreads();
  }

  if (threadIdx.x == 0) {
    st->rho = rho;
    st->theta = theta;
    st->thr = thr;
    st->scale = scale;
    st->nu = nu;
    st->nb_out = nb_out;
    st->relres_true = relres_true;
    st->k_total = k_total;
    st->outer = outer;
    st->status = status;
    st->final_status = final_status;
    st->done = 1;
    st->final_done = 1;
  }
}

bool small_fits(int m, int n, bool f32) {
  const size_t vb = f32 ? 4 : 8;
  const size_t ma = (size_t)((m + 31) & ~31), na = (size_t)((n + 31) & ~31);
  const size_t slices = (size_t)((((m + 63) / 64) + 31) & ~31) + (size_t)((n + 63) / 64);
  const size_t bytes = 8 * na + vb * (ma + 2 * na) +
                       4 * ((size_t)((m + 1 + 31) & ~31) + (size_t)((n + 1 + 31) & ~31) + slices);
  return bytes <= kSmallLds;
}

void launch_small(bool f32, const Desc* d, const int* sys, int n, hipStream_t s) {
  if (n <= 0) return;
  if (f32) k_small<float, float><<<n, kSmT, 0, s>>>(d, sys);
  else k_small<double, double><<<n, kSmT, 0, s>>>(d, sys);
  PLSS_HIP(hipGetLastError());
}

}  // namespace plss
