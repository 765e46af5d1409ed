// Striped sparse products: the gathered vector passes through LDS.
//
// A CSR product whose gathered vector x does not stay in a CU's caches is
// bound by the rate of scattered L2 requests, not by HBM.  The striped store
// turns the gather into a stream: a workgroup owns a block of rows (a
// "unit"), keeps the unit's row sums in LDS, and walks the columns in
// stripes of SW entries, staging each stripe's slice of x in LDS.  The
// entries of a unit are grouped stripe by stripe and, inside a stripe, kept
// in CSR order (row, then column); each entry packs its row inside the unit
// and its column inside the stripe into one 32-bit word, stored with the
// value as one record (12 bytes for float64, 8 for float32) that a lane
// loads with one instruction.
//
// Inside a (unit, stripe) segment the 16 waves of the workgroup take 16
// consecutive ranges of entries whose boundaries fall on row starts (fixed
// when the store is built), so every row's stripe sum has exactly one
// writer.  A wave walks its range in windows of at most 64*Q entries (Q <= 7
// per lane, chosen from the range length): each lane takes a run of
// consecutive entries, sums its runs of equal rows, and a wave-level
// segmented scan (DPP row shifts and broadcasts) carries the open run from
// lane to lane and from window to window.  Each window is stored
// lane-interleaved (the lane's k-th record at window start + 64 k + lane), so
// every load instruction of the wave reads 64 consecutive records.  Stripes
// are applied in order, so each row sum has one fixed order: the product is
// deterministic and does not depend on which other systems share a launch.
// Wave bounds are read two stripes ahead and first windows one stripe
// ahead, so their memory latency overlaps the arithmetic of the stripe in
// between.
#include "kernels.hpp"
#include "wave.hpp"
#include "window.hpp"

namespace plss {

namespace {

constexpr int kST = kSThreads;       // threads of the striped workgroups
constexpr int kSWaves = kST / 64;    // waves per striped workgroup

template <class T>
__device__ __forceinline__ T swsum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// first index i in [lo, hi) with a[i] > key (a non-decreasing)
__device__ __forceinline__ int upper_bound_i(const int* __restrict__ a, int lo, int hi, int key) {
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (a[mid] <= key) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

}  // namespace

// ------------------------------------------------------------------ build

// cnt[u * S + s] = entries of unit u whose column lies in stripe s.  The
// source is a CSR direction whose column indices are offset by colbase.
__global__ __launch_bounds__(kST) void k_st_count(const int* __restrict__ ptr, const int* __restrict__ idx,
                                                  const int* __restrict__ urow, int S, int colbase, int sw,
                                                  int* __restrict__ cnt) {
  extern __shared__ int s_h[];
  const int u = blockIdx.x;
  for (int s = threadIdx.x; s < S; s += kST) s_h[s] = 0;
  __syncthreads();
  const int e0 = ptr[urow[u]], e1 = ptr[urow[u + 1]];
  for (int e = e0 + threadIdx.x; e < e1; e += kST) atomicAdd(&s_h[(idx[e] - colbase) / sw], 1);
  __syncthreads();
  for (int s = threadIdx.x; s < S; s += kST) cnt[(size_t)u * S + s] = s_h[s];
}

// Stable scatter of one unit's entries into stripe order.  The unit's
// entries are taken kST at a time in CSR order; a batch is sorted in LDS by
// the key (stripe, position in the batch) (bitonic network), which gives
// each entry its rank among the batch's entries of the same stripe, and a
// per-stripe cursor (starting at the segment start seg[u * S + s]) places
// the batches one after the other.  CSR order is kept inside every stripe.
template <class Val>
__global__ __launch_bounds__(kST) void k_st_scatter(const int* __restrict__ ptr, const int* __restrict__ idx,
                                                    const Val* __restrict__ val, const int* __restrict__ urow,
                                                    const int* __restrict__ seg, int S, int colbase, int sw,
                                                    unsigned* __restrict__ opk, Val* __restrict__ oval) {
  extern __shared__ int s_cur[];  // S cursors
  __shared__ unsigned s_key[kST];
  __shared__ unsigned s_pk[kST];
  __shared__ Val s_val[kST];
  const int u = blockIdx.x;
  const int r0 = urow[u], r1 = urow[u + 1];
  for (int s = threadIdx.x; s < S; s += kST) s_cur[s] = seg[(size_t)u * S + s];
  const int e0 = ptr[r0], e1 = ptr[r1];
  const int t = threadIdx.x;
  for (int base = e0; base < e1; base += kST) {
    const int e = base + t;
    unsigned key = 0xFFFFFFFFu;
    if (e < e1) {
      const int col = idx[e] - colbase;
      const int st = col / sw;
      const int row = upper_bound_i(ptr, r0, r1 + 1, e) - 1;  // ptr[row] <= e < ptr[row + 1]
      s_pk[t] = ((unsigned)(row - r0) << 16) | (unsigned)(col - st * sw);
      s_val[t] = val[e];
      key = ((unsigned)st << 10) | (unsigned)t;
    }
    s_key[t] = key;
    __syncthreads();
    for (int k = 2; k <= kST; k <<= 1) {
      for (int j = k >> 1; j > 0; j >>= 1) {
        const int p = t ^ j;
        if (p > t) {
          const unsigned a = s_key[t], b = s_key[p];
          const bool up = (t & k) == 0;
          if ((a > b) == up) {
            s_key[t] = b;
            s_key[p] = a;
          }
        }
        __syncthreads();
      }
    }
    // thread t now handles sorted position t
    const unsigned k0 = s_key[t];
    int st = -1, first = 0;
    bool last = false;
    if (k0 != 0xFFFFFFFFu) {
      st = (int)(k0 >> 10);
      const unsigned lo_key = (unsigned)st << 10;
      int lo = 0, hi = t;  // first position with key >= lo_key
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (s_key[mid] < lo_key) lo = mid + 1;
        else hi = mid;
      }
      first = lo;
      const int src = (int)(k0 & 1023u);
      const int dst = s_cur[st] + (t - first);
      opk[dst] = s_pk[src];
      oval[dst] = s_val[src];
      last = (t + 1 == kST) || (int)(s_key[t + 1] >> 10) != st;
    }
    __syncthreads();
    if (last) s_cur[st] += t + 1 - first;
    __syncthreads();
  }
}

// Row-aligned wave ranges of every segment: wave w starts at the first row
// start at or after segment start + len * w / 16.
__global__ void k_st_split(const unsigned* __restrict__ pk, const int* __restrict__ seg, long long nseg,
                           int* __restrict__ wsp) {
  const long long total = nseg * kSWaves;
  for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < total;
       q += (long long)gridDim.x * blockDim.x) {
    const long long g = q / kSWaves;
    const int w = (int)(q % kSWaves);
    const int b0 = seg[g], b1 = seg[g + 1];
    int t = b0 + (int)((long long)(b1 - b0) * w / kSWaves);
    while (t > b0 && t < b1 && (pk[t] >> 16) == (pk[t - 1] >> 16)) ++t;
    wsp[q] = t;
  }
}

// Reorder every window of every wave range lane-interleaved into entry
// records: the lane's k-th entry (its entries are consecutive in CSR order)
// goes to record window start + 64 k + lane.  One wave per (segment, wave)
// range.
__device__ __forceinline__ void put_rec(unsigned* rec, long long i, unsigned pk, double v) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  rec[3 * i] = (unsigned)b;
  rec[3 * i + 1] = (unsigned)(b >> 32);
  rec[3 * i + 2] = pk;
}
__device__ __forceinline__ void put_rec(unsigned* rec, long long i, unsigned pk, float v) {
  rec[2 * i] = __builtin_bit_cast(unsigned, v);
  rec[2 * i + 1] = pk;
}
template <class Val>
__global__ void k_st_interleave(const unsigned* __restrict__ pk, const Val* __restrict__ val,
                                const int* __restrict__ seg, const int* __restrict__ wsp, long long nseg,
                                int qmax, unsigned* __restrict__ rec) {
  const int lane = threadIdx.x & 63;
  const long long nw = (long long)gridDim.x * (blockDim.x >> 6);
  for (long long q = (long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); q < nseg * kSWaves; q += nw) {
    const long long g = q / kSWaves;
    const int w = (int)(q % kSWaves);
    const int ws = wsp[q], we = (w + 1 < kSWaves) ? wsp[q + 1] : seg[g + 1];
    if (we <= ws) continue;
    const int Q = range_q(we - ws, qmax);
    for (int base = ws; base < we; base += 64 * Q) {
      const int c = min(64 * Q, we - base);
      const int Qw = (c + 63) >> 6, r = c - 64 * (Qw - 1);
      const int mine = lane < r ? Qw : Qw - 1;
      const int start = lane < r ? lane * Qw : r * Qw + (lane - r) * (Qw - 1);
      for (int k = 0; k < mine; ++k) put_rec(rec, base + 64 * k + lane, pk[base + start + k], val[base + start + k]);
    }
  }
}

// ------------------------------------------------------------------ product

// One workgroup per (system, unit).  MODE_RESID: r <- r - A p, partial rho
// per unit.  MODE_TRANSB: ypart[b] <- A_bᵀ r_b for row block b of A (the
// unit list entry carries b << 24 | unit).  MODE_REFINE: r64 <- b - A x in
// float64, partials of ||r64||^2 and ||b||^2.  MODE_PLAIN: r64 <- A p
// (float64), or ypart[b] <- A_bᵀ p for a transposed store; no state.
template <class Val, class Vin, class Acc, int MODE, int SW, int RB, int QM>
__global__ __launch_bounds__(kST) void k_sspmv(const Desc* __restrict__ D, const int2* __restrict__ list,
                                               int transposed) {
  __shared__ __attribute__((aligned(16))) Acc s_x[2][SW];
  // float row sums: 64 spare words past the unit's rows (see sum_window)
  __shared__ Acc s_acc[RB + (sizeof(Acc) == 4 ? 64 : 0)];
  // the epilogue's cross-wave partial sums reuse the slice buffers (no wave
  // reads them after the stripe loop's last barrier)
  double (*s_red)[kSWaves] = reinterpret_cast<double (*)[kSWaves]>(&s_x[0][0]);
  // staging of the vector slice: XE elements per load, XC loads per thread.
  // Float64 slices of four or more elements per thread go two to a load;
  // wider loads measured slower for the narrower slices and for float32.
  constexpr int XE = (sizeof(Vin) == 8 && SW / kST >= 4 && (SW / kST) % 2 == 0) ? 2 : 1;
  constexpr int XC = SW / (kST * XE);
  static_assert(XC * XE * kST == SW, "stripe width must be a multiple of the workgroup size");

  const int2 ent = list[blockIdx.x];
  if (ent.y < 0) return;  // padding of an XCD-interleaved list
  const Desc* d = D + ent.x;
  // The iteration's products (RESID, TRANSB) run far more often than they
  // skip, so they read the state's flags beside the first loads of the
  // product and leave only once those are issued: the flags' load then does
  // not lengthen the chain of dependent loads before the stream starts.  A
  // skipped launch reads a little of the store for nothing.
  constexpr bool kLate = MODE == MODE_RESID || MODE == MODE_TRANSB;
  bool skip = false;
  if (MODE != MODE_PLAIN) {
    const State* st = d->st;
    if (MODE == MODE_REFINE) {
      if (st->final_done || !st->done) return;
    } else {
      // all three read at once (no short-circuit: each test would wait for
      // its own load before the next is issued)
      const int fd = st->final_done, dn = st->done;
      const long long kk = MODE == MODE_RESID ? st->k : 1;
      skip = ((fd | dn) != 0) | (kk == 0);
      if (!kLate && skip) return;
    }
  }
  const bool tb = MODE == MODE_TRANSB || (MODE == MODE_PLAIN && transposed);
  const int blk = tb ? (ent.y >> 24) : 0;
  const int u = tb ? (ent.y & 0xFFFFFF) : ent.y;
  const StripeView& sv = tb ? d->sb[blk] : d->sa;
  const unsigned* __restrict__ rec = sv.rec;
  const int S = sv.S;
  const int r0 = sv.urow[u], nr = sv.urow[u + 1] - r0;
  const Vin* __restrict__ x;
  int xlen;
  if (MODE == MODE_RESID || (MODE == MODE_PLAIN && !tb)) {
    x = static_cast<const Vin*>(d->p);
    xlen = d->n;
  } else if (MODE == MODE_REFINE) {
    x = reinterpret_cast<const Vin*>(d->xo);
    xlen = d->n;
  } else if (MODE == MODE_TRANSB) {
    x = static_cast<const Vin*>(d->r) + sv.colbase;
    xlen = sv.ncols;
  } else {
    x = static_cast<const Vin*>(d->p) + sv.colbase;
    xlen = sv.ncols;
  }
  // the wave index is uniform: wave bounds come through scalar loads and the
  // window loop runs on scalar control flow
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);

  const int* __restrict__ seg = sv.seg + (size_t)u * S;
  const int* __restrict__ wsp = sv.wsp + (size_t)u * S * kSWaves;
  auto bounds = [&](int s, int& ws, int& we) {
    if (s < S) {
      ws = gload(&wsp[s * kSWaves + w]);
      we = (w + 1 < kSWaves) ? gload(&wsp[s * kSWaves + w + 1]) : gload(&seg[s + 1]);
    } else {
      ws = we = 0;
    }
  };
  // Two register sets alternate over the stripes: while stripe s is summed
  // from set "cur" (bounds and first window), the other set receives stripe
  // s + 1's first window (its bounds came a stripe earlier), and cur's
  // bounds then take stripe s + 2.  The loop is unrolled by two so the sets
  // keep fixed registers instead of being copied every stripe.
  int wsA, weA, wsB, weB;
  Ent<Val> eA[QM], eB[QM];
  bounds(0, wsA, weA);
  bounds(1, wsB, weB);
  load_window<Val, QM>(rec, wsA, min(64 * range_q(weA - wsA, QM), weA - wsA), eA);

  for (int i = threadIdx.x; i < nr; i += kST) s_acc[i] = Acc(0);
  for (int j = threadIdx.x; j < SW; j += kST) s_x[0][j] = j < xlen ? Acc(gload(&x[j])) : Acc(0);
  if (kLate && skip) return;  // the same for the whole workgroup
  __syncthreads();

  auto stripe = [&](int s, int& ws0, int& we0, const Ent<Val>* ce, int ws1, int we1, Ent<Val>* me) {
    // the next stripe's slice of x travels in registers during this stripe:
    // chunk c of thread t holds elements c kST XE + t XE .. + XE - 1, one
    // load each.  With XE > 1 a chunk that crosses the end of x loads the
    // last XE elements of x instead and picks its own out of them by index
    // (a vector shorter than XE is read from its start: every vector the
    // products read sits in an allocation of at least 16 bytes), so every
    // thread issues the same load without a branch.
    Acc nx[XC][XE];
#pragma unroll
    for (int c = 0; c < XC; ++c) {
      const int j0 = (s + 1) * SW + (c * kST + (int)threadIdx.x) * XE;
      if constexpr (XE == 1) {
        nx[c][0] = (s + 1 < S && j0 < xlen) ? Acc(gload(&x[j0])) : Acc(0);
      } else {
        const int jt = xlen > XE ? xlen - XE : 0;
        const int jc = j0 + XE <= xlen ? j0 : jt;
        const auto v = gload_vec<Vin, XE>(&x[jc]);
#pragma unroll
        for (int e = 0; e < XE; ++e) {
          const int k = j0 + e - jc;  // in [0, XE) for every element below xlen
          Vin pick = vec_elem(v, 0);
#pragma unroll
          for (int i = 1; i < XE; ++i) pick = k == i ? vec_elem(v, i) : pick;
          nx[c][e] = (s + 1 < S && j0 + e < xlen) ? Acc(pick) : Acc(0);
        }
      }
    }
    int ws2, we2;
    bounds(s + 2, ws2, we2);
    load_window<Val, QM>(rec, ws1, min(64 * range_q(we1 - ws1, QM), we1 - ws1), me);

    const Acc* __restrict__ xs = s_x[s & 1];
    if (we0 > ws0) {
      const int Q = range_q(we0 - ws0, QM);
      Acc wc = Acc(0);  // run open at the end of the previous window
      int wr = -1;
      sum_window<Val, Acc, QM, RB>(min(64 * Q, we0 - ws0), ce, xs, s_acc, wc, wr);
      for (int base = ws0 + 64 * Q; base < we0; base += 64 * Q) {
        const int c = min(64 * Q, we0 - base);
        Ent<Val> ev[QM];
        load_window<Val, QM>(rec, base, c, ev);
        sum_window<Val, Acc, QM, RB>(c, ev, xs, s_acc, wc, wr);
      }
      flush_open(s_acc, wc, wr);
    }
#pragma unroll
    for (int c = 0; c < XC; ++c)
#pragma unroll
      for (int e = 0; e < XE; ++e) s_x[(s + 1) & 1][(c * kST + threadIdx.x) * XE + e] = nx[c][e];
    ws0 = ws2;
    we0 = we2;
    __syncthreads();
  };
  for (int s = 0; s < S; s += 2) {
    stripe(s, wsA, weA, eA, wsB, weB, eB);
    if (s + 1 >= S) break;
    stripe(s + 1, wsB, weB, eB, wsA, weA, eA);
  }

  // epilogue over the unit's rows
  double part = 0.0, part2 = 0.0;
  for (int i = threadIdx.x; i < nr; i += kST) {
    const int row = r0 + i;
    const Acc sum = s_acc[i];
    if (MODE == MODE_RESID) {
      Vin* r = static_cast<Vin*>(d->r);
      const Acc rn = Acc(r[row]) - sum;
      r[row] = Vin(rn);
      part += double(rn) * double(rn);
    } else if (MODE == MODE_TRANSB) {
      static_cast<Vin*>(d->ypart)[(size_t)blk * d->n + row] = Vin(sum);
    } else if (MODE == MODE_REFINE) {
      const double bi = d->b[row];
      const double ri = bi - double(sum);
      d->r64[row] = ri;
      part += ri * ri;
      part2 += bi * bi;
    } else if (tb) {
      static_cast<double*>(d->ypart)[(size_t)blk * d->n + row] = double(sum);
    } else {
      d->r64[row] = double(sum);
    }
  }
  if (MODE == MODE_TRANSB || MODE == MODE_PLAIN) return;
  part = swsum(part);
  part2 = swsum(part2);
  if (lane == 0) {
    s_red[0][w] = part;
    s_red[1][w] = part2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = s_red[0][0], b2 = s_red[1][0];
    for (int q = 1; q < kSWaves; ++q) {
      a += s_red[0][q];
      b2 += s_red[1][q];
    }
    d->part_rho[u] = a;
    if (MODE == MODE_REFINE) d->part_b[u] = b2;
  }
}

// y_j = sum over row blocks of ypart[b][j] in block order (plain products)
__global__ void k_st_ysum(const double* __restrict__ yp, int nblk, int n, double* __restrict__ y) {
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
    double s = yp[j];
    for (int b = 1; b < nblk; ++b) s += yp[(size_t)b * n + j];
    y[j] = s;
  }
}

// ------------------------------------------------------------------ host side

static int st_grid(long long work, int per_block) {
  long long g = (work + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > 65536) g = 65536;
  return (int)g;
}

void st_count(const int* ptr, const int* idx, int nunits, const int* d_urow, int S, int colbase, int sw, int* d_cnt,
              hipStream_t s) {
  if (nunits <= 0 || S <= 0) return;
  k_st_count<<<nunits, kST, sizeof(int) * (size_t)S, s>>>(ptr, idx, d_urow, S, colbase, sw, d_cnt);
  PLSS_HIP(hipGetLastError());
}

void st_scatter(const int* ptr, const int* idx, const void* val, bool f32, int nunits, const int* d_urow,
                const int* d_seg, int S, int colbase, int sw, unsigned* opk, void* oval, hipStream_t s) {
  if (nunits <= 0 || S <= 0) return;
  const size_t lds = sizeof(int) * (size_t)S;
  if (f32)
    k_st_scatter<float><<<nunits, kST, lds, s>>>(ptr, idx, static_cast<const float*>(val), d_urow, d_seg, S,
                                                 colbase, sw, opk, static_cast<float*>(oval));
  else
    k_st_scatter<double><<<nunits, kST, lds, s>>>(ptr, idx, static_cast<const double*>(val), d_urow, d_seg, S,
                                                  colbase, sw, opk, static_cast<double*>(oval));
  PLSS_HIP(hipGetLastError());
}

void st_split(const unsigned* pk, const int* d_seg, long long nseg, int* d_wsp, hipStream_t s) {
  if (nseg <= 0) return;
  k_st_split<<<st_grid(nseg * kSWaves, 256), 256, 0, s>>>(pk, d_seg, nseg, d_wsp);
  PLSS_HIP(hipGetLastError());
}

void st_interleave(const unsigned* pk, const void* val, bool f32, const int* d_seg, const int* d_wsp, long long nseg,
                   int qmax, unsigned* rec, hipStream_t s) {
  if (nseg <= 0) return;
  const int grid = st_grid(nseg * kSWaves * 64, 256);
  if (f32)
    k_st_interleave<float><<<grid, 256, 0, s>>>(pk, static_cast<const float*>(val), d_seg, d_wsp, nseg, qmax, rec);
  else
    k_st_interleave<double><<<grid, 256, 0, s>>>(pk, static_cast<const double*>(val), d_seg, d_wsp, nseg, qmax,
                                                 rec);
  PLSS_HIP(hipGetLastError());
}

void st_ysum(const double* ypart, int nblk, int n, double* y, hipStream_t s) {
  k_st_ysum<<<st_grid(n, 256), 256, 0, s>>>(ypart, nblk, n, y);
  PLSS_HIP(hipGetLastError());
}

void launch_sspmv(int mode, bool f32, const Desc* d, const int2* list, int n, int transposed, hipStream_t s) {
  if (n <= 0) return;
  constexpr int A1 = kSWA, A2 = kRBA, A3 = kQmaxA, T1 = kSWT, T2 = kRBT, T3 = kQmaxT;
  constexpr int A1f = kSWA32, A3f = kQmaxA32, T1f = kSWT32, T3f = kQmaxT32;
  if (!f32) {
    switch (mode) {
      case MODE_RESID: k_sspmv<double, double, double, MODE_RESID, A1, A2, A3><<<n, kST, 0, s>>>(d, list, 0); break;
      case MODE_TRANSB: k_sspmv<double, double, double, MODE_TRANSB, T1, T2, T3><<<n, kST, 0, s>>>(d, list, 1); break;
      case MODE_REFINE: k_sspmv<double, double, double, MODE_REFINE, A1, A2, A3><<<n, kST, 0, s>>>(d, list, 0); break;
      default:
        if (transposed) k_sspmv<double, double, double, MODE_PLAIN, T1, T2, T3><<<n, kST, 0, s>>>(d, list, 1);
        else k_sspmv<double, double, double, MODE_PLAIN, A1, A2, A3><<<n, kST, 0, s>>>(d, list, 0);
        break;
    }
  } else {
    switch (mode) {
      case MODE_RESID: k_sspmv<float, float, float, MODE_RESID, A1f, A2, A3f><<<n, kST, 0, s>>>(d, list, 0); break;
      case MODE_TRANSB: k_sspmv<float, float, float, MODE_TRANSB, T1f, T2, T3f><<<n, kST, 0, s>>>(d, list, 1); break;
      case MODE_REFINE:
        k_sspmv<float, double, double, MODE_REFINE, A1f, A2, A3f><<<n, kST, 0, s>>>(d, list, 0);
        break;
      default:
        // the float64-accumulating plain product does not fit the float32
        // stores of Aᵀ (their stripes are 8192 wide): callers use the tiles
        if (transposed) throw InvalidArg{"plain transposed product on a float32 striped store"};
        k_sspmv<float, double, double, MODE_PLAIN, A1f, A2, A3f><<<n, kST, 0, s>>>(d, list, 0);
        break;
    }
  }
  PLSS_HIP(hipGetLastError());
}

}  // namespace plss
