// Matrix store: upload, validation, CSC build, tile tables.
#include "runtime.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>

#include "fused.hpp"

namespace plss {

void* dmalloc(size_t bytes) {
  void* p = nullptr;
  // at least 16 bytes, in whole 16-byte units: the striped products read a
  // vector shorter than one 16-byte load from its start
  bytes = bytes == 0 ? 16 : (bytes + 15) / 16 * 16;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw OutOfMemory{"hipMalloc of " + std::to_string(bytes) + " bytes failed: " +
                      hipGetErrorString(e)};
  }
  return p;
}

void dfree(void* p) {
  if (p) (void)hipFree(p);
}

std::vector<int> make_tiles(const std::vector<int>& ptr, int V) {
  const int T = tile_nnz(V);
  const int nrows = (int)ptr.size() - 1;
  std::vector<int> t;
  t.reserve(nrows / 8 + 2);
  t.push_back(0);
  long long cur = 0;
  int rows = 0;
  for (int i = 0; i < nrows; ++i) {
    const long long L = (long long)ptr[i + 1] - ptr[i];
    if (rows > 0 && (cur + L > T || rows == T)) {
      t.push_back(i);
      cur = 0;
      rows = 0;
    }
    cur += L;
    rows += 1;
  }
  if (nrows > 0) t.push_back(nrows);
  return t;
}

// Groups of 4 wave tiles for one workgroup each.  Tiles of one long row
// are sorted by length (longest first) and grouped with tiles of similar
// length, so no workgroup waits on one long row beside three short tiles;
// short tiles are grouped in row order.  Long groups come first in the
// launch order.
std::vector<int> make_groups(const std::vector<int>& ptr, const std::vector<int>& tiles, int V) {
  const int TW = tile_nnz(V);
  const int nwt = (int)tiles.size() - 1;
  std::vector<int> lng, sht;
  for (int t = 0; t < nwt; ++t) {
    const long long ne = (long long)ptr[tiles[t + 1]] - ptr[tiles[t]];
    (ne > TW ? lng : sht).push_back(t);
  }
  std::stable_sort(lng.begin(), lng.end(), [&](int a, int b) {
    return ptr[tiles[a] + 1] - ptr[tiles[a]] > ptr[tiles[b] + 1] - ptr[tiles[b]];
  });
  std::vector<int> g;
  for (auto* v : {&lng, &sht}) {
    for (size_t i = 0; i < v->size(); i += kWaves)
      for (int w = 0; w < kWaves; ++w) g.push_back(i + w < v->size() ? (*v)[i + w] : -1);
  }
  if (g.empty()) g.assign(kWaves, -1);
  return g;
}

void set_tiles(PlssDir& d, int V, hipStream_t s) {
  std::vector<int> t = make_tiles(d.h_ptr, V);
  std::vector<int> g = make_groups(d.h_ptr, t, V);
  // each wave's tile in one record, so a product reads its bounds with one
  // load instead of group -> tile -> row pointer
  std::vector<int4> wd(g.size());
  for (size_t q = 0; q < g.size(); ++q) {
    const int wt = g[q];
    wd[q] = wt >= 0 ? make_int4(t[wt], t[wt + 1], d.h_ptr[t[wt]], d.h_ptr[t[wt + 1]]) : make_int4(0, 0, 0, 0);
  }
  dfree(d.tile);
  dfree(d.grp);
  dfree(d.wtd);
  d.tile = nullptr;
  d.grp = nullptr;
  d.wtd = nullptr;
  d.tile = static_cast<int*>(dmalloc(sizeof(int) * t.size()));
  d.grp = static_cast<int*>(dmalloc(sizeof(int) * g.size()));
  d.wtd = static_cast<int4*>(dmalloc(sizeof(int4) * std::max<size_t>(wd.size(), 1)));
  PLSS_HIP(hipMemcpyAsync(d.tile, t.data(), sizeof(int) * t.size(), hipMemcpyHostToDevice, s));
  PLSS_HIP(hipMemcpyAsync(d.grp, g.data(), sizeof(int) * g.size(), hipMemcpyHostToDevice, s));
  if (!wd.empty()) PLSS_HIP(hipMemcpyAsync(d.wtd, wd.data(), sizeof(int4) * wd.size(), hipMemcpyHostToDevice, s));
  PLSS_HIP(hipStreamSynchronize(s));
  d.nwt = (int)t.size() - 1;
  d.ntiles = (int)g.size() / kWaves;
  d.V = V;
}

// Slice layout of a direction for the single-workgroup solve: rows of at most
// 64 entries in slices of 64 rows, each slice as wide as its longest such row
// (rounded up to 4); entry k of row 64 s + l at sl_base[s] + (k / 4) * 256 +
// 4 l + k % 4, so the lanes of a wave, one row each, read 4 entries apiece from
// one contiguous 1 KB (indices) span per load instead of from 64 rows apart.
void set_slices(PlssDir& d, bool f32, hipStream_t s) {
  const int nr = d.nrows, nsl = (nr + 63) / 64;
  std::vector<int> base(nsl + 1, 0);
  for (int q = 0; q < nsl; ++q) {
    int w = 0;
    for (int l = 0; l < 64; ++l) {
      const int i = 64 * q + l;
      if (i >= nr) break;
      const int len = d.h_ptr[i + 1] - d.h_ptr[i];
      if (len <= 64) w = std::max(w, len);
    }
    base[q + 1] = base[q] + (w + 3) / 4 * 4 * 64;
  }
  const long long nnz = d.h_ptr[nr];
  const size_t vb = f32 ? 4 : 8, tot = std::max(base[nsl], 1);
  std::vector<int> hidx((size_t)std::max<long long>(nnz, 1));
  std::vector<char> hval((size_t)std::max<long long>(nnz, 1) * vb);
  if (nnz > 0) {
    PLSS_HIP(hipMemcpyAsync(hidx.data(), d.idx, sizeof(int) * nnz, hipMemcpyDeviceToHost, s));
    PLSS_HIP(hipMemcpyAsync(hval.data(), d.val, vb * nnz, hipMemcpyDeviceToHost, s));
    PLSS_HIP(hipStreamSynchronize(s));
  }
  std::vector<int> sidx(tot, 0);
  std::vector<char> sval(tot * vb, 0);
  for (int i = 0; i < nr; ++i) {
    const int e0 = d.h_ptr[i], len = d.h_ptr[i + 1] - e0;
    if (len > 64) continue;
    const int sb = base[i / 64] + 4 * (i % 64);
    for (int k = 0; k < len; ++k) {
      const int o = sb + (k / 4) * 256 + k % 4;
      sidx[o] = hidx[e0 + k];
      std::memcpy(&sval[(size_t)o * vb], &hval[(size_t)(e0 + k) * vb], vb);
    }
  }
  dfree(d.sl_base);
  dfree(d.sl_idx);
  dfree(d.sl_val);
  d.sl_base = static_cast<int*>(dmalloc(sizeof(int) * (nsl + 1)));
  d.sl_idx = static_cast<int*>(dmalloc(sizeof(int) * tot));
  d.sl_val = dmalloc(vb * tot);
  PLSS_HIP(hipMemcpyAsync(d.sl_base, base.data(), sizeof(int) * (nsl + 1), hipMemcpyHostToDevice, s));
  PLSS_HIP(hipMemcpyAsync(d.sl_idx, sidx.data(), sizeof(int) * tot, hipMemcpyHostToDevice, s));
  PLSS_HIP(hipMemcpyAsync(d.sl_val, sval.data(), vb * tot, hipMemcpyHostToDevice, s));
  PLSS_HIP(hipStreamSynchronize(s));
  d.sl_n = (long long)tot;
}

void set_long_rows(PlssDir& d, hipStream_t s) {
  std::vector<int> l;
  for (int i = 0; i < d.nrows; ++i)
    if (d.h_ptr[i + 1] - d.h_ptr[i] > 64) l.push_back(i);
  dfree(d.lrows);
  d.lrows = static_cast<int*>(dmalloc(sizeof(int) * std::max<size_t>(1, l.size())));
  if (!l.empty()) {
    PLSS_HIP(hipMemcpyAsync(d.lrows, l.data(), sizeof(int) * l.size(), hipMemcpyHostToDevice, s));
    PLSS_HIP(hipStreamSynchronize(s));
  }
  d.nlong = (int)l.size();
}

size_t matrix_footprint(long long m, long long n, long long nnz, bool f32) {
  const size_t v = f32 ? 4 : 8;
  const bool blocked = (size_t)m * v > (3u << 20) && nnz >= 8 * 64;
  bool as = false, ts = false;
  auto_layout(m, n, nnz, f32, &as, &ts);
  const int copies = 2 + (blocked ? 1 : 0) + (as ? 1 : 0) + (ts ? 1 : 0);
  // slice layouts of a system that fits the single-workgroup solve: at most
  // 64 entries per row and direction, padding included
  const size_t slices = small_fits((int)m, (int)n, f32) ? (size_t)64 * (m + n + 128) * (v + 4) : 0;
  return slices + (size_t)nnz * (v + 4) * copies + (size_t)(m + n + 2) * 4 + (size_t)(m + n) / 64 * 4 +
         (blocked ? (size_t)kMaxBlk * (n + 1) * 4 : 0) + ((as || ts) ? (size_t)(m + n) / 64 * 4 + (1u << 20) : 0) +
         4096;
}

// ------------------------------------------------------------------ striped layout

int auto_unit_rows(long long rows, int nblk, int rbmax) {
  // units per block: enough for the 256 CUs over all blocks, rounded so that
  // every XCD gets the same count, and at most rbmax rows each
  const long long per_round = (256 + nblk - 1) / nblk;
  long long nu = (rows + rbmax - 1) / rbmax;
  nu = (nu + per_round - 1) / per_round * per_round;
  long long R = (rows + nu - 1) / nu;
  R = std::max<long long>(R, std::min<long long>(rows, 512));
  return (int)std::max<long long>(1, std::min<long long>(R, rbmax));
}

// Stripes pay when the gathered vector is re-read less than the entries are
// streamed: every unit reads its whole slice of the vector once.
void auto_layout(long long m, long long n, long long nnz, bool f32, bool* a_stripes, bool* t_stripes) {
  *a_stripes = *t_stripes = false;
  const double vb = f32 ? 4.0 : 8.0;
  if (nnz < (1LL << 23)) return;
  const double entry_bytes = (double)nnz * (4.0 + vb);
  {
    const int R = auto_unit_rows(m, 1, kRBA);
    const long long nu = (m + R - 1) / R;
    const long long S = (n + swa(f32) - 1) / swa(f32);
    if (S <= kMaxStripes && nu >= 128 && (double)nu * (double)n * vb <= 0.75 * entry_bytes) *a_stripes = true;
  }
  if ((double)m * vb > (double)(3u << 20)) {
    const int R = auto_unit_rows(n, kMaxBlk, kRBT);
    const long long nu = (long long)kMaxBlk * ((n + R - 1) / R);
    const long long S = (m / kMaxBlk + swt(f32)) / swt(f32);
    if (S <= kMaxStripes && nu >= 128 && (double)nu * ((double)m / kMaxBlk) * vb <= entry_bytes) *t_stripes = true;
  }
}

static void free_stripes(PlssStripes& st) {
  dfree(st.rec);
  dfree(st.urow);
  dfree(st.seg);
  dfree(st.wsp);
  st = PlssStripes();
}

void fill_stripe_view(const PlssStripes& st, StripeView* v) {
  v->rec = st.rec;
  v->urow = st.urow;
  v->seg = st.seg;
  v->wsp = st.wsp;
  v->nunits = st.nunits;
  v->S = st.S;
  v->colbase = st.colbase;
  v->ncols = st.ncols;
  v->sw = st.sw;
}

// Row starts of the units of a striped store over CSR row pointers ptr.
// Plain: units of R rows.  Balanced: at most ceil(rows / R) units of at most
// cap rows (cap >= R) whose largest entry count is as small as a greedy
// split can make it: the least bound T (binary search) for which cutting
// each unit at the last row that keeps it within T entries (at least one
// row, at most cap) needs no more units.  A launch ends with its heaviest
// unit, so with rows of very different lengths equal row counts leave most
// of the chip waiting for a few units.
std::vector<int> unit_starts(const std::vector<int>& ptr, int rows, int R, int cap, bool balance) {
  std::vector<int> st(1, 0);
  if (rows <= 0) return st;
  const int U = (rows + R - 1) / R;
  if (!balance) {
    for (int u = 1; u <= U; ++u) st.push_back((int)std::min<long long>(rows, (long long)u * R));
    return st;
  }
  auto split = [&](long long T, std::vector<int>* out) {
    int r = 0, u = 0;
    while (r < rows && u <= U) {
      const long long lim = (long long)ptr[r] + T;
      int e = (int)(std::upper_bound(ptr.begin() + r, ptr.begin() + rows + 1, lim) - ptr.begin()) - 1;
      e = std::min(std::max(e, r + 1), std::min(r + cap, rows));
      r = e;
      ++u;
      if (out) out->push_back(r);
    }
    return r < rows ? U + 1 : u;
  };
  const long long total = ptr[rows] - ptr[0];
  long long lo = (total + U - 1) / U, hi = std::max<long long>(lo, total);
  while (lo < hi) {  // split(total) fits: units of cap >= R rows, at most U of them
    const long long mid = lo + (hi - lo) / 2;
    if (split(mid, nullptr) <= U) hi = mid;
    else lo = mid + 1;
  }
  split(lo, &st);
  return st;
}

// Striped copy of the CSR direction `src` restricted to columns
// [colbase, colbase + ncols) (all of its entries lie there), in units of R
// rows or (balance) units balanced by entry count of at most cap rows.
static void build_stripes(const PlssDir& src, int colbase, int ncols, int R, int cap, bool balance, int sw, int qmax,
                          bool f32, PlssStripes& out, hipStream_t s) {
  const int rows = src.nrows;
  const long long nnz = src.h_ptr[rows];
  const std::vector<int> urow = unit_starts(src.h_ptr, rows, R, cap, balance);
  const int nunits = (int)urow.size() - 1;
  const int S = (ncols + sw - 1) / sw;
  if (S > kMaxStripes) throw InvalidArg{"too many columns for the striped layout"};
  const long long nseg = (long long)nunits * S;
  if (nseg * 16 >= (1LL << 31) - 1) throw InvalidArg{"too many stripe segments: raise unit_rows"};
  const size_t vb = f32 ? 4 : 8;
  PlssStripes st;
  int* cnt = nullptr;
  void* work = nullptr;
  unsigned* pk = nullptr;  // CSR-ordered entries of the segments, before the records
  void* val = nullptr;
  try {
    st.urow = static_cast<int*>(dmalloc(sizeof(int) * urow.size()));
    st.seg = static_cast<int*>(dmalloc(sizeof(int) * (size_t)(nseg + 1)));
    st.wsp = static_cast<int*>(dmalloc(sizeof(int) * (size_t)std::max<long long>(nseg * 16, 1)));
    pk = static_cast<unsigned*>(dmalloc(sizeof(unsigned) * (size_t)std::max<long long>(nnz, 1)));
    val = dmalloc(vb * (size_t)std::max<long long>(nnz, 1));
    cnt = static_cast<int*>(dmalloc(sizeof(int) * (size_t)std::max<long long>(nseg, 1)));
    work = dmalloc(sizeof(long long) * (size_t)((nseg + 1023) / 1024 + 2));
    PLSS_HIP(hipMemcpyAsync(st.urow, urow.data(), sizeof(int) * urow.size(), hipMemcpyHostToDevice, s));
    st_count(src.ptr, src.idx, nunits, st.urow, S, colbase, sw, cnt, s);
    scan_counts(cnt, (int)nseg, st.seg, work, s);
    int total = 0;
    PLSS_HIP(hipMemcpyAsync(&total, st.seg + nseg, sizeof(int), hipMemcpyDeviceToHost, s));
    PLSS_HIP(hipStreamSynchronize(s));
    if (total != nnz) {
      set_error("striped store: entry count mismatch");
      throw DeviceError();
    }
    st_scatter(src.ptr, src.idx, src.val, f32, nunits, st.urow, st.seg, S, colbase, sw, pk, val, s);
    st_split(pk, st.seg, nseg, st.wsp, s);
    // lane-interleaved windows of entry records (the padding past the end
    // is zero: row 0, column 0, value 0)
    const size_t words = (size_t)rec_words(f32);
    st.rec = static_cast<unsigned*>(dmalloc(sizeof(unsigned) * words * (size_t)(nnz + kStorePad)));
    PLSS_HIP(hipMemsetAsync(st.rec + words * (size_t)nnz, 0, sizeof(unsigned) * words * kStorePad, s));
    st_interleave(pk, val, f32, st.seg, st.wsp, nseg, qmax, st.rec, s);
    PLSS_HIP(hipStreamSynchronize(s));
  } catch (...) {
    dfree(cnt);
    dfree(work);
    dfree(pk);
    dfree(val);
    free_stripes(st);
    throw;
  }
  dfree(cnt);
  dfree(work);
  dfree(pk);
  dfree(val);
  st.nunits = nunits;
  st.S = S;
  st.colbase = colbase;
  st.ncols = ncols;
  st.unit_rows = R;
  st.balanced = balance;
  st.sw = sw;
  st.nnz = nnz;
  st.bytes = (size_t)(nnz + kStorePad) * (4 + vb) + sizeof(int) * (size_t)(nunits + 1 + (nseg + 1) + nseg * 16);
  free_stripes(out);
  out = st;
}

static void recount_bytes(plss_matrix* M) {
  const size_t vsz = M->f32 ? 4 : 8;
  const long long m = M->m, n = M->n, nnz = M->nnz;
  size_t b = (size_t)nnz * (vsz + 4) * (M->nblk > 1 ? 3 : 2) + sizeof(int) * (size_t)(m + n + 2) +
             sizeof(int) * (size_t)(M->A.ntiles + M->T.ntiles + 2) +
             (M->nblk > 1 ? sizeof(int) * (size_t)M->nblk * (n + 1) : 0);
  if (M->cnblk > 1) b += (size_t)nnz * (vsz + 4) + sizeof(int) * (size_t)M->cnblk * (m + 1);
  if (M->fz_pos) b += (size_t)std::max<long long>(nnz, 1) * (sizeof(int) + sizeof(double));
  for (const PlssDir* d : {&M->A, &M->T})
    if (d->sl_base) b += (size_t)d->sl_n * (vsz + 4) + sizeof(int) * (size_t)((d->nrows + 63) / 64 + 1);
  b += M->SA.bytes;
  for (int q = 0; q < kMaxBlk; ++q) b += M->SB[q].bytes;
  M->bytes = b;
}

void matrix_set_layout(plss_matrix* M, bool a_stripes, bool t_stripes, int unit_rows, hipStream_t s) {
  if (unit_rows < 0 || unit_rows > kRBT) throw InvalidArg{"unit_rows must be in [0, 16384]"};
  try {
    if (a_stripes) {
      const int R = unit_rows ? std::min(unit_rows, kRBA) : auto_unit_rows(M->m, 1, kRBA);
      const bool bal = unit_rows == 0;
      if (!M->a_striped || M->SA.unit_rows != R || M->SA.balanced != bal) {
        M->a_striped = false;
        build_stripes(M->A, 0, (int)M->n, R, kRBA, bal, swa(M->f32), qa(M->f32), M->f32, M->SA, s);
      }
    } else {
      free_stripes(M->SA);
    }
    M->a_striped = a_stripes;
    if (t_stripes) {
      build_row_blocks(M, s, true);
      const int R = unit_rows ? std::min(unit_rows, kRBT) : auto_unit_rows(M->n, M->nblk, kRBT);
      // the row blocks' units have near-equal entry counts already when
      // their rows (columns of A) are; balancing them measured no faster
      const bool bal = false;
      if (!M->t_striped || M->SB[0].unit_rows != R || M->SB[0].balanced != bal) {
        M->t_striped = false;
        for (int b = 0; b < M->nblk; ++b)
          build_stripes(M->TB[b], M->rb[b], M->rb[b + 1] - M->rb[b], R, kRBT, bal, swt(M->f32), qt(M->f32), M->f32,
                        M->SB[b], s);
      }
    } else {
      for (int b = 0; b < kMaxBlk; ++b) free_stripes(M->SB[b]);
    }
    M->t_striped = t_stripes;
  } catch (...) {
    if (!M->a_striped) free_stripes(M->SA);
    if (!M->t_striped)
      for (int b = 0; b < kMaxBlk; ++b) free_stripes(M->SB[b]);
    recount_bytes(M);
    throw;
  }
  recount_bytes(M);
}

static void check_args(const plss_csr* A) {
  if (!A) throw InvalidArg{"null matrix"};
  if (A->m <= 0 || A->n <= 0) throw InvalidArg{"m and n must be positive"};
  if (A->m >= (1LL << 31) - 1 || A->n >= (1LL << 31) - 1)
    throw InvalidArg{"m and n must be below 2^31-1"};
  if (A->nnz < 0 || A->nnz >= (1LL << 31) - 1) throw InvalidArg{"nnz must be in [0, 2^31-1)"};
  if (!A->row_ptr) throw InvalidArg{"null row_ptr"};
  if (A->nnz > 0 && (!A->col_idx || !A->values)) throw InvalidArg{"null col_idx or values"};
}

plss_matrix* matrix_create(plss_handle* h, const plss_csr* A, plss_dtype storage, hipStream_t s) {
  check_args(A);
  if (storage != PLSS_F64 && storage != PLSS_F32) throw InvalidArg{"unknown storage type"};
  const int m = (int)A->m, n = (int)A->n;
  const long long nnz = A->nnz;

  // row pointers: host copy, checked here
  std::vector<long long> rp(m + 1);
  PLSS_HIP(hipMemcpy(rp.data(), A->row_ptr, sizeof(long long) * (m + 1), hipMemcpyDefault));
  if (rp[0] != 0) throw InvalidArg{"row_ptr[0] must be 0"};
  for (int i = 0; i < m; ++i)
    if (rp[i + 1] < rp[i]) throw InvalidArg{"row_ptr must be non-decreasing"};
  if (rp[m] != nnz) throw InvalidArg{"row_ptr[m] must equal nnz"};

  plss_matrix* M = new plss_matrix();
  M->h = h;
  M->m = m;
  M->n = n;
  M->nnz = nnz;
  M->f32 = storage == PLSS_F32;
  const size_t vsz = M->f32 ? 4 : 8;
  long long* d_rp64 = nullptr;
  double* d_v64 = nullptr;
  int* dflag = nullptr;
  void* work = nullptr;
  try {
    PlssDir& a = M->A;
    PlssDir& t = M->T;
    a.nrows = m;
    a.ncols = n;
    t.nrows = n;
    t.ncols = m;
    a.h_ptr.resize(m + 1);
    for (int i = 0; i <= m; ++i) a.h_ptr[i] = (int)rp[i];
    a.ptr = static_cast<int*>(dmalloc(sizeof(int) * (m + 1)));
    a.idx = static_cast<int*>(dmalloc(sizeof(int) * std::max<long long>(nnz, 1)));
    a.val = dmalloc(vsz * std::max<long long>(nnz, 1));
    t.ptr = static_cast<int*>(dmalloc(sizeof(int) * (n + 1)));
    t.idx = static_cast<int*>(dmalloc(sizeof(int) * std::max<long long>(nnz, 1)));
    t.val = dmalloc(vsz * std::max<long long>(nnz, 1));
    PLSS_HIP(hipMemcpyAsync(a.ptr, a.h_ptr.data(), sizeof(int) * (m + 1), hipMemcpyHostToDevice, s));
    if (nnz > 0) {
      PLSS_HIP(hipMemcpyAsync(a.idx, A->col_idx, sizeof(int) * nnz, hipMemcpyDefault, s));
      // float64 source values on the device
      if (!M->f32) {
        d_v64 = static_cast<double*>(a.val);
      } else {
        d_v64 = static_cast<double*>(dmalloc(sizeof(double) * nnz));
      }
      PLSS_HIP(hipMemcpyAsync(d_v64, A->values, sizeof(double) * nnz, hipMemcpyDefault, s));
      d_rp64 = static_cast<long long*>(dmalloc(sizeof(long long) * (m + 1)));
      PLSS_HIP(hipMemcpyAsync(d_rp64, rp.data(), sizeof(long long) * (m + 1), hipMemcpyHostToDevice, s));
      dflag = static_cast<int*>(dmalloc(sizeof(int)));
      const int f = validate_csr_device(d_rp64, a.idx, d_v64, m, n, dflag, s);
      if (f & 1) throw InvalidArg{"column index out of range"};
      if (f & 2) throw InvalidArg{"column indices must be ascending and distinct within a row"};
      if (f & 4) throw InvalidArg{"non-finite value"};
      if (M->f32) convert_vals(d_v64, nnz, true, a.val, s);
    }
    work = dmalloc(csc_work_bytes(n, nnz));
    build_csc(a.ptr, a.idx, d_v64, m, n, nnz, M->f32, t.ptr, t.idx, t.val, work, s);
    t.h_ptr.resize(n + 1);
    PLSS_HIP(hipMemcpyAsync(t.h_ptr.data(), t.ptr, sizeof(int) * (n + 1), hipMemcpyDeviceToHost, s));
    PLSS_HIP(hipStreamSynchronize(s));
    set_tiles(a, 8, s);
    set_tiles(t, 8, s);
    set_long_rows(a, s);
    set_long_rows(t, s);
    if (small_fits(m, n, M->f32)) {
      set_slices(a, M->f32, s);
      set_slices(t, M->f32, s);
    }
    build_row_blocks(M, s);
  } catch (...) {
    if (d_v64 && d_v64 != M->A.val) dfree(d_v64);
    dfree(d_rp64);
    dfree(dflag);
    dfree(work);
    matrix_destroy(M);
    throw;
  }
  if (d_v64 != M->A.val) dfree(d_v64);
  dfree(d_rp64);
  dfree(dflag);
  dfree(work);
  recount_bytes(M);
  bool as = false, ts = false;
  auto_layout(m, n, nnz, M->f32, &as, &ts);
  if (as || ts) {
    try {
      matrix_set_layout(M, as, ts, 0, s);
    } catch (...) {
      matrix_destroy(M);
      throw;
    }
  }
  h->refs += 1;
  return M;
}

void matrix_destroy(plss_matrix* M) {
  if (!M) return;
  for (PlssDir* d : {&M->A, &M->T}) {
    dfree(d->ptr);
    dfree(d->idx);
    dfree(d->val);
    dfree(d->tile);
    dfree(d->grp);
    dfree(d->wtd);
    dfree(d->lrows);
    dfree(d->sl_base);
    dfree(d->sl_idx);
    dfree(d->sl_val);
  }
  for (int b = 0; b < kMaxBlk; ++b) {
    PlssDir& d = M->TB[b];
    dfree(d.idx);
    dfree(d.val);
    dfree(d.tile);
    dfree(d.grp);
    dfree(d.wtd);
    free_stripes(M->SB[b]);
    PlssDir& c = M->CB[b];
    dfree(c.idx);
    dfree(c.val);
    dfree(c.tile);
    dfree(c.grp);
    dfree(c.wtd);
  }
  free_stripes(M->SA);
  dfree(M->tb_ptr_all);
  dfree(M->cb_ptr_all);
  dfree(M->fz_pos);
  dfree(M->fz_c);
  delete M;
}

// Row blocks of the transposed store: when the gathered vector r (m
// entries) is larger than about 3 MB it does not stay in one XCD's 4 MB L2;
// splitting the rows into 8 blocks of equal nnz gives every XCD a slice of
// r that does.  Block b holds, column by column, the entries of its rows
// (a contiguous sub-segment of each CSC column).
void build_row_blocks(plss_matrix* M, hipStream_t s, bool force) {
  const size_t vb = M->f32 ? 4 : 8;
  const long long m = M->m, n = M->n, nnz = M->nnz;
  if (M->nblk > 1) return;
  if (!force && ((size_t)m * vb <= (3u << 20) || nnz < 8 * 64)) {
    M->nblk = 1;
    return;
  }
  const int nb = kMaxBlk;
  M->nblk = nb;
  // row boundaries balancing the entries
  const std::vector<int>& rp = M->A.h_ptr;
  M->rb[0] = 0;
  int i = 0;
  for (int b = 1; b < nb; ++b) {
    const long long target = nnz * b / nb;
    while (i < m && rp[i] < target) ++i;
    M->rb[b] = i;
  }
  M->rb[nb] = (int)m;
  int* d_rb = static_cast<int*>(dmalloc(sizeof(int) * (nb + 1)));
  int* d_cnt = static_cast<int*>(dmalloc(sizeof(int) * (size_t)nb * n));
  void* work = dmalloc(sizeof(long long) * ((size_t)(n + 1023) / 1024 + 64));
  try {
    M->tb_ptr_all = static_cast<int*>(dmalloc(sizeof(int) * (size_t)nb * (n + 1)));
    PLSS_HIP(hipMemcpyAsync(d_rb, M->rb, sizeof(int) * (nb + 1), hipMemcpyHostToDevice, s));
    blk_build(M->T.ptr, M->T.idx, (int)n, d_rb, nb, d_cnt, M->tb_ptr_all, work, s);
    std::vector<int> hp((size_t)nb * (n + 1));
    PLSS_HIP(hipMemcpyAsync(hp.data(), M->tb_ptr_all, sizeof(int) * hp.size(), hipMemcpyDeviceToHost, s));
    PLSS_HIP(hipStreamSynchronize(s));
    for (int b = 0; b < nb; ++b) {
      PlssDir& d = M->TB[b];
      d.nrows = (int)n;
      d.ncols = (int)m;
      d.h_ptr.assign(hp.begin() + (size_t)b * (n + 1), hp.begin() + (size_t)(b + 1) * (n + 1));
      const long long nz = d.h_ptr[n];
      d.ptr = M->tb_ptr_all + (size_t)b * (n + 1);
      d.idx = static_cast<int*>(dmalloc(sizeof(int) * std::max<long long>(nz, 1)));
      d.val = dmalloc(vb * std::max<long long>(nz, 1));
      blk_copy(M->T.ptr, M->T.idx, M->T.val, M->f32, (int)n, b, M->tb_ptr_all, d.idx, d.val, s);
      set_tiles(d, M->T.V, s);
    }
  } catch (...) {
    dfree(d_rb);
    dfree(d_cnt);
    dfree(work);
    throw;
  }
  dfree(d_rb);
  dfree(d_cnt);
  dfree(work);
}

// Column blocks of A: when the gathered vector of a product with A (n
// float64 entries) is larger than about 3 MB it does not stay in one XCD's
// 4 MB L2; splitting the columns into 8 blocks of equal nnz gives every XCD
// a slice that does.  Block b holds, row by row, the entries of its columns
// (a contiguous sub-segment of each CSR row: column indices ascend).
void build_fused(plss_matrix* M, hipStream_t s) {
  if (M->fz_pos) return;
  const size_t cnt = (size_t)std::max<long long>(M->nnz, 1);
  int* pos = static_cast<int*>(dmalloc(sizeof(int) * cnt));
  double* c = nullptr;
  try {
    c = static_cast<double*>(dmalloc(sizeof(double) * cnt));
    if (M->nnz > 0) launch_fz_pos(M->A.ptr, M->A.idx, M->T.ptr, M->T.idx, (int)M->n, pos, s);
    PLSS_HIP(hipStreamSynchronize(s));
  } catch (...) {
    dfree(pos);
    dfree(c);
    throw;
  }
  M->fz_pos = pos;
  M->fz_c = c;
  recount_bytes(M);
}

void build_col_blocks(plss_matrix* M, hipStream_t s) {
  const size_t vb = M->f32 ? 4 : 8;
  const long long m = M->m, n = M->n, nnz = M->nnz;
  if (M->cnblk > 1 || (size_t)n * 8 <= (3u << 20) || nnz < 8 * 64) return;
  const int nb = kMaxBlk;
  // column boundaries balancing the entries (the CSC pointers count them)
  const std::vector<int>& cp = M->T.h_ptr;
  int cbnd[kMaxBlk + 1];
  cbnd[0] = 0;
  int j = 0;
  for (int b = 1; b < nb; ++b) {
    const long long target = nnz * b / nb;
    while (j < n && cp[j] < target) ++j;
    cbnd[b] = j;
  }
  cbnd[nb] = (int)n;
  int* d_cb = static_cast<int*>(dmalloc(sizeof(int) * (nb + 1)));
  int* d_cnt = nullptr;
  void* work = nullptr;
  PlssDir CB[kMaxBlk];
  int* ptr_all = nullptr;
  try {
    d_cnt = static_cast<int*>(dmalloc(sizeof(int) * (size_t)nb * m));
    work = dmalloc(sizeof(long long) * ((size_t)(m + 1023) / 1024 + 64));
    ptr_all = static_cast<int*>(dmalloc(sizeof(int) * (size_t)nb * (m + 1)));
    PLSS_HIP(hipMemcpyAsync(d_cb, cbnd, sizeof(int) * (nb + 1), hipMemcpyHostToDevice, s));
    blk_build(M->A.ptr, M->A.idx, (int)m, d_cb, nb, d_cnt, ptr_all, work, s);
    std::vector<int> hp((size_t)nb * (m + 1));
    PLSS_HIP(hipMemcpyAsync(hp.data(), ptr_all, sizeof(int) * hp.size(), hipMemcpyDeviceToHost, s));
    PLSS_HIP(hipStreamSynchronize(s));
    for (int b = 0; b < nb; ++b) {
      PlssDir& d = CB[b];
      d.nrows = (int)m;
      d.ncols = (int)n;
      d.h_ptr.assign(hp.begin() + (size_t)b * (m + 1), hp.begin() + (size_t)(b + 1) * (m + 1));
      const long long nz = d.h_ptr[m];
      d.ptr = ptr_all + (size_t)b * (m + 1);
      d.idx = static_cast<int*>(dmalloc(sizeof(int) * std::max<long long>(nz, 1)));
      d.val = dmalloc(vb * std::max<long long>(nz, 1));
      blk_copy(M->A.ptr, M->A.idx, M->A.val, M->f32, (int)m, b, ptr_all, d.idx, d.val, s);
      set_tiles(d, M->A.V, s);
    }
    PLSS_HIP(hipStreamSynchronize(s));
  } catch (...) {
    for (auto& d : CB) {
      dfree(d.idx);
      dfree(d.val);
      dfree(d.tile);
      dfree(d.grp);
      dfree(d.wtd);
    }
    dfree(ptr_all);
    dfree(d_cb);
    dfree(d_cnt);
    dfree(work);
    throw;
  }
  dfree(d_cb);
  dfree(d_cnt);
  dfree(work);
  for (int b = 0; b < nb; ++b) M->CB[b] = std::move(CB[b]);
  std::memcpy(M->cbnd, cbnd, sizeof(cbnd));
  M->cb_ptr_all = ptr_all;
  M->cnblk = nb;
  recount_bytes(M);
}

void handle_release(plss_handle* h) {
  if (!h) return;
  const int left = --h->refs;
  if (h->closed && left <= 0) {
    (void)hipStreamSynchronize(h->stream);
    workspace_free(h->ws);
    (void)hipStreamDestroy(h->stream);
    delete h;
  }
}

}  // namespace plss
