// Matrix store: upload, validation, CSC build, tile tables.
#include "runtime.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace plss {

void* dmalloc(size_t bytes) {
  void* p = nullptr;
  if (bytes == 0) bytes = 8;
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
  dfree(d.tile);
  dfree(d.grp);
  d.tile = nullptr;
  d.grp = nullptr;
  d.tile = static_cast<int*>(dmalloc(sizeof(int) * t.size()));
  d.grp = static_cast<int*>(dmalloc(sizeof(int) * g.size()));
  PLSS_HIP(hipMemcpyAsync(d.tile, t.data(), sizeof(int) * t.size(), hipMemcpyHostToDevice, s));
  PLSS_HIP(hipMemcpyAsync(d.grp, g.data(), sizeof(int) * g.size(), hipMemcpyHostToDevice, s));
  PLSS_HIP(hipStreamSynchronize(s));
  d.nwt = (int)t.size() - 1;
  d.ntiles = (int)g.size() / kWaves;
  d.V = V;
}

size_t matrix_footprint(long long m, long long n, long long nnz, bool f32) {
  const size_t v = f32 ? 4 : 8;
  return (size_t)nnz * (v + 4) * 2 + (size_t)(m + n + 2) * 4 + (size_t)(m + n) / 64 * 4 + 4096;
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
  h->refs += 1;
  M->bytes = (size_t)nnz * (vsz + 4) * (M->nblk > 1 ? 3 : 2) + sizeof(int) * (size_t)(m + n + 2) +
             sizeof(int) * (size_t)(M->A.ntiles + M->T.ntiles + 2) +
             (M->nblk > 1 ? sizeof(int) * (size_t)M->nblk * (n + 1) : 0);
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
  }
  for (int b = 0; b < kMaxBlk; ++b) {
    PlssDir& d = M->TB[b];
    dfree(d.idx);
    dfree(d.val);
    dfree(d.tile);
    dfree(d.grp);
  }
  dfree(M->tb_ptr_all);
  delete M;
}

// Row blocks of the transposed store: when the gathered vector r (m
// entries) is larger than about 3 MB it does not stay in one XCD's 4 MB L2;
// splitting the rows into 8 blocks of equal nnz gives every XCD a slice of
// r that does.  Block b holds, column by column, the entries of its rows
// (a contiguous sub-segment of each CSC column).
void build_row_blocks(plss_matrix* M, hipStream_t s) {
  const size_t vb = M->f32 ? 4 : 8;
  const long long m = M->m, n = M->n, nnz = M->nnz;
  if ((size_t)m * vb <= (3u << 20) || nnz < 8 * 64) {
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

void handle_release(plss_handle* h) {
  if (!h) return;
  const int left = --h->refs;
  if (h->closed && left <= 0) {
    (void)hipStreamSynchronize(h->stream);
    (void)hipStreamDestroy(h->stream);
    delete h;
  }
}

}  // namespace plss
