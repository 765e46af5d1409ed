// Plain products with A / Aᵀ, input checks and the tile-width autotuner.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "runtime.hpp"
#include "solve.hpp"

namespace plss {

namespace {
// Device scratch freed on scope exit.
struct Scratch {
  std::vector<void*> p;
  void* get(size_t bytes) {
    p.push_back(dmalloc(bytes));
    return p.back();
  }
  ~Scratch() {
    for (void* q : p) dfree(q);
  }
};

void plain_launch(const plss_matrix* A, bool transpose, const double* dx, double* dy, Desc* d_desc,
                  int2* d_list, hipStream_t s) {
  const PlssDir& dir = transpose ? A->T : A->A;
  Desc d{};
  d.a_ptr = A->A.ptr;
  d.a_idx = A->A.idx;
  d.a_val = A->A.val;
  d.a_tile = A->A.tile;
  d.a_ntiles = A->A.ntiles;
  d.a_nwt = A->A.nwt;
  d.a_grp = A->A.grp;
  d.a_wtd = A->A.wtd;
  d.t_ptr = A->T.ptr;
  d.t_idx = A->T.idx;
  d.t_val = A->T.val;
  d.t_tile = A->T.tile;
  d.t_ntiles = A->T.ntiles;
  d.t_nwt = A->T.nwt;
  d.t_grp = A->T.grp;
  d.t_wtd = A->T.wtd;
  d.m = (int)A->m;
  d.n = (int)A->n;
  d.p = const_cast<double*>(dx);
  d.r64 = dy;
  std::vector<int2> l(dir.ntiles);
  for (int t = 0; t < dir.ntiles; ++t) l[t] = make_int2(0, t);
  PLSS_HIP(hipMemcpyAsync(d_desc, &d, sizeof(Desc), hipMemcpyHostToDevice, s));
  PLSS_HIP(hipMemcpyAsync(d_list, l.data(), sizeof(int2) * l.size(), hipMemcpyHostToDevice, s));
  launch_spmv(MODE_PLAIN, A->f32, dir.V, d_desc, d_list, dir.ntiles, transpose ? 1 : 0, s);
  PLSS_HIP(hipStreamSynchronize(s));  // the host vector l goes out of scope
}
}  // namespace

// Plain product through a striped store: A x from the store of A, or Aᵀ x
// as the fixed-order sum of the row blocks' products.
static void stripe_plain(const plss_matrix* A, bool transpose, const double* dx, double* dy, Scratch& sc,
                         hipStream_t s) {
  Desc d{};
  d.m = (int)A->m;
  d.n = (int)A->n;
  d.p = const_cast<double*>(dx);
  d.r64 = dy;
  std::vector<int2> l;
  double* yp = nullptr;
  if (!transpose) {
    fill_stripe_view(A->SA, &d.sa);
    for (int u = 0; u < A->SA.nunits; ++u) l.push_back(make_int2(0, u));
  } else {
    int qmax = 0;
    for (int b = 0; b < A->nblk; ++b) {
      fill_stripe_view(A->SB[b], &d.sb[b]);
      qmax = std::max(qmax, A->SB[b].nunits);
    }
    yp = static_cast<double*>(sc.get(8 * (size_t)A->nblk * A->n));
    d.ypart = yp;
    for (int q = 0; q < qmax; ++q)
      for (int b = 0; b < kMaxBlk; ++b)
        l.push_back(make_int2(0, (b < A->nblk && q < A->SB[b].nunits) ? ((b << 24) | q) : -1));
  }
  Desc* dd = static_cast<Desc*>(sc.get(sizeof(Desc)));
  int2* dl = static_cast<int2*>(sc.get(sizeof(int2) * std::max<size_t>(1, l.size())));
  PLSS_HIP(hipMemcpyAsync(dd, &d, sizeof(Desc), hipMemcpyHostToDevice, s));
  PLSS_HIP(hipMemcpyAsync(dl, l.data(), sizeof(int2) * l.size(), hipMemcpyHostToDevice, s));
  launch_sspmv(MODE_PLAIN, A->f32, dd, dl, (int)l.size(), transpose ? 1 : 0, s);
  if (transpose) st_ysum(yp, A->nblk, (int)A->n, dy, s);
  PLSS_HIP(hipStreamSynchronize(s));  // the host list goes out of scope
}

void spmv_plain(const plss_matrix* A, bool transpose, const double* x, double* y, hipStream_t s) {
  Scratch sc;
  const size_t nin = transpose ? A->m : A->n, nout = transpose ? A->n : A->m;
  double* dx = static_cast<double*>(sc.get(8 * nin));
  double* dy = static_cast<double*>(sc.get(8 * nout));
  // float32 stores of Aᵀ have stripes too wide for the float64-accumulating
  // plain product: it runs on the CSC tiles
  if (transpose ? (A->t_striped && !A->f32) : A->a_striped) {
    PLSS_HIP(hipMemcpyAsync(dx, x, 8 * nin, hipMemcpyDefault, s));
    stripe_plain(A, transpose, dx, dy, sc, s);
    PLSS_HIP(hipMemcpyAsync(y, dy, 8 * nout, hipMemcpyDefault, s));
    PLSS_HIP(hipStreamSynchronize(s));
    return;
  }
  Desc* dd = static_cast<Desc*>(sc.get(sizeof(Desc)));
  const PlssDir& dir = transpose ? A->T : A->A;
  int2* dl = static_cast<int2*>(sc.get(sizeof(int2) * std::max(1, dir.ntiles)));
  PLSS_HIP(hipMemcpyAsync(dx, x, 8 * nin, hipMemcpyDefault, s));
  plain_launch(A, transpose, dx, dy, dd, dl, s);
  PLSS_HIP(hipMemcpyAsync(y, dy, 8 * nout, hipMemcpyDefault, s));
  PLSS_HIP(hipStreamSynchronize(s));
}

// Arrays the host can read directly (plain or pinned host memory).
static bool host_readable(const void* p) {
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return true;  // not known to HIP: ordinary host memory
  }
  return a.type == hipMemoryTypeUnregistered || a.type == hipMemoryTypeHost;
}

// b, x0 finite; wi_diag finite and positive.  Host arrays are checked on the
// host (no device round trip for small solves), device arrays on the device.
void check_finite_inputs(const plss_matrix* A, const double* b, const plss_opts* o, hipStream_t s) {
  struct C {
    const double* p;
    size_t n;
    int pos;
    const char* msg;
  } cs[3] = {{b, (size_t)A->m, 0, "b has a non-finite entry"},
             {o->x0, (size_t)A->n, 0, "x0 has a non-finite entry"},
             {o->wi_diag, (size_t)A->n, 1, "wi_diag must be finite and positive"}};
  for (auto& c : cs) {
    if (!c.p) continue;
    if (host_readable(c.p)) {
      for (size_t i = 0; i < c.n; ++i) {
        const double v = c.p[i];
        if (!std::isfinite(v) || (c.pos && !(v > 0.0))) throw InvalidArg{c.msg};
      }
      continue;
    }
    Scratch sc;
    double* tmp = static_cast<double*>(sc.get(8 * c.n));
    int* flag = static_cast<int*>(sc.get(sizeof(int)));
    PLSS_HIP(hipMemsetAsync(flag, 0, sizeof(int), s));
    PLSS_HIP(hipMemcpyAsync(tmp, c.p, 8 * c.n, hipMemcpyDefault, s));
    launch_check(tmp, (long long)c.n, c.pos, flag, s);
    int hf = 0;
    PLSS_HIP(hipMemcpyAsync(&hf, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    PLSS_HIP(hipStreamSynchronize(s));
    if (hf) throw InvalidArg{c.msg};
  }
}

// Time the plain product for each tile width and keep the fastest.
void autotune_matrix(plss_handle* h, plss_matrix* A, hipStream_t s) {
  (void)h;
  Scratch sc;
  const size_t nmax = std::max(A->m, A->n);
  double* dx = static_cast<double*>(sc.get(8 * nmax));
  double* dy = static_cast<double*>(sc.get(8 * nmax));
  Desc* dd = static_cast<Desc*>(sc.get(sizeof(Desc)));
  std::vector<double> ones(nmax, 1.0);
  PLSS_HIP(hipMemcpyAsync(dx, ones.data(), 8 * nmax, hipMemcpyHostToDevice, s));
  hipEvent_t e0, e1;
  PLSS_HIP(hipEventCreate(&e0));
  PLSS_HIP(hipEventCreate(&e1));
  for (int tr = 0; tr < 2; ++tr) {
    PlssDir& dir = tr ? A->T : A->A;
    int best_v = dir.V;
    float best = 1e30f;
    for (int V : {4, 8, 16}) {
      set_tiles(dir, V, s);
      int2* dl = static_cast<int2*>(sc.get(sizeof(int2) * std::max(1, dir.ntiles)));
      plain_launch(A, tr != 0, dx, dy, dd, dl, s);  // warm-up
      const int reps = 5;
      std::vector<int2> l(dir.ntiles);
      for (int t = 0; t < dir.ntiles; ++t) l[t] = make_int2(0, t);
      PLSS_HIP(hipEventRecord(e0, s));
      for (int q = 0; q < reps; ++q)
        launch_spmv(MODE_PLAIN, A->f32, V, dd, dl, dir.ntiles, tr, s);
      PLSS_HIP(hipEventRecord(e1, s));
      PLSS_HIP(hipEventSynchronize(e1));
      float ms = 0;
      PLSS_HIP(hipEventElapsedTime(&ms, e0, e1));
      if (ms < best) {
        best = ms;
        best_v = V;
      }
    }
    set_tiles(dir, best_v, s);
  }
  for (int b = 0; b < A->nblk && A->nblk > 1; ++b) set_tiles(A->TB[b], A->T.V, s);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
}

}  // namespace plss
