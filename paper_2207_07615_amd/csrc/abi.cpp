// extern "C" entry points of plss.h.
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "fused.hpp"
#include "runtime.hpp"
#include "sketch.hpp"
#include "solve.hpp"
#include "multi.hpp"
#include "serve.hpp"

namespace plss {
static thread_local std::string g_err;
void set_error(const std::string& s) { g_err = s; }
}  // namespace plss

using namespace plss;

#define PLSS_GUARD_BEGIN try {
#define PLSS_GUARD_END                                                   \
  }                                                                      \
  catch (const InvalidArg& e) {                                          \
    set_error(e.msg);                                                    \
    return PLSS_EINVAL;                                                  \
  }                                                                      \
  catch (const OutOfMemory& e) {                                         \
    set_error(e.msg);                                                    \
    return PLSS_ENOMEM;                                                  \
  }                                                                      \
  catch (const DeviceError&) {                                           \
    return PLSS_EDEVICE;                                                 \
  }                                                                      \
  catch (const std::bad_alloc&) {                                        \
    set_error("host allocation failed");                                 \
    return PLSS_ENOMEM;                                                  \
  }

namespace {
struct DeviceScope {
  int prev = -1;
  explicit DeviceScope(int dev) {
    (void)hipGetDevice(&prev);
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceScope() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

plss_status worst(plss_status a, plss_status b) { return a != PLSS_OK ? a : b; }
}  // namespace

extern "C" {

void plss_opts_default(plss_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->sketch = PLSS_SKETCH_RESIDUAL;
  o->tol = 1e-8;
  o->maxit = 1000;
  o->refine = 1;
  o->inner_tol = 1e-4;
  o->max_outer = 20;
}

const char* plss_status_string(plss_status s) {
  switch (s) {
    case PLSS_OK: return "ok";
    case PLSS_NOT_CONVERGED: return "not converged";
    case PLSS_BREAKDOWN: return "breakdown";
    case PLSS_PENDING: return "pending";
    case PLSS_EINVAL: return "invalid argument";
    case PLSS_ENOMEM: return "out of memory";
    case PLSS_EDEVICE: return "device error";
    case PLSS_ECANCELLED: return "cancelled";
  }
  return "unknown status";
}

const char* plss_last_error(void) { return g_err.c_str(); }

plss_status plss_create(plss_handle** out, int device) {
  PLSS_GUARD_BEGIN
  if (!out) throw InvalidArg{"null output"};
  int count = 0;
  PLSS_HIP(hipGetDeviceCount(&count));
  if (device < 0 || device >= count) throw InvalidArg{"no such device"};
  DeviceScope ds(device);
  (void)scratch_ptr(device);  // this GPU's copy of the fixed scratch array (once per device)
  plss_handle* h = new plss_handle();
  h->device = device;
  hipError_t e = hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    delete h;
    set_error(hipGetErrorString(e));
    return PLSS_EDEVICE;
  }
  *out = h;
  return PLSS_OK;
  PLSS_GUARD_END
}

plss_status plss_destroy(plss_handle* h) {
  if (!h || h->closed) return PLSS_EINVAL;
  DeviceScope ds(h->device);
  h->closed = true;
  h->refs += 1;
  handle_release(h);  // frees now unless matrices or servers still use it
  return PLSS_OK;
}

plss_status plss_matrix_create(plss_handle* h, const plss_csr* A, plss_dtype storage,
                               plss_matrix** out) {
  PLSS_GUARD_BEGIN
  if (!h || !out) throw InvalidArg{"null handle or output"};
  if (h->closed) throw InvalidArg{"handle destroyed"};
  DeviceScope ds(h->device);
  std::lock_guard<std::mutex> lk(h->mu);
  *out = matrix_create(h, A, storage, h->stream);
  return PLSS_OK;
  PLSS_GUARD_END
}

plss_status plss_matrix_destroy(plss_matrix* A) {
  if (!A) return PLSS_EINVAL;
  plss_handle* h = A->h;
  DeviceScope ds(h->device);
  (void)hipStreamSynchronize(h->stream);
  matrix_destroy(A);
  handle_release(h);
  return PLSS_OK;
}

plss_status plss_matrix_info(const plss_matrix* A, int64_t* m, int64_t* n, int64_t* nnz,
                             int64_t* bytes) {
  if (!A) return PLSS_EINVAL;
  if (m) *m = A->m;
  if (n) *n = A->n;
  if (nnz) *nnz = A->nnz;
  if (bytes) *bytes = (int64_t)A->bytes;
  return PLSS_OK;
}

plss_status plss_matrix_csc(const plss_matrix* A, int64_t* col_ptr, int32_t* row_idx, double* values) {
  PLSS_GUARD_BEGIN
  if (!A) throw InvalidArg{"null matrix"};
  DeviceScope ds(A->h->device);
  hipStream_t s = A->h->stream;
  if (col_ptr) {
    std::vector<int64_t> cp(A->n + 1);
    for (long long j = 0; j <= A->n; ++j) cp[j] = A->T.h_ptr[j];
    PLSS_HIP(hipMemcpy(col_ptr, cp.data(), sizeof(int64_t) * cp.size(), hipMemcpyDefault));
  }
  if (row_idx && A->nnz)
    PLSS_HIP(hipMemcpyAsync(row_idx, A->T.idx, sizeof(int32_t) * A->nnz, hipMemcpyDefault, s));
  if (values && A->nnz) {
    if (!A->f32) {
      PLSS_HIP(hipMemcpyAsync(values, A->T.val, sizeof(double) * A->nnz, hipMemcpyDefault, s));
    } else {
      std::vector<float> f(A->nnz);
      PLSS_HIP(hipMemcpyAsync(f.data(), A->T.val, sizeof(float) * A->nnz, hipMemcpyDeviceToHost, s));
      PLSS_HIP(hipStreamSynchronize(s));
      std::vector<double> d(f.begin(), f.end());
      PLSS_HIP(hipMemcpy(values, d.data(), sizeof(double) * A->nnz, hipMemcpyDefault));
    }
  }
  PLSS_HIP(hipStreamSynchronize(s));
  return PLSS_OK;
  PLSS_GUARD_END
}

plss_status plss_matrix_autotune(plss_handle* h, plss_matrix* A, int32_t* wa, int32_t* wt) {
  PLSS_GUARD_BEGIN
  if (!h || !A) throw InvalidArg{"null handle or matrix"};
  DeviceScope ds(h->device);
  std::lock_guard<std::mutex> lk(h->mu);
  autotune_matrix(h, A, h->stream);
  if (wa) *wa = A->A.V;
  if (wt) *wt = A->T.V;
  return PLSS_OK;
  PLSS_GUARD_END
}

plss_status plss_matrix_layout(plss_handle* h, plss_matrix* A, const plss_layout* want, plss_layout* got) {
  PLSS_GUARD_BEGIN
  if (!h || !A) throw InvalidArg{"null handle or matrix"};
  DeviceScope ds(h->device);
  std::lock_guard<std::mutex> lk(h->mu);
  auto report = [&]() {
    if (got) {
      got->a_stripes = A->a_striped ? 1 : 0;
      got->t_stripes = A->t_striped ? 1 : 0;
      got->unit_rows = A->a_striped ? A->SA.unit_rows : (A->t_striped ? A->SB[0].unit_rows : 0);
    }
  };
  if (want) {
    try {
      matrix_set_layout(A, want->a_stripes != 0, want->t_stripes != 0, want->unit_rows, h->stream);
    } catch (...) {
      report();
      throw;
    }
  }
  report();
  return PLSS_OK;
  PLSS_GUARD_END
}

plss_status plss_spmv(plss_handle* h, const plss_matrix* A, int transpose, const double* x, double* y) {
  PLSS_GUARD_BEGIN
  if (!h || !A || !x || !y) throw InvalidArg{"null argument"};
  DeviceScope ds(h->device);
  std::lock_guard<std::mutex> lk(h->mu);
  spmv_plain(A, transpose != 0, x, y, h->stream);
  return PLSS_OK;
  PLSS_GUARD_END
}

plss_status plss_spmv_noalloc(plss_handle* h, const plss_matrix* A, int transpose, const double* x,
                              double* y) {
  PLSS_GUARD_BEGIN
  if (!h || !A || !x || !y) throw InvalidArg{"null argument"};
  DeviceScope ds(h->device);
  std::lock_guard<std::mutex> lk(h->mu);
  spmv_noalloc(h, A, transpose != 0, x, y, h->stream);
  return PLSS_OK;
  PLSS_GUARD_END
}

plss_status plss_release_workspace(plss_handle* h) {
  PLSS_GUARD_BEGIN
  if (!h) throw InvalidArg{"null handle"};
  DeviceScope ds(h->device);
  std::lock_guard<std::mutex> lk(h->mu);
  PLSS_HIP(hipStreamSynchronize(h->stream));
  if (h->ws) {
    workspace_free(h->ws);  // also waits for the second stream
    h->ws = nullptr;
  }
  return PLSS_OK;
  PLSS_GUARD_END
}

plss_status plss_residual_pair(plss_handle* h, plss_matrix* A, const double* p, double* r, double* y,
                               double* rho_phi) {
  PLSS_GUARD_BEGIN
  if (!h || !A || !p || !r || !y) throw InvalidArg{"null argument"};
  DeviceScope ds(h->device);
  std::lock_guard<std::mutex> lk(h->mu);
  residual_pair(h, A, p, r, y, rho_phi, h->stream);
  return PLSS_OK;
  PLSS_GUARD_END
}

plss_status plss_solve(plss_handle* h, const plss_matrix* A, const double* b, const plss_opts* o,
                       double* x, double* hist, int64_t hist_cap, plss_info* info) {
  PLSS_GUARD_BEGIN
  if (!h || !A || !b || !o || !x) throw InvalidArg{"null argument"};
  validate_opts(o, A->f32);
  DeviceScope ds(h->device);
  std::lock_guard<std::mutex> lk(h->mu);
  plss_info inf{};
  if (o->sketch == PLSS_SKETCH_BLOCK_IDENTITY || o->sketch == PLSS_SKETCH_BLOCK_MIXED) {
    block_solve(h, A, b, o, x, hist, hist_cap, &inf, h->stream);
  } else if (o->sketch == PLSS_SKETCH_RANDPROJ) {
    randproj_solve(h, A, b, o, x, hist, hist_cap, &inf, h->stream);
  } else if (o->sketch != PLSS_SKETCH_RESIDUAL) {
    sketch_solve(h, A, b, o, x, hist, hist_cap, &inf, h->stream);
  } else {
    check_finite_inputs(A, b, o, h->stream);
    BatchRunner br(h);
    br.add(A, b, o, std::min<long long>(o->maxit + 64, 1LL << 22));
    br.prepare(h->stream);
    br.run(h->stream, o->timing != 0, o->chunk);
    br.result(0, x, hist, hist_cap, &inf, h->stream);
  }
  if (info) *info = inf;
  return (plss_status)inf.status;
  PLSS_GUARD_END
}

plss_status plss_solve_batch(plss_handle* h, int32_t nsys, const plss_matrix* const* A,
                             const double* const* b, const plss_opts* o, double* const* x,
                             plss_info* info) {
  PLSS_GUARD_BEGIN
  if (!h || nsys <= 0 || !A || !b || !o || !x) throw InvalidArg{"null argument or empty batch"};
  DeviceScope ds(h->device);
  std::lock_guard<std::mutex> lk(h->mu);
  BatchRunner br(h);
  for (int i = 0; i < nsys; ++i) {
    if (!A[i] || !b[i] || !x[i]) throw InvalidArg{"null system in batch"};
    if (A[i]->h != h) throw InvalidArg{"matrix belongs to another handle"};
    check_finite_inputs(A[i], b[i], &o[i], h->stream);
    br.add(A[i], b[i], &o[i], 1);
  }
  br.prepare(h->stream);
  bool timing = false;
  int chunk = 0;
  for (int i = 0; i < nsys; ++i) {
    timing |= o[i].timing != 0;
    chunk = std::max<int>(chunk, o[i].chunk);
  }
  br.run(h->stream, timing, chunk);
  plss_status agg = PLSS_OK;
  for (int i = 0; i < nsys; ++i) {
    plss_info inf{};
    br.result(i, x[i], nullptr, 0, &inf, h->stream);
    if (info) info[i] = inf;
    agg = worst(agg, (plss_status)inf.status);
  }
  return agg;
  PLSS_GUARD_END
}

plss_status plss_solve_multi(plss_handle* h, const plss_matrix* A, int32_t nrhs, const double* B,
                             const plss_opts* o, double* X, plss_info* info) {
  PLSS_GUARD_BEGIN
  if (!h || !A || !B || !o || !X || nrhs <= 0) throw InvalidArg{"null argument"};
  validate_opts(o, A->f32);
  if (o->sketch != PLSS_SKETCH_RESIDUAL) throw InvalidArg{"multi-RHS solves use the residual sketch"};
  DeviceScope ds(h->device);
  std::lock_guard<std::mutex> lk(h->mu);
  return multi_solve(h, A, nrhs, B, o, X, info, h->stream);
  PLSS_GUARD_END
}

plss_status plss_kernel_times(plss_handle* h, double* ms4, int64_t* n4) {
  if (!h) return PLSS_EINVAL;
  for (int q = 0; q < 4; ++q) {
    if (ms4) ms4[q] = h->kt_ms[q];
    if (n4) n4[q] = h->kt_n[q];
    h->kt_ms[q] = 0;
    h->kt_n[q] = 0;
  }
  return PLSS_OK;
}

plss_status plss_server_create(plss_handle* h, size_t budget, int32_t max_slots, plss_server** out) {
  PLSS_GUARD_BEGIN
  if (!h || !out || max_slots <= 0 || budget == 0) throw InvalidArg{"bad server arguments"};
  *out = server_create(h, budget, max_slots);
  return PLSS_OK;
  PLSS_GUARD_END
}

plss_status plss_server_submit(plss_server* s, const plss_csr* A, plss_dtype storage, const double* b,
                               const plss_opts* o, uint64_t* req) {
  PLSS_GUARD_BEGIN
  if (!s || !A || !b || !o || !req) throw InvalidArg{"null argument"};
  return server_submit(s, A, storage, b, o, req);
  PLSS_GUARD_END
}

plss_status plss_server_poll(plss_server* s, uint64_t req, double* x, plss_info* info) {
  PLSS_GUARD_BEGIN
  if (!s) throw InvalidArg{"null server"};
  return server_poll(s, req, x, info);
  PLSS_GUARD_END
}

plss_status plss_server_drain(plss_server* s) {
  PLSS_GUARD_BEGIN
  if (!s) throw InvalidArg{"null server"};
  return server_drain(s);
  PLSS_GUARD_END
}

plss_status plss_server_cancel(plss_server* s, uint64_t req) {
  PLSS_GUARD_BEGIN
  if (!s) throw InvalidArg{"null server"};
  return server_cancel(s, req);
  PLSS_GUARD_END
}

plss_status plss_server_stats(plss_server* s, int64_t* submitted, int64_t* finished, int64_t* active,
                              int64_t* peak) {
  PLSS_GUARD_BEGIN
  if (!s) throw InvalidArg{"null server"};
  return server_stats(s, submitted, finished, active, peak);
  PLSS_GUARD_END
}

plss_status plss_server_destroy(plss_server* s) {
  PLSS_GUARD_BEGIN
  if (!s) throw InvalidArg{"null server"};
  server_destroy(s);
  return PLSS_OK;
  PLSS_GUARD_END
}

}  // extern "C"
