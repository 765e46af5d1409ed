// The fused residual pair on a handle: r <- r - A p and y = Aᵀ r with the
// updated r, in one pass over the CSR store (fused.hip), with the caller's
// vectors in host or device memory.
#include "fused.hpp"

#include "runtime.hpp"
#include "solve.hpp"

namespace plss {

namespace {
bool on_device(const void* p) {
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;  // not known to HIP: ordinary host memory
  }
  return a.type == hipMemoryTypeDevice;
}

size_t up(size_t v) { return (v + 255) / 256 * 256; }
}  // namespace

void residual_pair(plss_handle* h, plss_matrix* A, const double* p, double* r, double* y, double* out2,
                   hipStream_t s) {
  build_fused(A, s);
  const long long m = A->m, n = A->n;
  // device vectors are used in place; otherwise all three pass through the
  // handle's workspace
  const bool dev = on_device(p) && on_device(r) && on_device(y);
  const int g1 = fz_grid(m), gl = fz_long_grid(A->A.nlong), g2 = fz_grid(n);
  size_t off = 0;
  auto take = [&](size_t b) {
    const size_t o = off;
    off = up(off + b);
    return o;
  };
  const size_t o_part = take(sizeof(double) * (size_t)(g1 + gl + g2)), o_out = take(2 * sizeof(double));
  const size_t o_p = dev ? 0 : take(sizeof(double) * n), o_r = dev ? 0 : take(sizeof(double) * m);
  const size_t o_y = dev ? 0 : take(sizeof(double) * n);
  Workspace& ws = workspace(h);
  char* ar = ws.dev_block(off);
  double* hout = reinterpret_cast<double*>(ws.pin_block(2 * sizeof(double)));
  double* dp = dev ? const_cast<double*>(p) : reinterpret_cast<double*>(ar + o_p);
  double* dr = dev ? r : reinterpret_cast<double*>(ar + o_r);
  double* dy = dev ? y : reinterpret_cast<double*>(ar + o_y);
  if (!dev) {
    PLSS_HIP(hipMemcpyAsync(dp, p, sizeof(double) * n, hipMemcpyDefault, s));
    PLSS_HIP(hipMemcpyAsync(dr, r, sizeof(double) * m, hipMemcpyDefault, s));
  }
  double* part = reinterpret_cast<double*>(ar + o_part);
  double* dout = reinterpret_cast<double*>(ar + o_out);
  launch_fz_pair(A->f32, A->A.ptr, A->A.idx, A->A.val, (int)m, A->A.lrows, A->A.nlong, A->T.ptr, A->fz_pos,
                 (int)n, dp, dr, A->fz_c, dy, part, dout, s);
  PLSS_HIP(hipMemcpyAsync(hout, dout, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
  if (!dev) {
    PLSS_HIP(hipMemcpyAsync(r, dr, sizeof(double) * m, hipMemcpyDefault, s));
    PLSS_HIP(hipMemcpyAsync(y, dy, sizeof(double) * n, hipMemcpyDefault, s));
  }
  PLSS_HIP(hipStreamSynchronize(s));
  if (out2) {
    out2[0] = hout[0];
    out2[1] = hout[1];
  }
}

}  // namespace plss
