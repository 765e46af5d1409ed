// Driver of the randomized projection (fresh Gaussian sketch per iteration).
#include "randproj.hpp"

#include <algorithm>
#include <cstring>
#include <vector>

#include "kernels.hpp"
#include "sketch.hpp"
#include "solve.hpp"

namespace plss {

namespace {
size_t up(size_t v) { return (v + 255) / 256 * 256; }
}  // namespace

void randproj_solve(plss_handle* h, const plss_matrix* A, const double* b, const plss_opts* o, double* x,
                    double* hist, long long hist_cap_out, plss_info* info, hipStream_t s) {
  if (A->f32) throw InvalidArg{"the randomized projection needs float64 storage"};
  if (o->wi_diag) throw InvalidArg{"wi_diag applies to the residual sketch only"};
  if (o->x0) throw InvalidArg{"the randomized projection starts from x0 = 0"};
  const int r = o->block;
  if (r < 1 || r > 16) throw InvalidArg{"block (sketch columns) must be in 1..16 for the randomized projection"};
  check_finite_inputs(A, b, o, s);
  const int m = (int)A->m, n = (int)A->n;
  const int rp = (r + 3) & ~3;
  const int ngram = std::max(1, std::min(512, (n + 255) / 256));
  const int nsig = (m + kRpRows - 1) / kRpRows;

  // the products with A use the striped store when the matrix has one (the
  // partials of rho then come per unit); the system's arena, state,
  // descriptor, list and pinned state mirror come from the handle's
  // workspace (calls on a handle are serialised and synchronise before
  // returning)
  const bool as = A->a_striped;
  const int na = as ? A->SA.nunits : A->A.ntiles;
  Workspace& ws = workspace(h);
  const long long hist_len = std::min<long long>(o->maxit + 2, 1LL << 22);
  const Workspace::Call cm = ws.call_block(SysRun::arena_bytes(A, o, hist_len, true), sizeof(int2) * na + sizeof(int));
  State* d_state = cm.d_state;
  Desc* d_desc = cm.d_desc;
  State* h_state = cm.h_state;
  SysRun run;
  try {
    run.use_stripes = true;
    run.setup(A, b, o, hist_len, d_state, cm.arena);
    run.upload(b, nullptr, nullptr, s);
    size_t off = 0;
    const size_t oS = off; off = up(off + 8 * (size_t)m * rp);
    const size_t oY = off; off = up(off + 8 * (size_t)n * rp);
    const size_t oG = off; off = up(off + 8 * (size_t)ngram * 256);
    const size_t oSg = off; off = up(off + 8 * (size_t)nsig * 16);
    const size_t oC = off; off = up(off + 8 * 16);
    const size_t oRd = off; off = up(off + sizeof(RpDesc));
    char* mem = workspace(h).hist_block(off);
    RpDesc rd{};
    rd.S = reinterpret_cast<double*>(mem + oS);
    rd.Y = reinterpret_cast<double*>(mem + oY);
    rd.part_g = reinterpret_cast<double*>(mem + oG);
    rd.part_s = reinterpret_cast<double*>(mem + oSg);
    rd.c = reinterpret_cast<double*>(mem + oC);
    rd.r = r;
    rd.rp = rp;
    rd.ngram = ngram;
    rd.nsig = nsig;
    rd.k0 = (unsigned)(o->seed & 0xFFFFFFFFull);
    rd.k1 = (unsigned)(o->seed >> 32);
    RpDesc* d_rd = reinterpret_cast<RpDesc*>(mem + oRd);
    PLSS_HIP(hipMemcpyAsync(d_rd, &rd, sizeof(RpDesc), hipMemcpyHostToDevice, s));
    Desc d = run.desc;
    State st = run.st0;
    PLSS_HIP(hipMemcpyAsync(d_desc, &d, sizeof(Desc), hipMemcpyHostToDevice, s));
    PLSS_HIP(hipMemcpyAsync(d_state, &st, sizeof(State), hipMemcpyHostToDevice, s));
    // the A list: units of the striped store, or the CSR tile groups
    std::vector<int2> all;
    for (int t = 0; t < na; ++t) all.push_back(make_int2(0, t));
    char* d_lists = cm.lists;
    int2* dla = reinterpret_cast<int2*>(d_lists);
    int* dsys = reinterpret_cast<int*>(dla + na);
    PLSS_HIP(hipMemcpyAsync(d_lists, all.data(), sizeof(int2) * all.size(), hipMemcpyHostToDevice, s));
    PLSS_HIP(hipMemsetAsync(dsys, 0, sizeof(int), s));

    auto outer_seq = [&]() {
      if (as) launch_sspmv(MODE_REFINE, false, d_desc, dla, na, 0, s);
      else launch_spmv(MODE_REFINE, false, A->A.V, d_desc, dla, na, 0, s);
      launch_outer(d_desc, dsys, 1, s);
      launch_start(false, d_desc, dla, na, s);
    };
    hipEvent_t e0 = ws.t0, e1 = ws.t1;
    {
      PLSS_HIP(hipEventRecord(e0, s));
      outer_seq();
      launch_col_init(d_desc, dsys, 1, s);
      int chunk = o->chunk > 0 ? o->chunk : 16;
      while (true) {
        for (int c = 0; c < chunk; ++c)
          launch_rp_step(d_desc, d_rd, rp, m, n, A->A.V, dla, na, as, ngram, nsig, s);
        PLSS_HIP(hipMemcpyAsync(h_state, d_state, sizeof(State), hipMemcpyDeviceToHost, s));
        PLSS_HIP(hipStreamSynchronize(s));
        if (h_state->done || h_state->final_done) break;
        if (o->chunk <= 0) chunk = std::min(chunk * 2, 128);
      }
      outer_seq();  // true residual of the final x
      PLSS_HIP(hipMemcpyAsync(h_state, d_state, sizeof(State), hipMemcpyDeviceToHost, s));
      PLSS_HIP(hipEventRecord(e1, s));
      PLSS_HIP(hipEventSynchronize(e1));
    }
    float ms = 0;
    PLSS_HIP(hipEventElapsedTime(&ms, e0, e1));
    const State& fs = *h_state;
    PLSS_HIP(hipMemcpyAsync(x, run.desc.xo, 8 * (size_t)n, hipMemcpyDefault, s));
    const long long nh = std::min<long long>({hist_cap_out, fs.k_total + 1, run.hist_len});
    if (hist && nh > 0) PLSS_HIP(hipMemcpyAsync(hist, run.desc.hist, 8 * nh, hipMemcpyDefault, s));
    PLSS_HIP(hipStreamSynchronize(s));
    info->iters = fs.k_total;
    info->outer_iters = 1;
    info->relres = sqrt(fs.rho) * fs.scale;
    info->relres_true = fs.relres_true;
    info->status = fs.final_done ? fs.final_status : fs.status;
    info->ms = ms;
  } catch (...) {
    (void)hipStreamSynchronize(s);
    throw;
  }
}

}  // namespace plss
