// Driver of the many-right-hand-side path: columns advance in lock-step;
// each column has its own stop test, and the refinement (float32 storage)
// outer step runs when every unfinished column has finished its inner solve.
#include "multi.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "multi_kernels.hpp"
#include "solve.hpp"

namespace plss {

namespace {
size_t up(size_t v) { return (v + 255) / 256 * 256; }

plss_status run_group(plss_handle* h, const plss_matrix* A, int ncols, const double* Bcm, const plss_opts* o,
                      double* Xcm, plss_info* info, hipStream_t s) {
  const bool f32 = A->f32;
  const int m = (int)A->m, n = (int)A->n;
  int W = 8;
  while (W < ncols) W *= 2;
  const size_t vs = f32 ? 4 : 8;
  const int na_blk = (m + kRB - 1) / kRB, nt_blk = (n + kRB - 1) / kRB;
  const int nu_blk = (int)(((long long)n * W + kUE - 1) / kUE);
  size_t off = 0;
  auto take = [&](size_t b) {
    size_t r = off;
    off = up(off + b);
    return r;
  };
  const size_t oB = take(8ull * m * W), oR64 = take(8ull * m * W), oR = take(vs * m * W);
  const size_t oP = take(vs * n * W), oY = take(vs * n * W), oX = take(8ull * n * W);
  const size_t oXi = f32 ? take(8ull * n * W) : 0;
  const size_t oPr = take(8ull * na_blk * W), oPb = take(8ull * na_blk * W);
  const size_t oPp = take(8ull * nt_blk * W), oPt = take(8ull * nu_blk * W);
  // the right-hand sides in, then the solution out (n x ncols)
  const size_t oBin = take(8ull * std::max(m, n) * ncols);
  const size_t oSt = take(sizeof(MState)), oD = take(sizeof(MDesc));
  // device and pinned memory from the handle's workspace (calls on a handle
  // are serialised and synchronise before returning)
  Workspace& ws = workspace(h);
  char* ar = ws.dev_block(off);
  MState* hst = reinterpret_cast<MState*>(ws.pin_block(sizeof(MState)));
  plss_status agg = PLSS_OK;
  try {
    MDesc d{};
    d.a_ptr = A->A.ptr;
    d.a_idx = A->A.idx;
    d.a_val = A->A.val;
    d.t_ptr = A->T.ptr;
    d.t_idx = A->T.idx;
    d.t_val = A->T.val;
    d.m = m;
    d.n = n;
    d.s = W;
    d.W = W;
    d.na_blk = na_blk;
    d.nt_blk = nt_blk;
    d.nu_blk = nu_blk;
    d.is_f32 = f32;
    d.R = ar + oR;
    d.P = ar + oP;
    d.Y = ar + oY;
    d.X = reinterpret_cast<double*>(ar + oX);
    d.Xi = f32 ? reinterpret_cast<double*>(ar + oXi) : d.X;
    d.B = reinterpret_cast<double*>(ar + oB);
    d.R64 = reinterpret_cast<double*>(ar + oR64);
    d.part_rho = reinterpret_cast<double*>(ar + oPr);
    d.part_b = reinterpret_cast<double*>(ar + oPb);
    d.part_phi = reinterpret_cast<double*>(ar + oPp);
    d.part_theta = reinterpret_cast<double*>(ar + oPt);
    d.st = reinterpret_cast<MState*>(ar + oSt);
    MDesc* dd = reinterpret_cast<MDesc*>(ar + oD);
    // right-hand sides: caller's column-major block -> row-major, padded
    PLSS_HIP(hipMemcpyAsync(ar + oBin, Bcm, 8ull * m * ncols, hipMemcpyDefault, s));
    launch_transpose_in(reinterpret_cast<double*>(ar + oBin), m, ncols, W, const_cast<double*>(d.B), s);
    PLSS_HIP(hipMemsetAsync(d.X, 0, 8ull * n * W, s));
    if (f32) PLSS_HIP(hipMemsetAsync(d.Xi, 0, 8ull * n * W, s));
    PLSS_HIP(hipMemsetAsync(d.P, 0, vs * n * W, s));
    MState st;
    std::memset(&st, 0, sizeof(st));
    for (int c = 0; c < kMaxCols; ++c) {
      st.done[c] = 1;
      st.final_[c] = c >= ncols ? 1 : 0;
      st.nu[c] = f32 ? 0.0 : 1.0;
    }
    st.tol = o->tol;
    st.inner_tol = f32 && o->refine ? o->inner_tol : o->tol;
    st.maxit = o->maxit;
    st.max_outer = f32 && o->refine ? o->max_outer : 1;
    st.tol_abs = o->tol_absolute ? 1 : 0;
    PLSS_HIP(hipMemcpyAsync(d.st, &st, sizeof(st), hipMemcpyHostToDevice, s));
    PLSS_HIP(hipMemcpyAsync(dd, &d, sizeof(d), hipMemcpyHostToDevice, s));

    auto outer_step = [&]() {
      launch_maxpy(dd, std::min(65536, (int)(((long long)n * W + 1023) / 1024)), s);
      launch_spmm(MMODE_REFINE, f32, W, dd, na_blk, s);
      launch_mouter(dd, s);
      launch_mstart(f32, dd, na_blk, s);
    };
    hipEvent_t e0 = ws.t0, e1 = ws.t1;
    PLSS_HIP(hipEventRecord(e0, s));
    outer_step();
    // iterations per chunk: 8, then predicted from the residuals' decrease
    // (the slowest unfinished column of the inner solve; iterations past
    // the last column's stop exit at once)
    constexpr int kFirst = 8, kCap = 64;
    int chunk = o->chunk > 0 ? o->chunk : kFirst;
    std::vector<double> lr_prev(ncols, 0.0), kt_prev(ncols, -1.0);
    long long outer_prev = -1;
    const bool timing = o->timing != 0;
    // per-phase timing events (only with opts.timing) around the phases of
    // one iteration in eight (iterations 2, 10, ... of a chunk), read after
    // the chunk's state copy; destroyed on every exit
    constexpr int kTimeEvery = 8, kTimeOffset = 2;
    struct Events {
      std::vector<hipEvent_t> v;
      ~Events() {
        for (auto e : v) (void)hipEventDestroy(e);
      }
    } evs;
    std::vector<hipEvent_t>& ev = evs.v;
    std::vector<long long> kt_chunk(ncols, 0);  // updates of each column before the chunk
    while (true) {
      const int nsamp = chunk > kTimeOffset ? (chunk - kTimeOffset + kTimeEvery - 1) / kTimeEvery : 0;
      while (timing && (int)ev.size() < 5 * nsamp) {
        hipEvent_t e;
        PLSS_HIP(hipEventCreate(&e));
        ev.push_back(e);
      }
      int ne = 0;
      for (int c = 0; c < chunk; ++c) {
        const hipEvent_t* e = (timing && c % kTimeEvery == kTimeOffset) ? &ev[5 * ne++] : nullptr;
        if (e) PLSS_HIP(hipEventRecord(e[0], s));
        launch_spmm(MMODE_RESID, f32, W, dd, na_blk, s);
        if (e) PLSS_HIP(hipEventRecord(e[1], s));
        launch_spmm(MMODE_TRANS, f32, W, dd, nt_blk, s);
        if (e) PLSS_HIP(hipEventRecord(e[2], s));
        launch_mstep(dd, W, s);
        if (e) PLSS_HIP(hipEventRecord(e[3], s));
        launch_mupdate(f32, dd, nu_blk, s);
        if (e) PLSS_HIP(hipEventRecord(e[4], s));
      }
      PLSS_HIP(hipMemcpyAsync(hst, d.st, sizeof(MState), hipMemcpyDeviceToHost, s));
      PLSS_HIP(hipStreamSynchronize(s));
      if (timing) {
        // iterations in which some column made an update: the first `live`
        // of the chunk (a column's updates are consecutive); later ones only
        // exit early and are not counted
        long long live = 0;
        for (int c = 0; c < ncols; ++c) live = std::max(live, hst->k_total[c] - kt_chunk[c]);
        for (int it = 0; it < ne && kTimeOffset + kTimeEvery * it < live; ++it) {
          for (int q = 0; q < 4; ++q) {
            float ms = 0;
            PLSS_HIP(hipEventElapsedTime(&ms, ev[5 * it + q], ev[5 * it + q + 1]));
            h->kt_ms[q] += ms;
            h->kt_n[q] += 1;
          }
        }
      }
      if (hst->all_done) break;
      bool all_inner = true;
      for (int c = 0; c < ncols; ++c) all_inner &= (hst->done[c] != 0);
      if (all_inner) {
        outer_step();
        PLSS_HIP(hipMemcpyAsync(hst, d.st, sizeof(MState), hipMemcpyDeviceToHost, s));
        PLSS_HIP(hipStreamSynchronize(s));
        if (hst->all_done) break;
      }
      if (o->chunk <= 0) {
        bool known = hst->outer == outer_prev;
        double rem_max = 0.0;
        for (int c = 0; c < ncols; ++c) {
          if (hst->done[c]) continue;
          const double rem = known && kt_prev[c] >= 0.0
                                 ? steps_left(hst->rho[c], hst->thr[c], (double)hst->k_total[c], lr_prev[c], kt_prev[c])
                                 : -1.0;
          if (rem < 0.0) known = false;
          else rem_max = std::max(rem_max, std::min(rem, (double)(hst->maxit - hst->k_total[c])));
        }
        chunk = chunk_for(known ? rem_max : -1.0, kFirst, kCap);
        for (int c = 0; c < ncols; ++c) {
          lr_prev[c] = 0.5 * std::log(std::max(hst->rho[c], 1e-300));
          kt_prev[c] = hst->done[c] ? -1.0 : (double)hst->k_total[c];
        }
        outer_prev = hst->outer;
      }
      for (int c = 0; c < ncols; ++c) kt_chunk[c] = hst->k_total[c];
    }
    PLSS_HIP(hipEventRecord(e1, s));
    PLSS_HIP(hipEventSynchronize(e1));
    float ms = 0;
    PLSS_HIP(hipEventElapsedTime(&ms, e0, e1));
    // solution: row-major padded -> caller's column-major block
    double* out = reinterpret_cast<double*>(ar + oBin);
    launch_transpose_out(d.X, n, ncols, W, out, s);
    PLSS_HIP(hipMemcpyAsync(Xcm, out, 8ull * n * ncols, hipMemcpyDefault, s));
    PLSS_HIP(hipStreamSynchronize(s));
    for (int c = 0; c < ncols; ++c) {
      plss_info& inf = info[c];
      inf.iters = hst->k_total[c];
      inf.outer_iters = hst->outer - 1;
      inf.relres = hst->nu[c] > 0 ? sqrt(hst->rho[c]) * hst->nu[c] / (hst->nb_out[c] > 0 ? hst->nb_out[c] : 1.0) : 0.0;
      inf.relres_true = hst->relres_true[c];
      inf.status = hst->final_status[c];
      inf.ms = ms;
      if (agg == PLSS_OK && inf.status != PLSS_OK) agg = (plss_status)inf.status;
    }
  } catch (...) {
    (void)hipStreamSynchronize(s);
    throw;
  }
  return agg;
}
}  // namespace

plss_status multi_solve(plss_handle* h, const plss_matrix* A, int nrhs, const double* B, const plss_opts* o,
                        double* X, plss_info* info, hipStream_t s) {
  if (o->wi_diag || o->x0) throw InvalidArg{"multi-RHS solves take W = I and x0 = 0"};
  if (!info) throw InvalidArg{"info array required"};
  plss_status agg = PLSS_OK;
  for (int c0 = 0; c0 < nrhs; c0 += kMaxCols) {
    const int nc = std::min(kMaxCols, nrhs - c0);
    const plss_status st = run_group(h, A, nc, B + (size_t)c0 * A->m, o, X + (size_t)c0 * A->n, info + c0, s);
    if (agg == PLSS_OK) agg = st;
  }
  return agg;
}

}  // namespace plss
