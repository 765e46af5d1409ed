// Driver of the identity and mixed sketches (one sketch column per step).
#include "sketch.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "solve.hpp"

namespace plss {

namespace {
size_t up(size_t v) { return (v + 255) / 256 * 256; }
}  // namespace

void sketch_solve(plss_handle* h, const plss_matrix* A, const double* b, const plss_opts* o, double* x,
                  double* hist, long long hist_cap_out, plss_info* info, hipStream_t s) {
  if (A->f32) throw InvalidArg{"identity/mixed sketches need float64 storage"};
  if (o->wi_diag) throw InvalidArg{"wi_diag applies to the residual sketch only"};
  if (o->x0) throw InvalidArg{"identity/mixed sketches start from x0 = 0"};
  check_finite_inputs(A, b, o, s);
  const int m = (int)A->m, n = (int)A->n;
  long long cap = o->hist_cap > 0 ? o->hist_cap : std::min<long long>({(long long)m, (long long)n, 256});
  if (cap > 256) throw InvalidArg{"hist_cap must be at most 256"};
  cap = std::min<long long>(cap, std::min(m, n));
  // row order: validated permutation of 0..m-1
  std::vector<int> perm(m);
  if (o->row_perm) {
    PLSS_HIP(hipMemcpy(perm.data(), o->row_perm, sizeof(int) * m, hipMemcpyDefault));
    std::vector<char> seen(m, 0);
    for (int i = 0; i < m; ++i) {
      if (perm[i] < 0 || perm[i] >= m || seen[perm[i]]) throw InvalidArg{"row_perm is not a permutation"};
      seen[perm[i]] = 1;
    }
  } else {
    for (int i = 0; i < m; ++i) perm[i] = i;
  }

  // column blocks of A for the product A p when the new column of P does
  // not fit one XCD's L2 (built once per matrix, on its first sketch solve;
  // calls on the matrix's handle are serialised)
  build_col_blocks(const_cast<plss_matrix*>(A), s);
  const int cnb = A->cnblk;
  int qcb = 0;  // tile groups of the largest column block
  for (int b = 0; b < cnb && cnb > 1; ++b) qcb = std::max(qcb, A->CB[b].ntiles);
  const size_t ncbl = cnb > 1 ? (size_t)kMaxBlk * qcb : 0;

  // the system's arena, state, descriptor, lists and pinned state mirror
  // come from the handle's workspace (calls on a handle are serialised and
  // synchronise before returning)
  Workspace& ws = workspace(h);
  const long long hist_len = std::min<long long>(o->maxit + 2, 1LL << 22);
  const int wblk = (m + 1023) / 1024, u_nblk = (n + 1023) / 1024;
  const size_t nl = (size_t)A->A.ntiles + A->T.ntiles + u_nblk + wblk + ncbl;
  const Workspace::Call cm = ws.call_block(SysRun::arena_bytes(A, o, hist_len, false), sizeof(int2) * nl + sizeof(int));
  State* d_state = cm.d_state;
  Desc* d_desc = cm.d_desc;
  State* h_state = cm.h_state;
  SysRun run;
  char* extra = nullptr;
  try {
    run.use_stripes = false;  // the one-column steps use the tile partition of the partials
    run.setup(A, b, o, hist_len, d_state, cm.arena);
    run.upload(b, nullptr, nullptr, s);
    // history and scratch: P (n x cap), AP (m x cap), Θ, c, partial w, dense row, order
    size_t off = 0;
    const size_t oP = off; off = up(off + 8 * (size_t)n * cap);
    const size_t oAP = off; off = up(off + 8 * (size_t)m * cap);
    const size_t oTh = off; off = up(off + 8 * (size_t)cap);
    const size_t oCv = off; off = up(off + 8 * (size_t)cap);
    const size_t oPw = off; off = up(off + 8 * (size_t)cap * wblk);
    const size_t oDn = off; off = up(off + 8 * (size_t)n);
    const size_t oPm = off; off = up(off + 4 * (size_t)m);
    const size_t oAb = off; off = up(off + (cnb > 1 ? 8 * (size_t)m * cnb : 0));
    // kept by the handle between calls (they are serialised by its mutex and
    // synchronise before returning); nothing in it is read before this call
    // writes it, except the dense row, cleared here
    extra = workspace(h).hist_block(off);
    PLSS_HIP(hipMemsetAsync(extra + oDn, 0, 8 * (size_t)n, s));
    PLSS_HIP(hipMemcpyAsync(extra + oPm, perm.data(), 4 * (size_t)m, hipMemcpyHostToDevice, s));
    Desc d = run.desc;
    d.P = reinterpret_cast<double*>(extra + oP);
    d.AP = reinterpret_cast<double*>(extra + oAP);
    d.Th = reinterpret_cast<double*>(extra + oTh);
    d.cv = reinterpret_cast<double*>(extra + oCv);
    d.part_w = reinterpret_cast<double*>(extra + oPw);
    d.wblk = wblk;
    d.dense = reinterpret_cast<double*>(extra + oDn);
    d.perm = reinterpret_cast<const int*>(extra + oPm);
    d.cnblk = cnb;
    if (cnb > 1) {
      for (int b = 0; b < cnb; ++b) {
        d.cb_ptr[b] = A->CB[b].ptr;
        d.cb_idx[b] = A->CB[b].idx;
        d.cb_val[b] = A->CB[b].val;
        d.cb_tile[b] = A->CB[b].tile;
        d.cb_grp[b] = A->CB[b].grp;
        d.cb_wtd[b] = A->CB[b].wtd;
      }
      d.appart = reinterpret_cast<double*>(extra + oAb);
    }
    d.sketch = o->sketch == PLSS_SKETCH_IDENTITY ? 1 : 2;
    State st = run.st0;
    st.hist_cap = cap;
    st.max_cols = 4 * o->maxit + 4 * (long long)m;
    PLSS_HIP(hipMemcpyAsync(d_desc, &d, sizeof(Desc), hipMemcpyHostToDevice, s));
    PLSS_HIP(hipMemcpyAsync(d_state, &st, sizeof(State), hipMemcpyHostToDevice, s));

    // lists: CSR groups, CSC groups, update blocks, (AP)ᵀ r blocks, the system
    std::vector<int2> la, lt, lu, lw;
    for (int t = 0; t < A->A.ntiles; ++t) la.push_back(make_int2(0, t));
    for (int t = 0; t < A->T.ntiles; ++t) lt.push_back(make_int2(0, t));
    for (int t = 0; t < run.u_nblk; ++t) lu.push_back(make_int2(0, t));
    for (int t = 0; t < wblk; ++t) lw.push_back(make_int2(0, t));
    // column-block tile groups, group q of block b at position 8 q + b so
    // that block b's groups run on XCD b (-1: padding)
    std::vector<int2> lc;
    for (int q = 0; q < qcb && cnb > 1; ++q)
      for (int b = 0; b < kMaxBlk; ++b)
        lc.push_back(make_int2(0, (b < cnb && q < A->CB[b].ntiles) ? ((b << 24) | q) : -1));
    char* d_lists = cm.lists;
    int2* dla = reinterpret_cast<int2*>(d_lists);
    int2* dlt = dla + la.size();
    int2* dlu = dlt + lt.size();
    int2* dlw = dlu + lu.size();
    int2* dlc = dlw + lw.size();
    int* dsys = reinterpret_cast<int*>(dlc + lc.size());
    std::vector<int2> all;
    all.insert(all.end(), la.begin(), la.end());
    all.insert(all.end(), lt.begin(), lt.end());
    all.insert(all.end(), lu.begin(), lu.end());
    all.insert(all.end(), lw.begin(), lw.end());
    all.insert(all.end(), lc.begin(), lc.end());
    if (all.size() != nl) throw DeviceError{};  // the lists' space was sized from the same counts
    PLSS_HIP(hipMemcpyAsync(d_lists, all.data(), sizeof(int2) * nl, hipMemcpyHostToDevice, s));
    PLSS_HIP(hipMemsetAsync(dsys, 0, sizeof(int), s));

    auto outer_seq = [&]() {
      launch_spmv(MODE_REFINE, false, A->A.V, d_desc, dla, (int)la.size(), 0, s);
      launch_outer(d_desc, dsys, 1, s);
      launch_start(false, d_desc, dla, (int)la.size(), s);
    };
    hipEvent_t e0 = ws.t0, e1 = ws.t1;
    {
      PLSS_HIP(hipEventRecord(e0, s));
      outer_seq();
      launch_col_init(d_desc, dsys, 1, s);
      long long t = 0;
      // column steps per chunk: 16, then predicted from the residual's
      // decrease per column examined (steps past the stop exit at once)
      constexpr int kFirst = 16, kCap = 128;
      int chunk = o->chunk > 0 ? o->chunk : kFirst;
      double lr_prev = 0.0, col_prev = -1.0;
      while (true) {
        for (int c = 0; c < chunk; ++c, ++t) {
          const bool resid = (d.sketch == 2) && (t % 2 == 0);
          launch_sketch_step(d_desc, A->A.V, dla, (int)la.size(), dlt, (int)lt.size(), dlu, (int)lu.size(),
                             dlw, (int)lw.size(), dsys, 1, resid, A->T.V, dlc, (int)lc.size(),
                             cnb > 1 ? A->CB[0].V : A->A.V, s);
        }
        PLSS_HIP(hipMemcpyAsync(h_state, d_state, sizeof(State), hipMemcpyDeviceToHost, s));
        PLSS_HIP(hipStreamSynchronize(s));
        if (h_state->done || h_state->final_done) break;
        if (o->chunk <= 0) {
          const State& st = *h_state;
          double rem = col_prev >= 0.0 ? steps_left(st.rho, st.thr, (double)st.col, lr_prev, col_prev) : -1.0;
          if (rem >= 0.0 && st.max_cols > st.col) rem = std::min(rem, (double)(st.max_cols - st.col));
          chunk = chunk_for(rem, kFirst, kCap);
          lr_prev = 0.5 * std::log(std::max(st.rho, 1e-300));
          col_prev = (double)st.col;
        }
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
    info->outer_iters = fs.col;  // sketch columns examined
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
