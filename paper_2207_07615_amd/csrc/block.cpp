// Driver of the block sketches (a block of identity rows, optionally led by
// the residual, appended per step).
#include "block.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "kernels.hpp"
#include "sketch.hpp"
#include "solve.hpp"

namespace plss {

namespace {
size_t up(size_t v) { return (v + 255) / 256 * 256; }
}  // namespace

void block_solve(plss_handle* h, const plss_matrix* A, const double* b, const plss_opts* o, double* x,
                 double* hist, long long hist_cap_out, plss_info* info, hipStream_t s) {
  if (A->f32) throw InvalidArg{"block sketches need float64 storage"};
  if (o->wi_diag) throw InvalidArg{"wi_diag applies to the residual sketch only"};
  if (o->x0) throw InvalidArg{"block sketches start from x0 = 0"};
  const bool residual = o->sketch == PLSS_SKETCH_BLOCK_MIXED;
  const int block = o->block;
  if (block < 1 || block + (residual ? 1 : 0) > kBW)
    throw InvalidArg{residual ? "block must be in 1..15 for the mixed block sketch"
                              : "block must be in 1..16 for the identity block sketch"};
  check_finite_inputs(A, b, o, s);
  const int m = (int)A->m, n = (int)A->n;
  long long cap = o->hist_cap > 0 ? o->hist_cap : std::min<long long>({(long long)m, (long long)n, 256});
  if (cap > kBHist) throw InvalidArg{"hist_cap must be at most 1024 for block sketches"};
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
  const int w = block + (residual ? 1 : 0);
  const int lpr = w <= 4 ? 4 : (w <= 8 ? 8 : 16);
  // row stride of the history: the capacity, or one block when the capacity
  // is smaller (the history is then cleared before every block)
  const int kcap = (int)((std::max<long long>(cap, w) + 3) & ~3LL);
  const int wblk = (m + kBRows - 1) / kBRows;
  const int rows_per_wg = 256 / lpr;
  const int nparts = (m + rows_per_wg - 1) / rows_per_wg;

  // the system's arena, state, descriptor, lists and pinned state mirror
  // come from the handle's workspace (calls on a handle are serialised and
  // synchronise before returning)
  Workspace& ws = workspace(h);
  const long long hist_len = std::min<long long>(o->maxit + 2, 1LL << 22);
  const size_t nl = (size_t)A->A.ntiles + A->T.ntiles;
  const Workspace::Call cm = ws.call_block(SysRun::arena_bytes(A, o, hist_len, false), sizeof(int2) * nl + sizeof(int));
  State* d_state = cm.d_state;
  Desc* d_desc = cm.d_desc;
  State* h_state = cm.h_state;
  SysRun run;
  try {
    run.use_stripes = false;  // partials of rho / phi on the tile partition
    run.setup(A, b, o, hist_len, d_state, cm.arena);
    run.upload(b, nullptr, nullptr, s);
    // history and scratch, kept by the handle between calls (calls on a
    // handle are serialised and synchronise before returning); every part
    // is written before it is read
    size_t off = 0;
    const size_t oZ = off; off = up(off + 8 * (size_t)n * kcap);
    const size_t oAZ = off; off = up(off + 8 * (size_t)m * kcap);
    const size_t oL = off; off = up(off + 8 * (size_t)cap * kBW * kBW);
    const size_t oBo = off; off = up(off + 4 * (size_t)cap);
    const size_t oWh = off; off = up(off + 4 * (size_t)cap);
    const size_t oU = off; off = up(off + 8 * (size_t)kcap * kBW);
    const size_t oC = off; off = up(off + 8 * (size_t)kcap * kBW);
    const size_t oPw = off; off = up(off + 8 * (size_t)kcap * wblk);
    const size_t oPr = off; off = up(off + 8 * (size_t)nparts);
    const size_t oPm = off; off = up(off + 4 * (size_t)m);
    const size_t oBs = off; off = up(off + sizeof(BlkState));
    const size_t oBd = off; off = up(off + sizeof(BlkDesc));
    char* mem = workspace(h).hist_block(off);
    PLSS_HIP(hipMemcpyAsync(mem + oPm, perm.data(), 4 * (size_t)m, hipMemcpyHostToDevice, s));
    BlkDesc bd{};
    bd.Zh = reinterpret_cast<double*>(mem + oZ);
    bd.AZh = reinterpret_cast<double*>(mem + oAZ);
    bd.Lh = reinterpret_cast<double*>(mem + oL);
    bd.bo = reinterpret_cast<int*>(mem + oBo);
    bd.wh = reinterpret_cast<int*>(mem + oWh);
    bd.Ug = reinterpret_cast<double*>(mem + oU);
    bd.Cg = reinterpret_cast<double*>(mem + oC);
    bd.part_w = reinterpret_cast<double*>(mem + oPw);
    bd.part_r = reinterpret_cast<double*>(mem + oPr);
    bd.perm = reinterpret_cast<const int*>(mem + oPm);
    bd.bs = reinterpret_cast<BlkState*>(mem + oBs);
    bd.kcap = kcap;
    bd.wblk = wblk;
    bd.nparts = nparts;
    bd.block = block;
    bd.residual = residual ? 1 : 0;
    bd.lpr = lpr;
    BlkState bs{};
    bs.cap = cap;
    bs.max_steps = 4 * o->maxit + 4 * (long long)m;
    BlkDesc* d_bd = reinterpret_cast<BlkDesc*>(mem + oBd);
    PLSS_HIP(hipMemcpyAsync(d_bd, &bd, sizeof(BlkDesc), hipMemcpyHostToDevice, s));
    PLSS_HIP(hipMemcpyAsync(bd.bs, &bs, sizeof(BlkState), hipMemcpyHostToDevice, s));
    Desc d = run.desc;
    d.perm = bd.perm;
    State st = run.st0;
    PLSS_HIP(hipMemcpyAsync(d_desc, &d, sizeof(Desc), hipMemcpyHostToDevice, s));
    PLSS_HIP(hipMemcpyAsync(d_state, &st, sizeof(State), hipMemcpyHostToDevice, s));

    // lists: CSR groups (initial and final residual), CSC groups (y = Aᵀ r), the system
    std::vector<int2> all;
    for (int t = 0; t < A->A.ntiles; ++t) all.push_back(make_int2(0, t));
    for (int t = 0; t < A->T.ntiles; ++t) all.push_back(make_int2(0, t));
    char* d_lists = cm.lists;
    int2* dla = reinterpret_cast<int2*>(d_lists);
    int2* dlt = dla + A->A.ntiles;
    int* dsys = reinterpret_cast<int*>(dlt + A->T.ntiles);
    if (all.size() != nl) throw DeviceError{};  // the lists' space was sized from the same counts
    PLSS_HIP(hipMemcpyAsync(d_lists, all.data(), sizeof(int2) * all.size(), hipMemcpyHostToDevice, s));
    PLSS_HIP(hipMemsetAsync(dsys, 0, sizeof(int), s));

    auto outer_seq = [&]() {
      launch_spmv(MODE_REFINE, false, A->A.V, d_desc, dla, A->A.ntiles, 0, s);
      launch_outer(d_desc, dsys, 1, s);
      launch_start(false, d_desc, dla, A->A.ntiles, s);
    };
    hipEvent_t e0 = ws.t0, e1 = ws.t1;
    {
      PLSS_HIP(hipEventRecord(e0, s));
      outer_seq();
      launch_col_init(d_desc, dsys, 1, s);
      // block steps per chunk: 8, then predicted from the residual's
      // decrease per block step (steps past the stop exit at once)
      constexpr int kFirst = 8, kCap = 64;
      int chunk = o->chunk > 0 ? o->chunk : kFirst;
      double lr_prev = 0.0, steps_prev = -1.0;
      while (true) {
        for (int c = 0; c < chunk; ++c)
          launch_block_step(d_desc, d_bd, residual, lpr, A->T.V, dlt, A->T.ntiles, n, wblk, nparts, s);
        PLSS_HIP(hipMemcpyAsync(h_state, d_state, sizeof(State), hipMemcpyDeviceToHost, s));
        PLSS_HIP(hipStreamSynchronize(s));
        if (h_state->done || h_state->final_done) break;
        if (o->chunk <= 0) {
          const State& st = *h_state;  // st.col counts the block steps
          const double rem = steps_prev >= 0.0 ? steps_left(st.rho, st.thr, (double)st.col, lr_prev, steps_prev) : -1.0;
          chunk = chunk_for(rem, kFirst, kCap);
          lr_prev = 0.5 * std::log(std::max(st.rho, 1e-300));
          steps_prev = (double)st.col;
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
    info->outer_iters = fs.col;  // blocks examined
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
