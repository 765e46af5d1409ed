// Iteration driver: one or many residual-sketch systems advanced together.
//
// Every launch walks a list of (system, tile) pairs; systems that finished
// are dropped from the lists at the next host check.  Decisions of the
// method (stop test, breakdown, refinement restarts) are taken on the device
// by k_step / k_outer, so a chunk of iterations runs without host
// round-trips; the host only reads the per-system State once per chunk.
#include "solve.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>

namespace plss {

static size_t align_up(size_t v, size_t a = 256) { return (v + a - 1) / a * a; }

void validate_opts(const plss_opts* o, bool f32) {
  if (!o) throw InvalidArg{"null opts"};
  if (!(o->tol > 0.0) || !std::isfinite(o->tol)) throw InvalidArg{"tol must be positive and finite"};
  if (o->maxit <= 0) throw InvalidArg{"maxit must be positive"};
  if (o->sketch < PLSS_SKETCH_RESIDUAL || o->sketch > PLSS_SKETCH_RANDPROJ)
    throw InvalidArg{"unknown sketch"};
  if (f32 && o->refine && (!(o->inner_tol > 0.0) || !(o->inner_tol < 1.0)))
    throw InvalidArg{"inner_tol must be in (0, 1)"};
  if (f32 && o->refine && o->max_outer <= 0) throw InvalidArg{"max_outer must be positive"};
  if (o->chunk < 0) throw InvalidArg{"chunk must be >= 0"};
  if (o->engine < 0 || o->engine > 2) throw InvalidArg{"engine must be 0, 1 or 2"};
}

SysRun::~SysRun() {
  if (own_arena) dfree(arena);
}

namespace {
// Offsets of the per-system vectors and partials inside one arena.
struct Layout {
  size_t o_b, o_xo, o_x, o_r64, o_r, o_p, o_y, o_c, o_wi, o_pr, o_pb, o_pp, o_pt, o_yp, o_h, total;
  int rho_cnt;
};
Layout plan(const plss_matrix* M, const plss_opts* o, long long hist_len, bool use_stripes) {
  const bool f32 = M->f32;
  const size_t m = M->m, n = M->n;
  const size_t vs = f32 ? 4 : 8;
  const int u_nblk = (int)((n + 1023) / 1024);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o2 = off;
    off = align_up(off + bytes);
    return o2;
  };
  Layout L{};
  L.o_b = take(8 * m);
  L.o_xo = take(8 * n);
  L.o_x = f32 ? take(8 * n) : 0;
  L.o_r64 = take(8 * m);
  L.o_r = take(vs * m);
  L.o_p = take(vs * n);
  L.o_y = take(vs * n);
  L.o_c = f32 ? take(vs * m) : 0;
  L.o_wi = o->wi_diag ? take(8 * n) : 0;
  const bool as = use_stripes && M->a_striped;
  L.rho_cnt = as ? M->SA.nunits : M->A.ntiles;
  L.o_pr = take(8 * (size_t)L.rho_cnt);
  L.o_pb = take(8 * (size_t)L.rho_cnt);
  L.o_pp = take(8 * (size_t)std::max(M->T.ntiles, u_nblk));
  L.o_pt = take(8 * (size_t)u_nblk);
  L.o_yp = M->nblk > 1 ? take(vs * n * M->nblk) : 0;
  L.o_h = take(8 * (size_t)std::max<long long>(1, hist_len));
  L.total = off;
  return L;
}
}  // namespace

size_t SysRun::arena_bytes(const plss_matrix* M, const plss_opts* o, long long hist_len, bool use_stripes) {
  return plan(M, o, hist_len, use_stripes).total;
}

void SysRun::setup(const plss_matrix* M, const double* b_in, const plss_opts* o, long long hist_len_in,
                   State* d_state, char* mem) {
  (void)b_in;
  A = M;
  f32 = M->f32;
  const size_t m = M->m, n = M->n;
  u_nblk = (int)((n + 1023) / 1024);
  hist_len = std::max<long long>(1, hist_len_in);
  const Layout L = plan(M, o, hist_len, use_stripes);
  const size_t o_b = L.o_b, o_xo = L.o_xo, o_x = L.o_x, o_r64 = L.o_r64, o_r = L.o_r, o_p = L.o_p, o_y = L.o_y,
               o_c = L.o_c, o_wi = L.o_wi, o_pr = L.o_pr, o_pb = L.o_pb, o_pp = L.o_pp, o_pt = L.o_pt,
               o_yp = L.o_yp, o_h = L.o_h;
  const bool as = use_stripes && M->a_striped, ts = use_stripes && M->t_striped;
  const int rho_cnt = L.rho_cnt;
  if (mem) {
    arena = mem;
    own_arena = false;
  } else {
    arena = static_cast<char*>(dmalloc(L.total));
    own_arena = true;
  }
  bytes = L.total;
  std::memset(&desc, 0, sizeof(desc));
  desc.a_ptr = M->A.ptr;
  desc.a_idx = M->A.idx;
  desc.a_val = M->A.val;
  desc.a_tile = M->A.tile;
  desc.a_ntiles = M->A.ntiles;
  desc.a_nwt = M->A.nwt;
  desc.a_grp = M->A.grp;
  desc.a_wtd = M->A.wtd;
  desc.t_ptr = M->T.ptr;
  desc.t_idx = M->T.idx;
  desc.t_val = M->T.val;
  desc.t_tile = M->T.tile;
  desc.t_ntiles = M->T.ntiles;
  desc.t_nwt = M->T.nwt;
  desc.t_grp = M->T.grp;
  desc.t_wtd = M->T.wtd;
  desc.m = (int)m;
  desc.n = (int)n;
  desc.a_long = M->A.lrows;
  desc.t_long = M->T.lrows;
  desc.a_nlong = M->A.nlong;
  desc.t_nlong = M->T.nlong;
  desc.a_sl_base = M->A.sl_base;
  desc.a_sl_idx = M->A.sl_idx;
  desc.a_sl_val = M->A.sl_val;
  desc.t_sl_base = M->T.sl_base;
  desc.t_sl_idx = M->T.sl_idx;
  desc.t_sl_val = M->T.sl_val;
  desc.u_nblk = u_nblk;
  desc.nblk = M->nblk;
  for (int b = 0; b < M->nblk && M->nblk > 1; ++b) {
    desc.tb_ptr[b] = M->TB[b].ptr;
    desc.tb_idx[b] = M->TB[b].idx;
    desc.tb_val[b] = M->TB[b].val;
    desc.tb_tile[b] = M->TB[b].tile;
    desc.tb_grp[b] = M->TB[b].grp;
    desc.tb_wtd[b] = M->TB[b].wtd;
  }
  desc.a_striped = as ? 1 : 0;
  desc.t_striped = ts ? 1 : 0;
  desc.rho_cnt = rho_cnt;
  if (as) fill_stripe_view(M->SA, &desc.sa);
  if (ts)
    for (int b = 0; b < M->nblk; ++b) fill_stripe_view(M->SB[b], &desc.sb[b]);
  desc.ypart = M->nblk > 1 ? arena + o_yp : nullptr;
  desc.phi_cnt = M->nblk > 1 ? u_nblk : M->T.ntiles;
  desc.b = reinterpret_cast<double*>(arena + o_b);
  desc.xo = reinterpret_cast<double*>(arena + o_xo);
  desc.x = f32 ? reinterpret_cast<double*>(arena + o_x) : desc.xo;
  desc.r64 = reinterpret_cast<double*>(arena + o_r64);
  desc.r = arena + o_r;
  desc.p = arena + o_p;
  desc.y = arena + o_y;
  desc.c = f32 ? arena + o_c : nullptr;
  desc.wi = o->wi_diag ? reinterpret_cast<double*>(arena + o_wi) : nullptr;
  desc.part_rho = reinterpret_cast<double*>(arena + o_pr);
  desc.part_b = reinterpret_cast<double*>(arena + o_pb);
  desc.part_phi = reinterpret_cast<double*>(arena + o_pp);
  desc.part_theta = reinterpret_cast<double*>(arena + o_pt);
  desc.hist = reinterpret_cast<double*>(arena + o_h);
  desc.hist_len = hist_len;
  desc.st = d_state;
  desc.is_f32 = f32;

  // single-workgroup engine: residual sketch, vectors in LDS; automatic up
  // to kSmallNnz entries, where launches and host polls cost more than the work
  const bool fits = o->sketch == PLSS_SKETCH_RESIDUAL && small_fits((int)m, (int)n, f32);
  if (o->engine == 2 && !fits)
    throw InvalidArg{"engine 2 needs the residual sketch and vectors and row pointers within 156 KiB of LDS"};
  small = o->engine == 2 || (o->engine == 0 && fits && M->nnz <= kSmallNnz);

  std::memset(&st0, 0, sizeof(st0));
  st0.done = 1;  // the outer step runs first: r64 = b - A x0, then the inner start
  st0.final_done = 0;
  st0.tol = o->tol;
  st0.tol_out = o->tol;
  st0.tol_abs = o->tol_absolute ? 1 : 0;
  st0.inner_tol = f32 && o->refine ? o->inner_tol : o->tol;
  st0.maxit = o->maxit;
  st0.max_outer = f32 && o->refine ? o->max_outer : 1;
  st0.status = ST_OK;
  st0.nu = f32 ? 0.0 : 1.0;  // set by the outer step before any use
}

void SysRun::upload(const double* b_in, const double* x0, const double* wi, hipStream_t s) {
  const size_t m = A->m, n = A->n;
  PLSS_HIP(hipMemcpyAsync(const_cast<double*>(desc.b), b_in, 8 * m, hipMemcpyDefault, s));
  if (x0) PLSS_HIP(hipMemcpyAsync(desc.xo, x0, 8 * n, hipMemcpyDefault, s));
  else PLSS_HIP(hipMemsetAsync(desc.xo, 0, 8 * n, s));
  if (f32) PLSS_HIP(hipMemsetAsync(desc.x, 0, 8 * n, s));
  if (wi) PLSS_HIP(hipMemcpyAsync(const_cast<double*>(desc.wi), static_cast<const void*>(wi), 8 * n, hipMemcpyDefault, s));
}

// ------------------------------------------------------------------ batch runner

char* Workspace::dev_block(size_t bytes) {
  if (bytes > dev_cap) {
    dfree(dev);
    dev = nullptr;
    dev_cap = 0;
    const size_t want = std::max(bytes, dev_cap + dev_cap / 2);
    dev = static_cast<char*>(dmalloc(want));
    dev_cap = want;
  }
  return dev;
}

char* Workspace::pin_block(size_t bytes) {
  if (bytes > pin_cap) {
    if (pin) (void)hipHostFree(pin);
    pin = nullptr;
    pin_cap = 0;
    const size_t want = std::max<size_t>(bytes, 4096);
    PLSS_HIP(hipHostMalloc(reinterpret_cast<void**>(&pin), want, hipHostMallocDefault));
    pin_cap = want;
  }
  return pin;
}

char* Workspace::hist_block(size_t bytes) {
  if (bytes > hist_cap) {
    dfree(hist);
    hist = nullptr;
    hist_cap = 0;
    hist = static_cast<char*>(dmalloc(bytes));
    hist_cap = bytes;
  }
  return hist;
}

Workspace::Call Workspace::call_block(size_t arena_bytes, size_t list_bytes) {
  auto up = [](size_t v) { return (v + 255) / 256 * 256; };
  const size_t o_st = up(arena_bytes), o_d = up(o_st + sizeof(State)), o_l = up(o_d + sizeof(Desc));
  char* dv = dev_block(o_l + list_bytes + 64);
  Call c;
  c.arena = dv;
  c.d_state = reinterpret_cast<State*>(dv + o_st);
  c.d_desc = reinterpret_cast<Desc*>(dv + o_d);
  c.lists = dv + o_l;
  c.h_state = reinterpret_cast<State*>(pin_block(sizeof(State)));
  return c;
}

Workspace::~Workspace() {
  if (aux) (void)hipStreamSynchronize(aux);
  dfree(dev);
  dfree(hist);
  if (pin) (void)hipHostFree(pin);
  if (t0) (void)hipEventDestroy(t0);
  if (t1) (void)hipEventDestroy(t1);
  if (ready) (void)hipEventDestroy(ready);
  if (small_done) (void)hipEventDestroy(small_done);
  if (aux) (void)hipStreamDestroy(aux);
  for (auto e : iter_events) (void)hipEventDestroy(e);
}

Workspace& workspace(plss_handle* h) {
  if (!h->ws) {
    std::unique_ptr<Workspace> w(new Workspace());
    PLSS_HIP(hipEventCreate(&w->t0));
    PLSS_HIP(hipEventCreate(&w->t1));
    PLSS_HIP(hipEventCreateWithFlags(&w->ready, hipEventDisableTiming));
    PLSS_HIP(hipEventCreateWithFlags(&w->small_done, hipEventDisableTiming));
    PLSS_HIP(hipStreamCreateWithFlags(&w->aux, hipStreamNonBlocking));
    h->ws = w.release();
  }
  return *h->ws;
}

void workspace_free(Workspace* w) { delete w; }

BatchRunner::BatchRunner(plss_handle* h) : h_(h), ws_(workspace(h)) {}

BatchRunner::~BatchRunner() {
  // after an error the second stream may still run on workspace memory
  if (aux_used_) (void)hipStreamSynchronize(ws_.aux);
}

// ------------------------------------------------------------------ launch lists

ListSet::~ListSet() {
  dfree(d);
  if (hbuf) (void)hipHostFree(hbuf);
}

void ListSet::build(const std::vector<std::pair<int, const SysRun*>>& items, hipStream_t s) {
  std::map<int, std::vector<int2>> la, lt, lu, laf, lsa, lsb;
  std::vector<int> ls;
  any_f32 = any_blk = false;
  for (const auto& it : items) {
    const int i = it.first;
    const SysRun& r = *it.second;
    const plss_matrix* M = r.A;
    const int f = r.f32 ? 1 : 0;
    any_f32 |= r.f32;
    auto& AF = laf[f];
    if (r.desc.a_striped) {
      auto& A = lsa[f];
      for (int q = 0; q < M->SA.nunits; ++q) {
        A.push_back(make_int2(i, q));
        AF.push_back(make_int2(i, q));
      }
    } else {
      auto& A = la[f * 100 + M->A.V];
      for (int t = 0; t < M->A.ntiles; ++t) {
        A.push_back(make_int2(i, t));
        AF.push_back(make_int2(i, t));
      }
    }
    if (r.desc.t_striped) {
      // unit q of block b at position 8 q + b: block b's units run on XCD b
      any_blk = true;
      auto& T = lsb[f];
      int qmax = 0;
      for (int b = 0; b < M->nblk; ++b) qmax = std::max(qmax, M->SB[b].nunits);
      for (int q = 0; q < qmax; ++q)
        for (int b = 0; b < kMaxBlk; ++b)
          T.push_back(make_int2(i, (b < M->nblk && q < M->SB[b].nunits) ? ((b << 24) | q) : -1));
    } else if (M->nblk > 1) {
      any_blk = true;
      auto& T = lt[1000 + f * 100 + M->T.V];
      int qmax = 0;
      for (int b = 0; b < M->nblk; ++b) qmax = std::max(qmax, M->TB[b].ntiles);
      for (int q = 0; q < qmax; ++q)
        for (int b = 0; b < kMaxBlk; ++b)
          T.push_back(make_int2(i, (b < M->nblk && q < M->TB[b].ntiles) ? ((b << 24) | q) : -1));
    } else {
      auto& T = lt[f * 100 + M->T.V];
      for (int t = 0; t < M->T.ntiles; ++t) T.push_back(make_int2(i, t));
    }
    auto& U = lu[f];
    for (int t = 0; t < r.u_nblk; ++t) U.push_back(make_int2(i, t));
    ls.push_back(i);
  }
  size_t total = ls.size() * sizeof(int) + 64;
  for (auto* mp : {&la, &lt, &lu, &laf, &lsa, &lsb})
    for (auto& kv : *mp) total += kv.second.size() * sizeof(int2) + 64;
  if (total > cap) {
    dfree(d);
    d = nullptr;
    if (hbuf) (void)hipHostFree(hbuf);
    hbuf = nullptr;
    cap = total * 2;
    d = static_cast<char*>(dmalloc(cap));
    PLSS_HIP(hipHostMalloc(reinterpret_cast<void**>(&hbuf), cap, hipHostMallocDefault));
  }
  // the host buffer may still feed a copy of the previous build
  PLSS_HIP(hipStreamSynchronize(s));
  size_t off = 0;
  auto put = [&](std::map<int, std::vector<int2>>& mp, std::vector<Group>& out) {
    out.clear();
    for (auto& kv : mp) {
      if (kv.second.empty()) continue;
      std::memcpy(hbuf + off, kv.second.data(), kv.second.size() * sizeof(int2));
      out.push_back({kv.first, reinterpret_cast<const int2*>(d + off), (int)kv.second.size()});
      off = align_up(off + kv.second.size() * sizeof(int2), 64);
    }
  };
  put(la, a);
  put(lt, t);
  put(lu, u);
  put(laf, af);
  put(lsa, sa);
  put(lsb, sb);
  std::memcpy(hbuf + off, ls.data(), ls.size() * sizeof(int));
  sys = reinterpret_cast<const int*>(d + off);
  nsys = (int)ls.size();
  off += ls.size() * sizeof(int);
  PLSS_HIP(hipMemcpyAsync(d, hbuf, off, hipMemcpyHostToDevice, s));
}

void ListSet::outer_seq(const Desc* dd, hipStream_t s) const {
  for (auto& g : u) launch_axpy_out(dd, g.list, g.n, s);
  for (auto& g : a) launch_spmv(MODE_REFINE, g.key >= 100, g.key % 100, dd, g.list, g.n, 0, s);
  for (auto& g : sa) launch_sspmv(MODE_REFINE, g.key == 1, dd, g.list, g.n, 0, s);
  launch_outer(dd, sys, nsys, s);
  for (auto& g : af) launch_start(g.key == 1, dd, g.list, g.n, s);
}

void ListSet::iteration(const Desc* dd, hipStream_t s, hipEvent_t* ev) const {
  if (ev) PLSS_HIP(hipEventRecord(ev[0], s));
  for (auto& g : a) launch_spmv(MODE_RESID, g.key >= 100, g.key % 100, dd, g.list, g.n, 0, s);
  for (auto& g : sa) launch_sspmv(MODE_RESID, g.key == 1, dd, g.list, g.n, 0, s);
  if (ev) PLSS_HIP(hipEventRecord(ev[1], s));
  for (auto& g : t) {
    const int k = g.key % 1000;
    launch_spmv(g.key >= 1000 ? MODE_TRANSB : MODE_TRANS, k >= 100, k % 100, dd, g.list, g.n, 1, s);
  }
  for (auto& g : sb) launch_sspmv(MODE_TRANSB, g.key == 1, dd, g.list, g.n, 1, s);
  if (ev) PLSS_HIP(hipEventRecord(ev[2], s));
  if (any_blk)
    for (auto& g : u) launch_ycomb(g.key == 1, dd, g.list, g.n, s);
  launch_step(dd, sys, nsys, s);
  if (ev) PLSS_HIP(hipEventRecord(ev[3], s));
  for (auto& g : u) launch_update(g.key == 1, dd, g.list, g.n, s);
  if (ev) PLSS_HIP(hipEventRecord(ev[4], s));
}

void BatchRunner::add(const plss_matrix* A, const double* b, const plss_opts* o, long long hist_len) {
  validate_opts(o, A->f32);
  if (o->sketch != PLSS_SKETCH_RESIDUAL) throw InvalidArg{"batched solves use the residual sketch"};
  if (o->wi_diag && o->sketch != PLSS_SKETCH_RESIDUAL) throw InvalidArg{"wi_diag needs the residual sketch"};
  Item it;
  it.A = A;
  it.b = b;
  it.o = *o;
  it.hist_len = hist_len;
  items_.push_back(it);
}

void BatchRunner::prepare(hipStream_t s) {
  const int ns = (int)items_.size();
  // one device block from the handle's workspace: states, descriptors, the
  // single-workgroup system list, then every system's arena
  const size_t o_state = 0;
  const size_t o_desc = align_up(o_state + sizeof(State) * ns);
  const size_t o_small = align_up(o_desc + sizeof(Desc) * ns);
  size_t off = align_up(o_small + sizeof(int) * ns);
  std::vector<size_t> o_arena(ns);
  for (int i = 0; i < ns; ++i) {
    o_arena[i] = off;
    off = align_up(off + SysRun::arena_bytes(items_[i].A, &items_[i].o, std::max<long long>(1, items_[i].hist_len),
                                             true));
  }
  char* dev = ws_.dev_block(off);
  // pinned: states, descriptors, single-workgroup system list (sized once here,
  // so the block does not move while copies from it are pending)
  char* pin = ws_.pin_block(sizeof(State) * ns + sizeof(Desc) * ns + sizeof(int) * ns);
  d_state_ = reinterpret_cast<State*>(dev + o_state);
  d_desc_ = reinterpret_cast<Desc*>(dev + o_desc);
  d_small_ = reinterpret_cast<int*>(dev + o_small);
  h_state_ = reinterpret_cast<State*>(pin);
  Desc* h_desc = reinterpret_cast<Desc*>(pin + sizeof(State) * ns);
  h_small_ = reinterpret_cast<int*>(pin + sizeof(State) * ns + sizeof(Desc) * ns);
  runs_.resize(ns);
  for (int i = 0; i < ns; ++i) {
    Item& it = items_[i];
    runs_[i].reset(new SysRun());
    SysRun& r = *runs_[i];
    r.setup(it.A, it.b, &it.o, it.hist_len, d_state_ + i, dev + o_arena[i]);
    r.upload(it.b, it.o.x0, it.o.wi_diag, s);
    h_desc[i] = r.desc;
    h_state_[i] = r.st0;
  }
  PLSS_HIP(hipMemcpyAsync(d_desc_, h_desc, sizeof(Desc) * ns, hipMemcpyHostToDevice, s));
  PLSS_HIP(hipMemcpyAsync(d_state_, h_state_, sizeof(State) * ns, hipMemcpyHostToDevice, s));
}

void BatchRunner::build_lists(const std::vector<int>& active, hipStream_t s) {
  std::vector<std::pair<int, const SysRun*>> items;
  for (int i : active) items.push_back({i, runs_[i].get()});
  ws_.lists.build(items, s);
}

double steps_left(double rho, double thr, double steps, double lr_prev, double steps_prev) {
  const double ds = steps - steps_prev;
  if (!(ds >= 2.0) || !(thr > 0.0)) return -1.0;
  const double lr = 0.5 * std::log(std::max(rho, 1e-300));
  const double rate = (lr - lr_prev) / ds;
  if (!(rate < 0.0)) return -1.0;
  return std::max(0.0, (std::log(thr) - lr) / rate);
}

int chunk_for(double rem, int unknown, int cap) {
  if (rem < 0.0) return std::min(unknown, cap);
  const double want = rem <= 16.0 ? std::ceil(rem) + 1.0 : std::ceil(0.5 * rem);
  return (int)std::min<double>(cap, std::max(2.0, want));
}

// most iterations between host checks; the phases of one iteration in
// kTimeEvery carry timing events (iterations kTimeOffset, kTimeOffset +
// kTimeEvery, ... of a chunk: never one that directly follows an outer
// step, which comes before iterations that are multiples of 4)
constexpr int kChunkMax = 256;
constexpr int kTimeEvery = 8, kTimeOffset = 2;

void BatchRunner::run(hipStream_t s, bool timing, int chunk_req) {
  const int ns = (int)items_.size();
  std::vector<int> active, small64, small32;
  for (int i = 0; i < ns; ++i) {
    if (!runs_[i]->small) active.push_back(i);
    else (runs_[i]->f32 ? small32 : small64).push_back(i);
  }
  hipEvent_t t0 = ws_.t0, t1 = ws_.t1;
  PLSS_HIP(hipEventRecord(t0, s));
  const bool any_small = !small64.empty() || !small32.empty();
  if (any_small) {
    // one persistent launch per storage type on the second stream, after the
    // uploads; each workgroup solves its system while the per-phase launches
    // of the other systems run on `s`
    int k = 0;
    for (int i : small64) h_small_[k++] = i;
    for (int i : small32) h_small_[k++] = i;
    PLSS_HIP(hipMemcpyAsync(d_small_, h_small_, sizeof(int) * k, hipMemcpyHostToDevice, s));
    PLSS_HIP(hipEventRecord(ws_.ready, s));
    PLSS_HIP(hipStreamWaitEvent(ws_.aux, ws_.ready, 0));
    aux_used_ = true;
    launch_small(false, d_desc_, d_small_, (int)small64.size(), ws_.aux);
    launch_small(true, d_desc_, d_small_ + small64.size(), (int)small32.size(), ws_.aux);
    PLSS_HIP(hipEventRecord(ws_.small_done, ws_.aux));
  }
  if (active.empty()) {
    PLSS_HIP(hipStreamWaitEvent(s, ws_.small_done, 0));
    PLSS_HIP(hipMemcpyAsync(h_state_, d_state_, sizeof(State) * ns, hipMemcpyDeviceToHost, s));
    PLSS_HIP(hipEventRecord(t1, s));
    PLSS_HIP(hipEventSynchronize(t1));
    float ms = 0;
    PLSS_HIP(hipEventElapsedTime(&ms, t0, t1));
    elapsed_ms_ = ms;
    return;
  }
  build_lists(active, s);
  bool any_f32 = false;
  double bytes_iter = 0;
  for (int i = 0; i < ns; ++i) {
    any_f32 |= runs_[i]->f32;
    const plss_matrix* M = runs_[i]->A;
    bytes_iter += (M->f32 ? 16.0 : 24.0) * M->nnz + 28.0 * M->m + 60.0 * M->n;
  }
  // Iterations per chunk (between host checks).  The first chunk is short
  // (small systems finish early); after it, a system's observed decrease of
  // ln ||r|| per update over the last chunk predicts the updates left to its
  // stop test, and the next chunk covers the slowest prediction.  An
  // iteration launched after a system stopped costs only early-exit
  // launches; a chunk ended too soon costs one more host check.
  const double t_iter = bytes_iter / 4.0e12 + 20e-6;
  const int cfirst = (int)std::min(16.0, std::max(4.0, 4e-3 / t_iter));
  int chunk = chunk_req > 0 ? chunk_req : cfirst;
  // float32 storage: the outer (refinement) step also runs every outer_every
  // iterations inside a chunk, so an inner solve that stops between host
  // checks is refined soon; often in a batch, where systems stop at
  // different times and the last one sets the batch's length
  const int outer_every = !any_f32 ? 1 << 30 : (ns > 1 ? 4 : 16);  // multiples of 4
  std::vector<hipEvent_t>& events_ = ws_.iter_events;
  if (timing && events_.empty()) {
    events_.resize(5 * (kChunkMax / kTimeEvery + 1));
    for (auto& e : events_) PLSS_HIP(hipEventCreate(&e));
  }
  std::vector<double> lr_prev(ns, 0.0);
  std::vector<long long> kt_prev(ns, -1), outer_prev(ns, -1), kt_chunk(ns, 0);
  const ListSet& lists_ = ws_.lists;
  // the outer step ends every chunk, so it starts only the first: after it
  // no running system is stopped and unrefined, and repeating it changes nothing
  lists_.outer_seq(d_desc_, s);
  while (!active.empty()) {
    const int c = std::min(chunk, kChunkMax);
    // iterations timed: one in kTimeEvery, so the events barely slow the
    // rest, and never one right after an outer step, whose product with A
    // is skipped when it starts an inner solve
    int ne = 0;
    // updates of each system so far (h_state_ holds the last sync)
    for (int i : active) kt_chunk[i] = h_state_[i].k_total;
    for (int it = 0; it < c; ++it) {
      if (it > 0 && it % outer_every == 0) lists_.outer_seq(d_desc_, s);
      const bool tev = timing && it % kTimeEvery == kTimeOffset;
      lists_.iteration(d_desc_, s, tev ? &events_[5 * ne++] : nullptr);
    }
    lists_.outer_seq(d_desc_, s);
    PLSS_HIP(hipMemcpyAsync(h_state_, d_state_, sizeof(State) * ns, hipMemcpyDeviceToHost, s));
    PLSS_HIP(hipStreamSynchronize(s));
    // iterations that made an update: a system's updates are consecutive, so
    // those of the chunk are its first (k_total advanced) ones; the launches
    // after every system stopped only exit early and are not timed
    long long live = 0;
    for (int i : active) live = std::max(live, h_state_[i].k_total - kt_chunk[i]);
    for (int it = 0; it < ne && kTimeOffset + kTimeEvery * it < live; ++it) {
      for (int q = 0; q < 4; ++q) {
        float ms = 0;
        PLSS_HIP(hipEventElapsedTime(&ms, events_[5 * it + q], events_[5 * it + q + 1]));
        h_->kt_ms[q] += ms;
        h_->kt_n[q] += 1;
      }
    }
    std::vector<int> still;
    for (int i : active)
      if (!h_state_[i].final_done) still.push_back(i);
    if (still.size() != active.size()) {
      active.swap(still);
      if (!active.empty()) build_lists(active, s);
    }
    // predicted updates left: the slowest system whose last chunk measured a
    // decrease inside one inner solve
    bool known = !active.empty();
    double rem_max = 0.0;
    for (int i : active) {
      const State& st = h_state_[i];
      const long long dk = st.k_total - kt_prev[i];
      double rem = -1.0;
      if (kt_prev[i] >= 0 && st.outer == outer_prev[i] && !st.done && st.k > dk)
        rem = steps_left(st.rho, st.thr, (double)st.k_total, lr_prev[i], (double)kt_prev[i]);
      if (rem < 0.0) known = false;
      else rem_max = std::max(rem_max, std::min(rem, (double)(st.maxit - st.k_total)));
      kt_prev[i] = st.k_total;
      lr_prev[i] = 0.5 * std::log(std::max(st.rho, 1e-300));
      outer_prev[i] = st.outer;
    }
    if (chunk_req <= 0) chunk = chunk_for(known ? rem_max : -1.0, cfirst, kChunkMax);
  }
  if (any_small) {
    // the single-workgroup systems' final states
    PLSS_HIP(hipStreamWaitEvent(s, ws_.small_done, 0));
    PLSS_HIP(hipMemcpyAsync(h_state_, d_state_, sizeof(State) * ns, hipMemcpyDeviceToHost, s));
  }
  PLSS_HIP(hipEventRecord(t1, s));
  PLSS_HIP(hipEventSynchronize(t1));
  float ms = 0;
  PLSS_HIP(hipEventElapsedTime(&ms, t0, t1));
  elapsed_ms_ = ms;
}

void BatchRunner::result(int i, double* x, double* hist, long long hist_cap, plss_info* info,
                         hipStream_t s) {
  const SysRun& r = *runs_[i];
  const State& st = h_state_[i];
  if (x) PLSS_HIP(hipMemcpyAsync(x, r.desc.xo, 8 * (size_t)r.A->n, hipMemcpyDefault, s));
  const long long nh = std::min<long long>({hist_cap, st.k_total + 1, r.hist_len});
  if (hist && nh > 0) PLSS_HIP(hipMemcpyAsync(hist, r.desc.hist, 8 * nh, hipMemcpyDefault, s));
  PLSS_HIP(hipStreamSynchronize(s));
  if (info) {
    info->iters = st.k_total;
    info->outer_iters = st.outer;
    info->relres = sqrt(st.rho) * st.scale;
    info->relres_true = st.relres_true;
    info->status = st.final_status;
    info->ms = elapsed_ms_;
  }
}

}  // namespace plss
