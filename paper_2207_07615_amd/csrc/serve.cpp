// Request loop with continuous batching.
//
// A server thread owns three streams of the handle's device.  Each pass of
// its loop enqueues one chunk of iterations for every admitted system on the
// main stream, then - while that chunk runs - admits queued requests: their
// device footprint must fit under the budget next to the admitted systems
// and a slot must be free; admission uploads the matrix and builds its CSC
// copy on the side stream.  After the chunk, finished systems are copied back
// to host memory, their device memory is freed and their slot released, and
// the systems admitted meanwhile join the next chunk (the per-phase engine:
// all in-flight systems share every launch, which keeps the whole GPU busy).
// A request that asks for the single-workgroup engine (opts.engine = 2)
// instead runs whole, one launch, on the third stream beside the chunks, and
// retires when its event completes.  A system's arithmetic depends only on
// its own data, so its result does not depend on which other systems share
// the GPU.
#include "serve.hpp"

#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <thread>
#include <unordered_map>
#include <vector>

#include "solve.hpp"

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

enum ReqState { RQ_QUEUED, RQ_ACTIVE, RQ_DONE, RQ_CANCELLED, RQ_FAILED };

struct Req {
  uint64_t id = 0;
  ReqState state = RQ_QUEUED;
  bool cancel = false;
  // host copies of the inputs
  long long m = 0, n = 0, nnz = 0;
  std::vector<int64_t> rp;
  std::vector<int> ci;
  std::vector<double> va, b;
  plss_dtype storage = PLSS_F64;
  plss_opts o{};
  size_t resident = 0, transient = 0;
  // while admitted
  plss_matrix* M = nullptr;
  std::unique_ptr<plss::SysRun> run;
  int slot = -1;
  // results
  std::vector<double> x;
  plss_info info{};
  plss_status fail = PLSS_OK;
  double t_submit = 0, t_done = 0;
  hipEvent_t done_ev = nullptr;  // single-workgroup solve finished (small systems)
};

}  // namespace

struct plss_server {
  plss_handle* h = nullptr;
  size_t budget = 0;
  int max_slots = 0;
  std::thread th;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  bool stop = false;
  uint64_t next_id = 1;
  std::deque<Req*> queue;
  std::unordered_map<uint64_t, Req*> reqs;
  std::vector<Req*> active;
  size_t in_use = 0, peak = 0;
  long long submitted = 0, finished = 0;
  // device side (server thread only)
  hipStream_t main = nullptr, side = nullptr;
  plss::State* d_slots = nullptr;
  plss::State* h_slots = nullptr;
  plss::Desc* d_desc = nullptr;
  std::vector<plss::Desc> h_desc;
  std::vector<int> free_slots;
  plss::ListSet lists;
  hipStream_t small = nullptr;  // single-workgroup solves, beside the chunks on `main`
  int* d_slot_ids = nullptr;     // slot i holds i: the system list of a one-system launch
};

namespace plss {

namespace {

size_t sysrun_bytes(long long m, long long n, long long nnz, bool f32, bool wi) {
  const size_t vs = f32 ? 4 : 8;
  const size_t groups = (size_t)(nnz / 64 + m / 64 + n / 64 + 64);
  return 8 * (size_t)m * 2 + 8 * (size_t)n * (f32 ? 2 : 1) + vs * ((size_t)m * (f32 ? 2 : 1) + 2 * (size_t)n) +
         (wi ? 8 * (size_t)n : 0) + 8 * groups * 4 + 64 * 1024;
}

void host_validate(const Req& r) {
  if (r.m <= 0 || r.n <= 0) throw InvalidArg{"m and n must be positive"};
  if (r.rp[0] != 0 || r.rp[r.m] != r.nnz) throw InvalidArg{"row_ptr must start at 0 and end at nnz"};
  for (long long i = 0; i < r.m; ++i) {
    if (r.rp[i + 1] < r.rp[i]) throw InvalidArg{"row_ptr must be non-decreasing"};
    for (long long e = r.rp[i]; e < r.rp[i + 1]; ++e) {
      if (r.ci[e] < 0 || r.ci[e] >= r.n) throw InvalidArg{"column index out of range"};
      if (e + 1 < r.rp[i + 1] && r.ci[e + 1] <= r.ci[e])
        throw InvalidArg{"column indices must be ascending and distinct within a row"};
      if (!std::isfinite(r.va[e])) throw InvalidArg{"non-finite value"};
    }
  }
  for (double v : r.b)
    if (!std::isfinite(v)) throw InvalidArg{"b has a non-finite entry"};
}

// Launch lists of the admitted systems that run on the per-phase engine
// (small systems run whole in one workgroup and are not stepped by chunks).
void rebuild_lists(plss_server* S) {
  std::vector<std::pair<int, const SysRun*>> items;
  for (Req* r : S->active)
    if (!r->run->small) items.push_back({r->slot, r->run.get()});
  S->lists.build(items, S->main);
}

// Small systems that joined run whole, one workgroup each, on the stream of
// their own beside the chunks on `main`; an event marks each one's end.
void launch_joined_small(plss_server* S, const std::vector<Req*>& joined) {
  for (Req* r : joined) {
    if (!r->run->small) continue;
    launch_small(r->run->f32, S->d_desc, S->d_slot_ids + r->slot, 1, S->small);
    if (!r->done_ev) PLSS_HIP(hipEventCreateWithFlags(&r->done_ev, hipEventDisableTiming));
    PLSS_HIP(hipEventRecord(r->done_ev, S->small));
  }
}

// A single-workgroup solve has ended (its memory may then be released).
bool small_finished(Req* r) {
  const hipError_t e = hipEventQuery(r->done_ev);
  if (e == hipSuccess) return true;
  if (e != hipErrorNotReady) {
    set_error(std::string("hipEventQuery: ") + hipGetErrorString(e));
    throw DeviceError();
  }
  (void)hipGetLastError();
  return false;
}

// Upload and prepare one request on the side stream (server thread).
void prepare(plss_server* S, Req* r) {
  plss_csr c;
  c.m = r->m;
  c.n = r->n;
  c.nnz = r->nnz;
  c.row_ptr = r->rp.data();
  c.col_idx = r->ci.data();
  c.values = r->va.data();
  r->M = matrix_create(S->h, &c, r->storage, S->side);  // holds a handle reference
  r->run.reset(new SysRun());
  r->run->setup(r->M, r->b.data(), &r->o, 1, S->d_slots + r->slot, nullptr);
  // throughput: served systems are stepped together on the per-phase engine
  // unless the request asks for the single-workgroup engine (engine 2)
  if (r->o.engine != 2) r->run->small = false;
  r->run->upload(r->b.data(), r->o.x0, r->o.wi_diag, S->side);
  PLSS_HIP(hipMemcpyAsync(S->d_slots + r->slot, &r->run->st0, sizeof(State), hipMemcpyHostToDevice, S->side));
  PLSS_HIP(hipMemcpyAsync(S->d_desc + r->slot, &r->run->desc, sizeof(Desc), hipMemcpyHostToDevice, S->side));
  PLSS_HIP(hipStreamSynchronize(S->side));
  // the inputs are on the device now
  std::vector<int64_t>().swap(r->rp);
  std::vector<int>().swap(r->ci);
  std::vector<double>().swap(r->va);
}

void release(plss_server* S, Req* r) {
  if (r->done_ev) {
    (void)hipEventSynchronize(r->done_ev);  // a single-workgroup solve may still run on this memory
    (void)hipEventDestroy(r->done_ev);
    r->done_ev = nullptr;
  }
  r->run.reset();
  if (r->M) {
    matrix_destroy(r->M);
    handle_release(S->h);
    r->M = nullptr;
  }
  if (r->slot >= 0) S->free_slots.push_back(r->slot);
  r->slot = -1;
}

// Admit queued requests that fit; returns the newly admitted ones.
std::vector<Req*> admit(plss_server* S) {
  std::vector<Req*> out;
  while (true) {
    Req* r = nullptr;
    {
      std::lock_guard<std::mutex> lk(S->mu);
      while (!S->queue.empty() && S->queue.front()->cancel) {
        Req* q = S->queue.front();
        S->queue.pop_front();
        q->state = RQ_CANCELLED;
        S->finished += 1;
        S->cv_done.notify_all();
      }
      if (S->queue.empty() || S->free_slots.empty()) break;
      Req* q = S->queue.front();
      if (S->in_use + q->resident + q->transient > S->budget) break;
      S->queue.pop_front();
      r = q;
      r->slot = S->free_slots.back();
      S->free_slots.pop_back();
      S->in_use += r->resident;
      if (S->in_use > S->peak) S->peak = S->in_use;
    }
    try {
      prepare(S, r);
      out.push_back(r);
    } catch (const InvalidArg& e) {
      r->fail = PLSS_EINVAL;
      set_error(e.msg);
    } catch (const OutOfMemory& e) {
      r->fail = PLSS_ENOMEM;
      set_error(e.msg);
    } catch (const DeviceError&) {
      r->fail = PLSS_EDEVICE;
    }
    if (r->fail != PLSS_OK) {
      release(S, r);
      std::lock_guard<std::mutex> lk(S->mu);
      S->in_use -= r->resident;
      r->state = RQ_FAILED;
      r->t_done = now_s();
      S->finished += 1;
      S->cv_done.notify_all();
    }
  }
  return out;
}

void loop(plss_server* S) {
  (void)hipSetDevice(S->h->device);
  std::vector<Req*> joining;
  bool failed = false;
  while (true) {
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv_work.wait(lk, [&] { return S->stop || !S->queue.empty() || !S->active.empty() || !joining.empty(); });
      if (S->stop && S->queue.empty() && S->active.empty() && joining.empty()) break;
    }
    try {
      if (failed) throw DeviceError();
      // systems admitted during the last chunk join now
      std::vector<Req*> more = admit(S);
      joining.insert(joining.end(), more.begin(), more.end());
      // retire cancelled ones
      bool changed = !joining.empty();
      for (Req* r : joining) {
        std::lock_guard<std::mutex> lk(S->mu);
        r->state = RQ_ACTIVE;
        S->active.push_back(r);
      }
      std::vector<Req*> joined;
      joined.swap(joining);
      std::vector<Req*> keep;
      for (Req* r : S->active) {
        if (r->cancel) {
          release(S, r);
          std::lock_guard<std::mutex> lk(S->mu);
          S->in_use -= r->resident;
          r->state = RQ_CANCELLED;
          S->finished += 1;
          S->cv_done.notify_all();
          changed = true;
        } else {
          keep.push_back(r);
        }
      }
      S->active.swap(keep);
      if (S->active.empty()) continue;
      if (changed) rebuild_lists(S);
      std::vector<Req*> joined_live;
      for (Req* r : joined)
        if (r->state == RQ_ACTIVE) joined_live.push_back(r);
      launch_joined_small(S, joined_live);
      // one chunk for every admitted system on the per-phase engine
      if (S->lists.nsys > 0) {
        const int chunk = 16;
        const int outer_every = S->lists.any_f32 ? 4 : chunk;
        S->lists.outer_seq(S->d_desc, S->main);
        for (int it = 0; it < chunk; ++it) {
          if (it > 0 && it % outer_every == 0) S->lists.outer_seq(S->d_desc, S->main);
          S->lists.iteration(S->d_desc, S->main, nullptr);
        }
        S->lists.outer_seq(S->d_desc, S->main);
      }
      PLSS_HIP(hipMemcpyAsync(S->h_slots, S->d_slots, sizeof(State) * S->max_slots, hipMemcpyDeviceToHost, S->main));
      // overlap: admit while the chunk runs
      more = admit(S);
      joining.insert(joining.end(), more.begin(), more.end());
      PLSS_HIP(hipStreamSynchronize(S->main));
      // retire finished systems
      keep.clear();
      bool retired = false;
      for (Req* r : S->active) {
        State small_st;
        const State* stp = &S->h_slots[r->slot];
        if (r->run->small) {
          // the chunk's state copy does not order after the other stream
          if (!small_finished(r)) {
            keep.push_back(r);
            continue;
          }
          PLSS_HIP(hipMemcpy(&small_st, S->d_slots + r->slot, sizeof(State), hipMemcpyDeviceToHost));
          stp = &small_st;
        }
        const State& st = *stp;
        if (!st.final_done) {
          keep.push_back(r);
          continue;
        }
        r->x.resize(r->n);
        PLSS_HIP(hipMemcpyAsync(r->x.data(), r->run->desc.xo, 8 * (size_t)r->n, hipMemcpyDeviceToHost, S->main));
        PLSS_HIP(hipStreamSynchronize(S->main));
        r->info.iters = st.k_total;
        r->info.outer_iters = st.outer;
        r->info.relres = sqrt(st.rho) * st.scale;
        r->info.relres_true = st.relres_true;
        r->info.status = st.final_status;
        release(S, r);
        std::lock_guard<std::mutex> lk(S->mu);
        S->in_use -= r->resident;
        r->t_done = now_s();
        r->info.ms = 1e3 * (r->t_done - r->t_submit);
        r->state = RQ_DONE;
        S->finished += 1;
        retired = true;
      }
      S->active.swap(keep);
      if (retired) {
        S->cv_done.notify_all();
        if (!S->active.empty()) rebuild_lists(S);
      } else if (S->lists.nsys == 0 && joining.empty()) {
        // only single-workgroup solves in flight: do not spin on their events
        std::this_thread::sleep_for(std::chrono::microseconds(100));
      }
    } catch (...) {
      // device failure: fail everything still admitted or queued
      failed = true;
      std::lock_guard<std::mutex> lk(S->mu);
      for (auto* v : {&S->active, &joining})
        for (Req* r : *v) {
          r->fail = PLSS_EDEVICE;
          r->state = RQ_FAILED;
          S->finished += 1;
        }
      S->active.clear();
      joining.clear();
      for (Req* r : S->queue) {
        r->fail = PLSS_EDEVICE;
        r->state = RQ_FAILED;
        S->finished += 1;
      }
      S->queue.clear();
      S->cv_done.notify_all();
    }
  }
}

}  // namespace

plss_server* server_create(plss_handle* h, size_t budget, int max_slots) {
  if (h->closed) throw InvalidArg{"handle destroyed"};
  plss_server* S = new plss_server();
  S->h = h;
  S->budget = budget;
  S->max_slots = max_slots;
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(h->device);
  try {
    PLSS_HIP(hipStreamCreateWithFlags(&S->main, hipStreamNonBlocking));
    PLSS_HIP(hipStreamCreateWithFlags(&S->side, hipStreamNonBlocking));
    S->d_slots = static_cast<State*>(dmalloc(sizeof(State) * max_slots));
    S->d_desc = static_cast<Desc*>(dmalloc(sizeof(Desc) * max_slots));
    PLSS_HIP(hipStreamCreateWithFlags(&S->small, hipStreamNonBlocking));
    S->d_slot_ids = static_cast<int*>(dmalloc(sizeof(int) * max_slots));
    std::vector<int> ids(max_slots);
    for (int i = 0; i < max_slots; ++i) ids[i] = i;
    PLSS_HIP(hipMemcpy(S->d_slot_ids, ids.data(), sizeof(int) * max_slots, hipMemcpyHostToDevice));
    PLSS_HIP(hipHostMalloc(reinterpret_cast<void**>(&S->h_slots), sizeof(State) * max_slots, hipHostMallocDefault));
    std::memset(S->h_slots, 0, sizeof(State) * max_slots);
  } catch (...) {
    dfree(S->d_slots);
    dfree(S->d_desc);
    dfree(S->d_slot_ids);
    if (S->h_slots) (void)hipHostFree(S->h_slots);
    if (S->main) (void)hipStreamDestroy(S->main);
    if (S->side) (void)hipStreamDestroy(S->side);
    if (S->small) (void)hipStreamDestroy(S->small);
    delete S;
    (void)hipSetDevice(prev);
    throw;
  }
  (void)hipSetDevice(prev);
  for (int i = max_slots - 1; i >= 0; --i) S->free_slots.push_back(i);
  h->refs += 1;
  S->th = std::thread(loop, S);
  return S;
}

plss_status server_submit(plss_server* S, const plss_csr* A, plss_dtype storage, const double* b,
                          const plss_opts* o, uint64_t* req) {
  if (storage != PLSS_F64 && storage != PLSS_F32) throw InvalidArg{"unknown storage"};
  if (o->sketch != PLSS_SKETCH_RESIDUAL) throw InvalidArg{"served solves use the residual sketch"};
  if (o->x0 || o->wi_diag) throw InvalidArg{"served solves take x0 = 0 and W = I"};
  validate_opts(o, storage == PLSS_F32);
  if (A->m <= 0 || A->n <= 0 || A->nnz < 0 || A->nnz >= (1LL << 31) - 1 || !A->row_ptr)
    throw InvalidArg{"bad matrix sizes"};
  std::unique_ptr<Req> r(new Req());
  r->m = A->m;
  r->n = A->n;
  r->nnz = A->nnz;
  r->rp.resize(A->m + 1);
  r->ci.resize(A->nnz);
  r->va.resize(A->nnz);
  r->b.resize(A->m);
  PLSS_HIP(hipMemcpy(r->rp.data(), A->row_ptr, sizeof(long long) * (A->m + 1), hipMemcpyDefault));
  if (A->nnz) {
    PLSS_HIP(hipMemcpy(r->ci.data(), A->col_idx, sizeof(int) * A->nnz, hipMemcpyDefault));
    PLSS_HIP(hipMemcpy(r->va.data(), A->values, sizeof(double) * A->nnz, hipMemcpyDefault));
  }
  PLSS_HIP(hipMemcpy(r->b.data(), b, sizeof(double) * A->m, hipMemcpyDefault));
  host_validate(*r);
  r->storage = storage;
  r->o = *o;
  const bool f32 = storage == PLSS_F32;
  r->resident = matrix_footprint(A->m, A->n, A->nnz, f32) + sysrun_bytes(A->m, A->n, A->nnz, f32, false);
  r->transient = csc_work_bytes((int)A->n, A->nnz) + (f32 ? 8 * (size_t)A->nnz : 0) + 8 * (size_t)(A->m + 1) + 4096;
  if (r->resident + r->transient > S->budget) throw OutOfMemory{"system larger than the server's memory budget"};
  std::lock_guard<std::mutex> lk(S->mu);
  if (S->stop) throw InvalidArg{"server is shutting down"};
  r->id = S->next_id++;
  r->t_submit = now_s();
  *req = r->id;
  Req* raw = r.release();
  S->reqs[raw->id] = raw;
  S->queue.push_back(raw);
  S->submitted += 1;
  S->cv_work.notify_all();
  return PLSS_OK;
}

plss_status server_poll(plss_server* S, uint64_t id, double* x, plss_info* info) {
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(id);
  if (it == S->reqs.end()) throw InvalidArg{"unknown or already collected request"};
  Req* r = it->second;
  if (r->state == RQ_QUEUED || r->state == RQ_ACTIVE) return PLSS_PENDING;
  plss_status ret;
  if (r->state == RQ_DONE) {
    if (x) PLSS_HIP(hipMemcpy(x, r->x.data(), 8 * (size_t)r->n, hipMemcpyDefault));
    if (info) *info = r->info;
    ret = (plss_status)r->info.status;
  } else if (r->state == RQ_CANCELLED) {
    ret = PLSS_ECANCELLED;
  } else {
    ret = r->fail;
  }
  S->reqs.erase(it);
  delete r;
  return ret;
}

plss_status server_drain(plss_server* S) {
  std::unique_lock<std::mutex> lk(S->mu);
  S->cv_done.wait(lk, [&] { return S->finished >= S->submitted; });
  return PLSS_OK;
}

plss_status server_cancel(plss_server* S, uint64_t id) {
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(id);
  if (it == S->reqs.end()) throw InvalidArg{"unknown request"};
  Req* r = it->second;
  if (r->state == RQ_QUEUED || r->state == RQ_ACTIVE) r->cancel = true;
  S->cv_work.notify_all();
  return PLSS_OK;
}

plss_status server_stats(plss_server* S, int64_t* submitted, int64_t* finished, int64_t* active, int64_t* peak) {
  std::lock_guard<std::mutex> lk(S->mu);
  if (submitted) *submitted = S->submitted;
  if (finished) *finished = S->finished;
  if (active) *active = (int64_t)S->active.size();
  if (peak) *peak = (int64_t)S->peak;
  return PLSS_OK;
}

void server_destroy(plss_server* S) {
  {
    std::lock_guard<std::mutex> lk(S->mu);
    for (Req* r : S->queue) r->cancel = true;
    for (Req* r : S->active) r->cancel = true;
    S->stop = true;
    S->cv_work.notify_all();
  }
  if (S->th.joinable()) S->th.join();
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(S->h->device);
  (void)hipStreamSynchronize(S->small);
  for (auto& kv : S->reqs) {
    release(S, kv.second);
    delete kv.second;
  }
  dfree(S->d_slots);
  dfree(S->d_desc);
  dfree(S->d_slot_ids);
  if (S->h_slots) (void)hipHostFree(S->h_slots);
  (void)hipStreamDestroy(S->main);
  (void)hipStreamDestroy(S->side);
  (void)hipStreamDestroy(S->small);
  plss_handle* h = S->h;
  delete S;
  handle_release(h);
  (void)hipSetDevice(prev);
}

}  // namespace plss
