// Residual-sketch iteration driver (single system = batch of one).
#pragma once

#include <memory>
#include <vector>

#include "runtime.hpp"

namespace plss {

void validate_opts(const plss_opts* o, bool f32);

// Chunks of steps between host checks.  steps_left predicts how many more
// steps a solve needs to reach its stop test sqrt(rho) <= thr from the
// decrease of ln sqrt(rho) per step since the last check (lr_prev, at step
// count steps_prev, both of the same inner solve); -1 when that is unknown
// or not a decrease.  chunk_for turns the slowest prediction into the next
// chunk: a short one exactly plus one, a long one by half (the decrease
// often speeds up as a solve goes on, and a chunk that ends early costs one
// more check, one that runs past the stop only early-exit launches), within
// [2, cap]; `unknown` when there is no prediction.
double steps_left(double rho, double thr, double steps, double lr_prev, double steps_prev);
int chunk_for(double rem, int unknown, int cap);

// Device buffers and descriptor of one system.
struct SysRun {
  const plss_matrix* A = nullptr;
  bool f32 = false;
  Desc desc{};
  State st0{};
  char* arena = nullptr;
  bool own_arena = false;
  size_t bytes = 0;
  long long hist_len = 0;
  int u_nblk = 0;
  bool use_stripes = true;  // the residual path may use the matrix's striped stores
  bool small = false;       // solved by one workgroup (single-workgroup engine)
  ~SysRun();
  // device bytes of the arena setup() lays out
  static size_t arena_bytes(const plss_matrix* M, const plss_opts* o, long long hist_len, bool use_stripes);
  // mem: arena_bytes() of device memory owned by the caller, or null (own allocation)
  void setup(const plss_matrix* M, const double* b, const plss_opts* o, long long hist_len,
             State* d_state, char* mem);
  void upload(const double* b, const double* x0, const double* wi, hipStream_t s);
};

// Launch lists of the phase kernels over a set of systems (slot, run):
// CSR groups and CSC groups keyed by (storage, tile width), update blocks
// keyed by storage, and the systems.  Row-blocked transposes get a list
// interleaved so that entry i belongs to block i mod 8 (workgroups are
// dealt to the 8 XCDs round-robin, so block b's tiles run on XCD b).
struct ListSet {
  struct Group {
    int key;
    const int2* list;
    int n;
  };
  std::vector<Group> a, t, u, af;
  std::vector<Group> sa, sb;  // striped units: products with A, block products with Aᵀ
  const int* sys = nullptr;
  int nsys = 0;
  bool any_f32 = false, any_blk = false;
  char* d = nullptr;
  char* hbuf = nullptr;
  size_t cap = 0;
  ~ListSet();
  void build(const std::vector<std::pair<int, const SysRun*>>& items, hipStream_t s);
  void outer_seq(const Desc* dd, hipStream_t s) const;
  void iteration(const Desc* dd, hipStream_t s, hipEvent_t* ev) const;
};

// Scratch reused by the calls on one handle (they are serialised by the
// handle's mutex and synchronise before returning): one device block and
// one pinned host block that only grow, the launch lists and events.
struct Workspace {
  char* dev = nullptr;
  size_t dev_cap = 0;
  char* pin = nullptr;
  size_t pin_cap = 0;
  char* hist = nullptr;  // history block of the identity/mixed sketches (P, AP and their scratch)
  size_t hist_cap = 0;
  ListSet lists;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  hipEvent_t ready = nullptr, small_done = nullptr;
  hipStream_t aux = nullptr;             // second stream: single-workgroup solves beside the phases
  std::vector<hipEvent_t> iter_events;  // 5 per timed iteration
  char* dev_block(size_t bytes);
  char* pin_block(size_t bytes);
  char* hist_block(size_t bytes);
  // One call's device memory in the blocks above: a system's arena, its
  // State and Desc, list_bytes of launch lists; and a pinned State mirror
  // (for the sketch, block and projection solves, which run one system).
  struct Call {
    char* arena;
    State* d_state;
    Desc* d_desc;
    char* lists;
    State* h_state;
  };
  Call call_block(size_t arena_bytes, size_t list_bytes);
  ~Workspace();
};
Workspace& workspace(plss_handle* h);

class BatchRunner {
 public:
  explicit BatchRunner(plss_handle* h);
  ~BatchRunner();
  void add(const plss_matrix* A, const double* b, const plss_opts* o, long long hist_len);
  void prepare(hipStream_t s);
  void run(hipStream_t s, bool timing, int chunk);
  void result(int i, double* x, double* hist, long long hist_cap, plss_info* info, hipStream_t s);
  const State& state(int i) const { return h_state_[i]; }
  float elapsed_ms() const { return elapsed_ms_; }

 private:
  struct Item {
    const plss_matrix* A;
    const double* b;
    plss_opts o;
    long long hist_len;
  };
  void build_lists(const std::vector<int>& active, hipStream_t s);

  plss_handle* h_;
  Workspace& ws_;
  std::vector<Item> items_;
  std::vector<std::unique_ptr<SysRun>> runs_;
  Desc* d_desc_ = nullptr;
  State* d_state_ = nullptr;
  int* d_small_ = nullptr;  // systems of the single-workgroup engine (float64 first, then float32)
  State* h_state_ = nullptr;
  int* h_small_ = nullptr;
  bool aux_used_ = false;  // work was enqueued on the workspace's second stream
  float elapsed_ms_ = 0;
};

}  // namespace plss
