// Residual-sketch iteration driver (single system = batch of one).
#pragma once

#include <memory>
#include <vector>

#include "runtime.hpp"

namespace plss {

void validate_opts(const plss_opts* o, bool f32);

// Device buffers and descriptor of one system.
struct SysRun {
  const plss_matrix* A = nullptr;
  bool f32 = false;
  Desc desc{};
  State st0{};
  char* arena = nullptr;
  size_t bytes = 0;
  long long hist_len = 0;
  int u_nblk = 0;
  ~SysRun();
  void setup(const plss_matrix* M, const double* b, const plss_opts* o, long long hist_len,
             State* d_state, Desc* unused);
  void upload(const double* b, const double* x0, const double* wi, hipStream_t s);
};

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
  struct Group {
    int key;
    const int2* list;
    int n;
  };
  void build_lists(const std::vector<int>& active, hipStream_t s);
  void outer_seq(hipStream_t s);
  void iteration(hipStream_t s, hipEvent_t* ev);

  plss_handle* h_;
  std::vector<Item> items_;
  std::vector<std::unique_ptr<SysRun>> runs_;
  Desc* d_desc_ = nullptr;
  State* d_state_ = nullptr;
  State* h_state_ = nullptr;
  char* d_lists_ = nullptr;
  char* h_lists_ = nullptr;
  size_t lists_cap_ = 0;
  std::vector<Group> groups_a_, groups_t_, groups_u_, groups_af_;
  const int* d_sys_ = nullptr;
  int n_sys_ = 0;
  std::vector<hipEvent_t> events_;
  float elapsed_ms_ = 0;
};

}  // namespace plss
