// Device structures and launchers of the many-right-hand-side path.
#pragma once

#include "common.hpp"

namespace plss {

constexpr int kMB = 1024;      // threads per workgroup of the block products and updates
constexpr int kRB = 256;       // rows per workgroup of the block products (kMB / W in flight)
constexpr int kUE = 16 * kMB;  // block elements per workgroup of the update
constexpr int kMaxCols = 64;   // right-hand sides per block

enum MMode : int { MMODE_RESID = 0, MMODE_TRANS = 1, MMODE_REFINE = 2 };

// per-column scalars (struct of arrays); columns >= nrhs are padding and
// finished from the start
struct MState {
  double rho[kMaxCols], phi[kMaxCols], beta[kMaxCols], gamma[kMaxCols];
  double nb[kMaxCols], thr[kMaxCols], nu[kMaxCols], nb_out[kMaxCols], relres_true[kMaxCols];
  long long k[kMaxCols], k_total[kMaxCols];
  int status[kMaxCols], done[kMaxCols], fresh[kMaxCols], final_[kMaxCols], final_status[kMaxCols];
  double tol, inner_tol;
  long long maxit, outer, max_outer;
  int tol_abs;
  int all_done;
};

struct MDesc {
  const int* a_ptr;
  const int* a_idx;
  const void* a_val;
  const int* t_ptr;
  const int* t_idx;
  const void* t_val;
  int m, n;
  int s;            // block width (columns, power of two >= 8)
  int W;            // == s
  int na_blk, nt_blk, nu_blk;
  int is_f32;
  void* R;          // m x s (Vec)
  void* P;          // n x s (Vec)
  void* Y;          // n x s (Vec)
  double* X;        // n x s, solution
  double* Xi;       // n x s, inner solution (== X for float64 storage)
  const double* B;  // m x s, right-hand sides (row-major)
  double* R64;      // m x s, b - A x
  double* part_rho; // na_blk x s
  double* part_b;   // na_blk x s
  double* part_phi; // nt_blk x s
  double* part_theta;  // nu_blk x s
  MState* st;
};

void launch_spmm(int mode, bool f32, int W, const MDesc* d, int grid, hipStream_t s);
void launch_mstep(const MDesc* d, int ncols, hipStream_t s);  // ncols = MDesc::s
void launch_mouter(const MDesc* d, hipStream_t s);
void launch_mupdate(bool f32, const MDesc* d, int grid, hipStream_t s);
void launch_mstart(bool f32, const MDesc* d, int grid, hipStream_t s);
void launch_maxpy(const MDesc* d, int grid, hipStream_t s);
void launch_transpose_in(const double* src, int m, int ncols, int s, double* dst, hipStream_t st);
void launch_transpose_out(const double* src, int n, int ncols, int s, double* dst, hipStream_t st);

}  // namespace plss
