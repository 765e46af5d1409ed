// Block sketches: a block of sketch columns appended per step (identity rows,
// or the residual followed by identity rows).  Device layout and launchers.
#pragma once

#include "common.hpp"

namespace plss {

constexpr int kBW = 16;       // most columns per block (one MFMA output tile)
constexpr int kBHist = 1024;  // most history columns

// Scalars of a block solve (device memory), beside the Algorithm-1 State
// that carries rho, the stop test, counts and the final status.
struct BlkState {
  long long pos;        // position of the next row in the pass through the row order
  long long nblk;       // history blocks held
  long long K;          // history columns held
  long long steps;      // blocks examined (skipped ones included)
  long long max_steps;  // bound on blocks examined
  long long cap;        // history capacity in columns
  int nrow;             // identity rows of the current block
  int wk;               // kept columns of the current block
  int res_kept;         // the residual column (first) is kept
  int pass_end;         // the current block ends a pass through the rows
  int skip;             // the current block keeps no column (no update)
  int pad;
  int rows[kBW];        // rows of the kept identity columns (compacted, after the residual)
  double cp[kBW];       // Delta^{-1} sigma on the kept columns
};

// History: the projected blocks Z_j = Y_j - Z_{<j} C (n x w_j each) side by
// side as columns of one row-major n x kcap matrix, A Z_j likewise (m x kcap),
// and per block its column offset, width and the lower Cholesky factor of
// Delta_j = Z_jᵀ Z_j.  Blocks are mutually orthogonal, so the projection on
// the span of the history is sum_j Z_j Delta_j^{-1} Z_jᵀ.
struct BlkDesc {
  double* Zh;           // n x kcap
  double* AZh;          // m x kcap
  double* Lh;           // kBHist x kBW x kBW factors
  int* bo;              // column offset of each block
  int* wh;              // kept columns of each block
  double* Ug;           // kcap x kBW: W, then L^{-1} W (block-diagonal L)
  double* Cg;           // kcap x kBW projection coefficients C = Delta^{-1} W
  double* part_w;       // kcap x wblk partial (A Z)ᵀ r
  double* part_r;       // partial rho of the block product, one per workgroup
  const int* perm;      // row order (m)
  BlkState* bs;
  int kcap;             // row stride of Zh and AZh (capacity, at least one block, rounded up to 4)
  int wblk;             // row chunks of the (A Z)ᵀ r kernel
  int nparts;           // workgroups of the block product
  int block;            // identity rows per step
  int residual;         // residual column first
  int lpr;              // lanes per row of the block product (4, 8 or 16)
};

constexpr int kBRows = 1024;  // rows per workgroup of the (A Z)ᵀ r kernel

void launch_block_step(const Desc* d, const BlkDesc* bd, bool residual, int lpr, int VT, const int2* tlist,
                       int nt, int n, int wblk, int nparts, hipStream_t s);

}  // namespace plss
