// Library-internal objects behind the opaque handles of plss.h.
#pragma once

#include <atomic>
#include <mutex>
#include <vector>

#include "../../include/plss.h"
#include "common.hpp"
#include "kernels.hpp"

// One direction of the matrix store: CSR of A, or CSR of Aᵀ (= CSC of A).
struct PlssDir {
  int nrows = 0, ncols = 0;
  int* ptr = nullptr;    // nrows + 1
  int* idx = nullptr;    // nnz
  void* val = nullptr;   // nnz, f64 or f32
  int* tile = nullptr;   // nwt + 1 row starts of the wave tiles
  int* grp = nullptr;    // 4 * ntiles wave-tile ids (-1 = none)
  int4* wtd = nullptr;   // 4 * ntiles: each wave's tile as {first row, end row, first entry, end entry} (zeros: none)
  int nwt = 0;           // wave tiles
  int ntiles = 0;        // groups of 4 wave tiles (workgroups per launch)
  int V = 8;             // entries per lane of a wave tile (64*V entries)
  int* lrows = nullptr;  // rows of more than 64 entries (single-workgroup solve)
  // slice layout for the single-workgroup solve: slice s (rows 64 s .. 64 s + 63)
  // starts at sl_base[s]; entry k of its row 64 s + l is at
  // sl_base[s] + (k / 4) * 256 + 4 l + k % 4 (rows of at most 64 entries)
  int* sl_base = nullptr;
  int* sl_idx = nullptr;
  void* sl_val = nullptr;
  long long sl_n = 0;     // entries of the slice layout, padding included
  int nlong = 0;
  std::vector<int> h_ptr;  // host copy of ptr (tile construction)
};

// A striped store of one direction (stripe.hip): units of unit_rows rows (or
// balanced by entry count), stripes of sw columns of the gathered vector.
struct PlssStripes {
  unsigned* rec = nullptr; // nnz + kStorePad entry records (rec_words each)
  int* urow = nullptr;     // nunits + 1
  int* seg = nullptr;      // nunits * S + 1
  int* wsp = nullptr;      // nunits * S * 16
  int nunits = 0, S = 0, colbase = 0, ncols = 0, unit_rows = 0, sw = 0;
  bool balanced = false;   // units balanced by entry count (at most ceil(rows / unit_rows) of them)
  long long nnz = 0;
  size_t bytes = 0;
};

namespace plss {
struct Workspace;
void workspace_free(Workspace* w);
}  // namespace plss

struct plss_handle {
  int device = 0;
  hipStream_t stream = nullptr;
  std::mutex mu;
  // matrices and servers created on the handle keep it alive: plss_destroy
  // only frees it once the last of them is destroyed
  std::atomic<int> refs{0};
  bool closed = false;
  double kt_ms[4] = {0, 0, 0, 0};
  long long kt_n[4] = {0, 0, 0, 0};
  plss::Workspace* ws = nullptr;  // scratch of the calls on this handle (solve.cpp)
};

struct plss_matrix {
  plss_handle* h = nullptr;
  long long m = 0, n = 0, nnz = 0;
  bool f32 = false;
  PlssDir A, T;
  // row-blocked copy of the transpose (one block per XCD) for the product
  // with Aᵀ when r does not fit one XCD's L2; nblk = 1 means none
  int nblk = 1;
  int rb[plss::kMaxBlk + 1] = {0};
  PlssDir TB[plss::kMaxBlk];
  int* tb_ptr_all = nullptr;   // nblk x (n+1) pointers shared by the blocks
  // column-blocked copy of A (one block of columns per XCD) for the products
  // with A whose gathered vector does not fit one XCD's L2 (the identity and
  // mixed sketches' A p); built on first use, cnblk = 1 means none
  int cnblk = 1;
  int cbnd[plss::kMaxBlk + 1] = {0};
  PlssDir CB[plss::kMaxBlk];
  int* cb_ptr_all = nullptr;   // cnblk x (m+1) pointers shared by the blocks
  // fused residual pair: the CSR position of every CSC slot and the per-entry
  // contributions a_ij r_i (float64); built on first use
  int* fz_pos = nullptr;
  double* fz_c = nullptr;
  // striped stores: SA for products with A, SB[b] for row block b of Aᵀ
  bool a_striped = false, t_striped = false;
  PlssStripes SA;
  PlssStripes SB[plss::kMaxBlk];
  size_t base_bytes = 0;       // bytes of the CSR, CSC and row-blocked stores
  size_t bytes = 0;
};

namespace plss {

// device allocation that reports ENOMEM through an exception
void* dmalloc(size_t bytes);
void dfree(void* p);

// tile table of a pointer array for tiles of 256*V entries
std::vector<int> make_tiles(const std::vector<int>& ptr, int V);
std::vector<int> make_groups(const std::vector<int>& ptr, const std::vector<int>& tiles, int V);
void set_tiles(PlssDir& d, int V, hipStream_t s);
void set_long_rows(PlssDir& d, hipStream_t s);
// slice layout of a direction for the single-workgroup solve (runtime.cpp)
void set_slices(PlssDir& d, bool f32, hipStream_t s);

// validated store creation (throws InvalidArg / OutOfMemory / DeviceError)
plss_matrix* matrix_create(plss_handle* h, const plss_csr* A, plss_dtype storage, hipStream_t s);
void matrix_destroy(plss_matrix* A);
void handle_release(plss_handle* h);  // drop one reference; frees a closed handle at zero
void build_row_blocks(plss_matrix* M, hipStream_t s, bool force = false);
// Column blocks of A, when the gathered vector of a product with A (n
// float64 entries) exceeds about 3 MB; a no-op once built or when it fits.
void build_col_blocks(plss_matrix* M, hipStream_t s);
// Position map and contribution buffer of the fused residual pair (12 bytes
// per entry); a no-op once built.
void build_fused(plss_matrix* M, hipStream_t s);
size_t matrix_footprint(long long m, long long n, long long nnz, bool f32);

// Striped layout: build or drop the stores (unit_rows 0 = from the shape).
void matrix_set_layout(plss_matrix* M, bool a_stripes, bool t_stripes, int unit_rows, hipStream_t s);
// Layout chosen from the shape at creation.
void auto_layout(long long m, long long n, long long nnz, bool f32, bool* a_stripes, bool* t_stripes);
int auto_unit_rows(long long rows, int nblk, int rbmax);
std::vector<int> unit_starts(const std::vector<int>& ptr, int rows, int R, int cap, bool balance);
void fill_stripe_view(const PlssStripes& st, StripeView* v);

}  // namespace plss
