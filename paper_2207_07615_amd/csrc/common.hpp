// Shared definitions of the PLSS GPU library (gfx950 / CDNA4).
//
// Device-side layout:
//  * A is held twice: CSR (rows of A) and CSC (rows of Aᵀ), int32 pointers
//    and indices, values in float64 or float32 storage.
//  * Each direction carries a table of wave tiles: tile t covers rows
//    [tile[t], tile[t+1]) with at most 64*V stored entries and at most that
//    many rows, or exactly one row when that row alone is longer.  Four
//    wave tiles of similar cost form a group, the unit of one workgroup:
//    long-row tiles are grouped by length, short tiles in row order.
//  * Per system, a Desc (plain pointers) and a State (scalars of the
//    iteration) live in device memory; a launch of any phase kernel walks a
//    list of (system, tile) pairs, so one launch serves one system or many.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

namespace plss {

constexpr int kWG = 256;           // threads per workgroup (4 wave64)
constexpr int kWaves = kWG / 64;

// statuses stored in State::status (mirror plss_status of the C ABI)
constexpr int ST_OK = 0;
constexpr int ST_NOT_CONVERGED = 1;
constexpr int ST_BREAKDOWN = 2;

enum SpmvMode : int {
  MODE_RESID = 0,   // r <- r - A p ; partial rho = sum r^2              (Alg. 1 r update, rho)
  MODE_TRANS = 1,   // y <- Aᵀ r   ; partial phi = sum y^2 / wi         (Alg. 1 y, phi)
  MODE_REFINE = 2,  // out <- b - A x (float64) ; partial sum out^2, sum b^2
  MODE_PLAIN = 3,   // out <- A x (float64 in/out)
  MODE_AP = 4,      // ap <- A p ; r <- r - ap ; partial rho          (Section 7 storage of A p)
  MODE_TRANSB = 5,  // ypart[b] <- A_bᵀ r_b for row block b (XCD-local gather of r)
  MODE_APB = 6,     // appart[b] <- A_b p for column block b (XCD-local gather of p; Section 7 A p)
};

constexpr int kMaxBlk = 8;         // row blocks of the transposed store (one per XCD)

// Striped store (stripe.hip): a work unit keeps its row sums in LDS while the
// gathered vector passes through LDS in stripes; kSThreads threads per unit.
// Stores of A: stripes of 6144 columns, units of at most 8192 rows (float64:
// 2 x 48 KB of stripes + 64 KB of row sums, all of the 160 KB of LDS; fewer,
// wider stripes cut the fixed cost per stripe).  Row-block stores of Aᵀ:
// stripes of 2048, units of at most 16384 rows, so that the product with Aᵀ
// runs one unit per CU (2 x 16 KB + 128 KB).  A stripe width need not be a
// power of two: an entry keeps its column inside the stripe in 16 bits.
constexpr int kSWA = 6144, kRBA = 8192;
constexpr int kSWT = 2048, kRBT = 16384;
// Float32 row-block stores of Aᵀ: the row sums of a 16384-row unit take
// 64 KB, so the stripes can be 8192 wide (2 x 32 KB): four times fewer
// stripes, and their fixed costs, than at 2048.  The plain product, which
// accumulates in float64, runs on the CSC tiles for these stores.
constexpr int kSWT32 = 8192;
// Float32 stores of A: the unit's row sums take 32 KB, so the stripes of the
// float32 kernel can be as wide as kSWA32 (2 x 48 KB at 12288).
constexpr int kSWA32 = 6144;
inline int swa(bool f32) { return f32 ? kSWA32 : kSWA; }
inline int swt(bool f32) { return f32 ? kSWT32 : kSWT; }
constexpr int kSThreads = 1024;
// most entries per lane in one window of a wave range (a window holds up to
// 64 x this many entries); at the large shapes a wave's range in a stripe of
// A averages about 410 entries, one of Aᵀ about 270 (eight for A measured
// slower than seven, though fewer ranges then take a second window).
constexpr int kQmaxA = 7, kQmaxT = 6;
// the same for float32 stores (an entry takes two registers instead of three)
constexpr int kQmaxA32 = 7, kQmaxT32 = 6;
inline int qa(bool f32) { return f32 ? kQmaxA32 : kQmaxA; }
inline int qt(bool f32) { return f32 ? kQmaxT32 : kQmaxT; }
constexpr int kMaxStripes = 8192;  // stripes per store (cursor table of the builder in LDS)
constexpr size_t kSmallLds = 156 * 1024;  // LDS for r, p, y of a single-workgroup solve
constexpr long long kSmallNnz = 1 << 18;  // automatic single-workgroup solves up to this many entries
constexpr int kStorePad = 64;      // records allocated past the end of a striped store: a
                                   // float32 window's last slot is loaded by every lane

// Entry records of a striped store, in 32-bit words: a float64 value in
// words 0-1 and the packed (row in unit) << 16 | (column in stripe) in word
// 2; a float32 value in word 0 and the packed word in word 1.  One load
// instruction per lane brings a whole entry.
constexpr int rec_words(bool f32) { return f32 ? 2 : 3; }

struct StripeView {
  const unsigned* rec;         // entry records (rec_words per entry)
  const int* urow;             // nunits + 1 row starts of the units
  const int* seg;              // nunits * S + 1 entry starts of the (unit, stripe) segments
  const int* wsp;              // 16 row-aligned wave starts per segment
  int nunits, S;
  int colbase, ncols;          // columns [colbase, colbase + ncols) of the gathered vector
  int sw;                      // stripe width (kSWA, kSWA32, kSWT or kSWT32)
};

struct State {
  // Algorithm 1 scalars (float64 always)
  double rho, phi, theta, beta, gamma;
  double nb, thr, scale;       // inner right-hand side norm, stop threshold, history scale
  // refinement (outer) scalars
  double nu;                   // norm of the current outer residual (1 when unrefined)
  double nb_out;               // ||b||
  double tol_out;              // outer tolerance (relative unless tol_abs)
  double inner_tol;
  double relres_true;
  long long k;                 // updates applied in the current inner solve
  long long k_total;           // updates applied over all inner solves
  long long maxit;             // bound on k_total
  long long outer, max_outer;
  int status;                  // inner status when done
  int done;                    // inner solve finished
  int final_status;
  int final_done;              // whole solve finished (x final, relres_true set)
  int fresh;                   // next update is the first of an inner solve
  int tol_abs;
  double tol;                  // requested tolerance (inner when unrefined)
  // one-column sketch steps (identity / mixed)
  long long kh;                // stored history columns
  long long col;               // sketch columns examined
  long long hist_cap;          // history capacity
  long long max_cols;          // bound on sketch columns examined (skips included)
  int skip;                    // current column skipped
  int col_kind;                // 0 residual column, 1 identity column
  int row;                     // identity row of the current column
  int prev_row;                // row scattered into the dense scratch (-1 none)
  double sigma, delta;
};

struct Desc {
  // CSR of A
  const int* a_ptr;
  const int* a_idx;
  const void* a_val;
  const int* a_tile;           // row start of every wave tile (a_nwt + 1)
  const int* a_grp;            // 4 wave tiles per group (-1 = none), a_ntiles groups
  const int4* a_wtd;           // per (group, wave): {first row, end row, first entry, end entry}
  int a_nwt;                   // wave tiles
  int a_ntiles;                // groups of 4 wave tiles (one workgroup, one partial each)
  // CSC of A (= CSR of Aᵀ)
  const int* t_ptr;
  const int* t_idx;
  const void* t_val;
  const int* t_tile;
  const int* t_grp;
  const int4* t_wtd;
  int t_nwt;
  int t_ntiles;
  int m, n;
  // rows of more than 64 entries of the CSR and the CSC (single-workgroup solve)
  const int* a_long;
  const int* t_long;
  int a_nlong, t_nlong;
  const int* a_sl_base;
  const int* a_sl_idx;
  const void* a_sl_val;
  const int* t_sl_base;
  const int* t_sl_idx;
  const void* t_sl_val;
  int u_nblk;                  // blocks of the vector-update kernel
  // row-blocked CSC: block b holds the entries of rows [rb[b], rb[b+1])
  int nblk;                    // 1: products with Aᵀ use the CSC above
  const int* tb_ptr[kMaxBlk];
  const int* tb_idx[kMaxBlk];
  const void* tb_val[kMaxBlk];
  const int* tb_tile[kMaxBlk];
  const int* tb_grp[kMaxBlk];
  const int4* tb_wtd[kMaxBlk];
  void* ypart;                 // nblk x n block products (Vec)
  // column-blocked CSR: block b holds the entries of columns [cb[b], cb[b+1])
  int cnblk;                   // 1: products with A use the CSR above
  const int* cb_ptr[kMaxBlk];
  const int* cb_idx[kMaxBlk];
  const void* cb_val[kMaxBlk];
  const int* cb_tile[kMaxBlk];
  const int* cb_grp[kMaxBlk];
  const int4* cb_wtd[kMaxBlk];
  double* appart;              // cnblk x m block products of A p (identity / mixed sketches)
  int phi_cnt;                 // partials of phi (t_ntiles, or u_nblk when blocked)
  // striped stores (used instead of the tiles when set)
  int a_striped;               // products with A (r update, refinement residual)
  int t_striped;               // block products with Aᵀ (needs nblk > 1)
  int rho_cnt;                 // partials of rho and ||b||^2 (a_ntiles, or sa.nunits)
  StripeView sa;
  StripeView sb[kMaxBlk];
  // iteration vectors (Vec = double for float64 storage, float for float32)
  void* r;                     // m
  void* p;                     // n
  void* y;                     // n
  double* x;                   // n, inner solution (== xo when unrefined)
  double* xo;                  // n, solution
  const double* b;             // m
  void* c;                     // m, inner right-hand side (float32 mode) or null
  double* r64;                 // m, float64 residual b - A x
  const double* wi;            // n, diagonal of BᵀB or null (W = I)
  // partial sums, one per tile / block
  double* part_rho;            // a_ntiles
  double* part_b;              // a_ntiles
  double* part_phi;            // t_ntiles
  double* part_theta;          // u_nblk
  double* hist;
  long long hist_len;
  State* st;
  // one-column sketch state
  double* P;                   // n x cap, column-major
  double* AP;                  // m x cap, column-major
  double* Th;                  // cap
  double* cv;                  // cap, c = w / Θ
  double* part_w;              // cap x wblk, partial (AP)ᵀ r
  int wblk;                    // blocks of the (AP)ᵀ r kernel
  double* dense;               // n, scratch holding one row of A as a dense vector
  const int* perm;             // m, identity-sketch row order
  int sketch;                  // 0 residual, 1 identity, 2 mixed
  int is_f32;
};

inline int tile_nnz(int V) { return 64 * V; }

// thread-local error text of the C ABI
void set_error(const std::string& s);

}  // namespace plss

#define PLSS_HIP(call)                                                            \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess) {                                                       \
      ::plss::set_error(std::string(#call) + ": " + hipGetErrorString(e_));       \
      throw ::plss::DeviceError();                                                \
    }                                                                             \
  } while (0)

namespace plss {
struct DeviceError {};
struct InvalidArg {
  std::string msg;
};
struct OutOfMemory {
  std::string msg;
};
}  // namespace plss
