// Lane-interleaved windows of a striped store (shared by the striped
// product kernels).
//
// A wave walks a row-aligned range of entries in windows of at most 64 * Q
// entries (Q <= QM per lane; QM is fixed per store: kQmaxA for stores of A,
// kQmaxT for the row-block stores of Aᵀ).  In a window of c entries, lanes
// below r = c - 64 (Qw - 1) hold Qw = ceil(c / 64) consecutive entries (in
// CSR order) and the others Qw - 1; the window is stored lane-interleaved,
// the lane's k-th entry at window start + 64 k + lane.  Each entry is a
// record of a value and a packed (row << 16 | column) word.
#pragma once

#include "common.hpp"
#include "wave.hpp"

namespace plss {


// Segmented scan over the 64 lanes of (f, v), where a set flag starts a new
// segment after the element: incl_j = f_j ? v_j : incl_{j-1} + v_j.  Returns
// incl_{j-1} (0 in lane 0); incl_63 goes to out63.  Shifts by 1, 2, 4, 8
// inside rows of 16 lanes, then row 0's last lane into row 1 (and row 2's
// into row 3), then lane 31 into rows 2 and 3.
template <class T>
__device__ __forceinline__ T wseg_excl(int f, T v, T& out63) {
  T sv = v;
  int sf = f;
#define PLSS_SEG_STEP(CTRL, RM, BC)              \
  {                                              \
    const T ov = dppv<CTRL, RM, BC>(sv);         \
    const int of = dpp32<CTRL, RM, BC>(sf);      \
    if (!sf) sv = ov + sv;                       \
    sf |= of;                                    \
  }
  PLSS_SEG_STEP(kRowShr1, 0xF, true)
  PLSS_SEG_STEP(kRowShr2, 0xF, true)
  PLSS_SEG_STEP(kRowShr4, 0xF, true)
  PLSS_SEG_STEP(kRowShr8, 0xF, true)
  PLSS_SEG_STEP(kRowBcast15, 0xA, false)
  PLSS_SEG_STEP(kRowBcast31, 0xC, false)
#undef PLSS_SEG_STEP
  out63 = lane63(sv);
  return dppv<kWaveShr1, 0xF, true>(sv);
}

// s_acc[i] += v.  Each row has a single writer per stripe (wave ranges and
// lane runs are row-aligned, or carried to the lane that ends the row), so
// the result is the plain sum in a fixed order either way.  For float64 the
// LDS atomic add does the read-modify-write in one instruction and measured
// faster than a separate read and write; for float32 the atomic add measured
// twice as slow on this access pattern, so float sums use the plain form.
__device__ __forceinline__ void lds_add(double* p, double v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_add(float* p, float v) { *p += v; }

// Entries per lane in a window of c entries: Qw = ceil(c / 64) for lanes
// below r = c - 64 (Qw - 1), Qw - 1 for the others.
__device__ __forceinline__ int win_count(int c, int lane) {
  const int Qw = (c + 63) >> 6;
  return lane < c - 64 * (Qw - 1) ? Qw : Qw - 1;
}

// wave range [ws, we): windows of 64 * Q entries, the last one shorter
__host__ __device__ __forceinline__ int range_q(int len, int qmax) {
  const int Q = (len + 63) >> 6;
  return Q > qmax ? qmax : (Q < 1 ? 1 : Q);
}

// One entry record in registers: (value, packed word) loaded by one
// instruction and taken apart where it is used.
template <class Val> struct EntOf;
template <> struct EntOf<double> { using type = u32x3; };
template <> struct EntOf<float> { using type = u32x2; };
template <class Val> using Ent = typename EntOf<Val>::type;
__device__ __forceinline__ unsigned ent_pk(u32x3 e) { return e.z; }
__device__ __forceinline__ unsigned ent_pk(u32x2 e) { return e.y; }
__device__ __forceinline__ double ent_val(u32x3 e) {
  return __builtin_bit_cast(double, ((unsigned long long)e.y << 32) | e.x);
}
__device__ __forceinline__ float ent_val(u32x2 e) { return __builtin_bit_cast(float, e.x); }

// One lane-interleaved window of c entries into registers (the lane's
// entries in CSR order), one record load per entry; a slot without an entry
// holds row 0xFFFF, column 0 and value 0 (its product reads a valid slot of
// the slice and is never used).  Float values: every lane
// loads all Qw = ceil(c / 64) slots, so the loads depend on wave-uniform
// values only; a lane without an entry in the last slot reads one of the 63
// records past the window (the store has kStorePad records of padding past
// its end) and never uses it.  Double values: only the lane's own slots are
// loaded (the uniform form needs more registers than the double kernel has
// to spare).
template <class Val, int QM>
__device__ __forceinline__ void load_window(const unsigned* __restrict__ rec, int base, int c, Ent<Val>* e) {
  const int lane = threadIdx.x & 63;
  if constexpr (sizeof(Val) == 4) {
    const int Qw = (c + 63) >> 6;
    const unsigned* wp = rec + 2 * (size_t)(base + lane);
#pragma unroll
    for (int q = 0; q < QM; ++q) e[q] = q < Qw ? gload_nt2(wp + 128 * q) : u32x2{0u, 0xFFFF0000u};
  } else {
    const int mine = c > 0 ? win_count(c, lane) : 0;
    const unsigned* wp = rec + 3 * (size_t)(base + lane);
#pragma unroll
    for (int q = 0; q < QM; ++q) e[q] = q < mine ? gload_nt3(wp + 192 * q) : u32x3{0u, 0u, 0xFFFF0000u};
  }
}

// Row sums of one window of c > 0 entries of a wave range, added to s_acc.
// The run that is open at the window's end (the last lane's final run,
// with the carries of the lanes before it) is not written here: it goes out
// in (wc, wr) = (partial sum, row), and the next window of the range adds it
// to its first run if that run continues the row, or writes it first if
// not; after the range's last window the caller writes it (flush_open).
// No global load is needed to find where that run ends.  On entry wr = -1
// if nothing is carried.
//
// Float sums (no LDS atomic add: see lds_add) batch the window's run ends:
// every slot's row sum is read first, then all are written, so the wave
// waits for LDS once per window instead of once per slot.  The rows a
// window ends are distinct, so the reads see no write of the same window.
// A slot without a run end reads and writes the lane's spare word
// s_acc[RB + lane] instead (the kernel's s_acc has RB + 64 words).
template <class Val, class Acc, int QM, int RB>
__device__ __forceinline__ void sum_window(int c, const Ent<Val>* e, const Acc* __restrict__ xs, Acc* s_acc,
                                           Acc& wc, int& wr) {
  constexpr bool kBatch = sizeof(Acc) == 4;
  const int lane = threadIdx.x & 63;
  const int Qw = (c + 63) >> 6, r = c - 64 * (Qw - 1);
  const int mine = lane < r ? Qw : Qw - 1;
  const int last = Qw > 1 ? 63 : r - 1;  // last lane holding entries (lanes 0..last do)
  // row of the entry after this lane's last one, for lanes before `last`
  unsigned pv[QM];
  Val vv[QM];
#pragma unroll
  for (int q = 0; q < QM; ++q) {
    pv[q] = ent_pk(e[q]);
    vv[q] = ent_val(e[q]);
  }
  const int frow = mine > 0 ? (int)(pv[0] >> 16) : -1;
  const int nrow = dpp32<kWaveShl1, 0xF, true>(frow);
  const int frow0 = __builtin_amdgcn_readfirstlane(frow);
  if (wr >= 0 && wr != frow0) {  // the carried run ended at the window boundary
    if (lane == 0) lds_add(&s_acc[wr], wc);
    wr = -1;
  }
  int cur = -1, fr = 0;
  bool hend = false;
  Acc acc = Acc(0), fv = Acc(0);
  // all gathers of the window first (back to back in LDS); a slot without an
  // entry reads a valid address and its product is never used
  Acc prods[QM];
#pragma unroll
  for (int q = 0; q < QM; ++q) prods[q] = Acc(vv[q]) * xs[pv[q] & 0xFFFFu];
  // slots past the lane's entries leave the state unchanged (selects, so the
  // wave runs the slots without branching)
  int wrow[QM];  // batched run ends: row (or the spare word) and sum
  Acc wval[QM];
#pragma unroll
  for (int q = 0; q < QM; ++q) {
    const bool act = q < mine;
    const int rr = (int)(pv[q] >> 16);
    const bool brk = act && rr != cur;
    const bool ended = brk && cur >= 0;  // the run of `cur` ends before this entry
    if constexpr (kBatch) {
      wrow[q] = (ended && hend) ? cur : RB + lane;
      wval[q] = acc;
    } else {
      if (ended && hend) lds_add(&s_acc[cur], acc);
    }
    const bool first = ended && !hend;   // the lane's first run end waits for the carry
    fv = first ? acc : fv;
    fr = first ? cur : fr;
    hend = hend || ended;
    const Acc sum = acc + prods[q];
    acc = brk ? prods[q] : (act ? sum : acc);
    cur = act ? rr : cur;
  }
  if constexpr (kBatch) {
    Acc old[QM];
#pragma unroll
    for (int q = 0; q < QM; ++q) old[q] = s_acc[wrow[q]];
#pragma unroll
    for (int q = 0; q < QM; ++q) s_acc[wrow[q]] = old[q] + wval[q];
  }
  if (lane < last && nrow != cur) {  // the lane's final run ends inside the window
    if (!hend) {
      hend = true;
      fr = cur;
      fv = acc;
    } else {
      lds_add(&s_acc[cur], acc);
    }
    acc = Acc(0);
  }
  if (lane == 0 && wr >= 0) {
    if (hend) fv = wc + fv;
    else acc = wc + acc;
  }
  Acc out63;
  const Acc carry = wseg_excl<Acc>(hend ? 1 : 0, acc, out63);
  if (hend) lds_add(&s_acc[fr], fv + carry);
  wc = out63;
  wr = __builtin_amdgcn_readlane(cur, last);
}

// Writes the run left open by a wave range's last window.
template <class Acc>
__device__ __forceinline__ void flush_open(Acc* s_acc, Acc wc, int wr) {
  if (wr >= 0 && (threadIdx.x & 63) == 0) lds_add(&s_acc[wr], wc);
}

}  // namespace plss
