// Lane-interleaved windows of a striped store (shared by the striped and
// single-workgroup kernels).
//
// A wave walks a row-aligned range of entries in windows of at most 64 * Q
// entries (Q <= kQmax per lane).  In a window of c entries, lanes below
// r = c - 64 (Qw - 1) hold Qw = ceil(c / 64) consecutive entries (in CSR
// order) and the others Qw - 1; the window is stored lane-interleaved, the
// lane's k-th entry at window start + 64 k + lane.  Each entry is a packed
// (row << 16 | column) word and a value.
#pragma once

#include "common.hpp"
#include "wave.hpp"

namespace plss {

constexpr int kQmax = 6;  // entries per lane of one window

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
__device__ __forceinline__ int range_q(int len) {
  const int Q = (len + 63) >> 6;
  return Q > kQmax ? kQmax : (Q < 1 ? 1 : Q);
}

// One lane-interleaved window of c entries into registers (the lane's
// entries in CSR order).  Float values: every lane loads all Qw =
// ceil(c / 64) slots, so the loads depend on wave-uniform values only and
// share one address; a lane without an entry in the last slot reads one of
// the 63 entries past the window (the store has kStorePad entries of padding
// past its end) and never uses it.  Double values: only the lane's own
// slots are loaded (the uniform form needs more registers than the double
// kernel has to spare, and measured 1-2 % slower there).
template <class Val>
__device__ __forceinline__ void load_window(const unsigned* __restrict__ pk, const Val* __restrict__ val, int base,
                                            int c, unsigned* pv, Val* vv) {
  const int lane = threadIdx.x & 63;
  if constexpr (sizeof(Val) == 4) {
    const int Qw = (c + 63) >> 6;
    const unsigned* pp = pk + base + lane;
    const Val* vp = val + base + lane;
#pragma unroll
    for (int q = 0; q < kQmax; ++q) {
      if (q < Qw) {
        pv[q] = gload_nt(pp + 64 * q);
        vv[q] = gload_nt(vp + 64 * q);
      } else {
        pv[q] = 0xFFFFFFFFu;
        vv[q] = Val(0);
      }
    }
  } else {
    const int mine = c > 0 ? win_count(c, lane) : 0;
#pragma unroll
    for (int q = 0; q < kQmax; ++q) {
      if (q < mine) {
        pv[q] = gload_nt(&pk[base + 64 * q + lane]);
        vv[q] = gload_nt(&val[base + 64 * q + lane]);
      } else {
        pv[q] = 0xFFFFFFFFu;
        vv[q] = Val(0);
      }
    }
  }
}

// Row sums of one window [base, wend) of a wave range ending at we, added
// to s_acc.  wc: open row sum carried in from the previous window, and out
// to the next one.
template <int SW, class Val, class Acc>
__device__ __forceinline__ void sum_window(const unsigned* __restrict__ pk, int base, int wend, int we,
                                           const unsigned* pv, const Val* vv, const Acc* __restrict__ xs,
                                           Acc* s_acc, Acc& wc) {
  const int lane = threadIdx.x & 63;
  const int c = wend - base;
  const int Qw = (c + 63) >> 6, r = c - 64 * (Qw - 1);
  const int mine = lane < r ? Qw : Qw - 1;
  const int next_has = (lane + 1 < r ? Qw : Qw - 1) > 0;
  const int last = Qw > 1 ? 63 : r - 1;  // last lane holding entries
  // row of the entry after this lane's last one (-1: the range ends there)
  const int frow = mine > 0 ? (int)(pv[0] >> 16) : -1;
  const int nb = dpp32<kWaveShl1, 0xF, true>(frow);
  int nrow = -1;
  if (lane < 63 && next_has) nrow = nb;
  else if (lane == last && wend < we) nrow = (int)(gload_nt(&pk[wend]) >> 16);
  int cur = -1, fr = 0;
  bool hend = false;
  Acc acc = Acc(0), fv = Acc(0);
  // all gathers of the window first (back to back in LDS); a slot without an
  // entry reads a valid address and its product is never used
  Acc prods[kQmax];
#pragma unroll
  for (int q = 0; q < kQmax; ++q) prods[q] = Acc(vv[q]) * xs[pv[q] & (SW - 1)];
  // slots past the lane's entries leave the state unchanged (selects, so the
  // wave runs the slots without branching)
#pragma unroll
  for (int q = 0; q < kQmax; ++q) {
    const bool act = q < mine;
    const int rr = (int)(pv[q] >> 16);
    const bool brk = act && rr != cur;
    const bool ended = brk && cur >= 0;  // the run of `cur` ends before this entry
    if (ended && hend) lds_add(&s_acc[cur], acc);
    const bool first = ended && !hend;   // the lane's first run end waits for the carry
    fv = first ? acc : fv;
    fr = first ? cur : fr;
    hend = hend || ended;
    const Acc sum = acc + prods[q];
    acc = brk ? prods[q] : (act ? sum : acc);
    cur = act ? rr : cur;
  }
  if (cur >= 0 && nrow != cur) {
    if (!hend) {
      hend = true;
      fr = cur;
      fv = acc;
    } else {
      lds_add(&s_acc[cur], acc);
    }
    acc = Acc(0);
  }
  if (lane == 0) {
    if (hend) fv = wc + fv;
    else acc = wc + acc;
  }
  Acc out63;
  const Acc carry = wseg_excl<Acc>(hend ? 1 : 0, acc, out63);
  if (hend) lds_add(&s_acc[fr], fv + carry);
  wc = out63;
}

}  // namespace plss
