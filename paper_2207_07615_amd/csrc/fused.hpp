// The fused residual pair (fused.hip): both products of one iteration in one
// pass over the CSR store, with a two-level fixed-order sum for y.
#pragma once

#include "common.hpp"

struct plss_handle;
struct plss_matrix;

namespace plss {

// most workgroups of a fused launch (16 rows or columns each at a time); the
// grid depends only on the row / column count, so sums are reproducible
constexpr int kFzMaxGrid = 4096;
int fz_grid(long long rows);

// CSR position of every CSC slot (n columns; cptr / ridx the CSC of A)
void launch_fz_pos(const int* aptr, const int* aidx, const int* cptr, const int* ridx, int n, int* pos,
                   hipStream_t s);

// workgroups of the long-row kernel (0 without long rows)
int fz_long_grid(int nlong);

// r <- r - A p (m rows; lrows lists the nlong rows of more than 64 entries,
// ascending), c_e = a_e r_i, y = Aᵀ r (n columns), out2 = {||r||², ||y||²};
// part holds fz_grid(m) + fz_long_grid(nlong) + fz_grid(n) doubles
void launch_fz_pair(bool f32, const int* ptr, const int* idx, const void* val, int m, const int* lrows,
                    int nlong, const int* cptr, const int* pos, int n, const double* p, double* r, double* c,
                    double* y, double* part, double* out2, hipStream_t s);

// The whole call on a handle (builds the position map on first use):
// r <- r - A p, y = Aᵀ r; out2 (host, may be null) = {||r||², ||y||²}.
// p, r, y: host or device memory, not overlapping.
void residual_pair(plss_handle* h, plss_matrix* A, const double* p, double* r, double* y, double* out2,
                   hipStream_t s);

}  // namespace plss
