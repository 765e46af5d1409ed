// Host-side launchers of the device kernels (kernels.hip, sketch.hip, multi.hip).
#pragma once

#include "common.hpp"

namespace plss {

// tile SpMV family; `list` holds (system, tile) pairs, n of them
void launch_spmv(int mode, bool f32, int V, const Desc* d, const int2* list, int n, int transpose,
                 hipStream_t s);
void launch_axpy_out(const Desc* d, const int2* ulist, int n, hipStream_t s);
void launch_outer(const Desc* d, const int* sys, int n, hipStream_t s);
void launch_start(bool f32, const Desc* d, const int2* alist, int n, hipStream_t s);
void launch_step(const Desc* d, const int* sys, int n, hipStream_t s);
void launch_update(bool f32, const Desc* d, const int2* ulist, int n, hipStream_t s);

// CSC (transpose) builder: device CSR (int32) -> device CSC, rows ascending in
// every column; values gathered from the float64 input and stored as f32/f64
void build_csc(const int* ptr, const int* idx, const double* vals64, int m, int n, long long nnz,
               bool f32, int* cptr, int* ridx, void* cvals, void* work, hipStream_t s);
size_t csc_work_bytes(int n, long long nnz);
void convert_vals(const double* src, long long nnz, bool f32, void* dst, hipStream_t s);
void ptr64_to_32(const long long* src, int n1, int* dst, hipStream_t s);

// one-column sketch steps (identity / mixed)
void launch_col_init(const Desc* d, const int* sys, int ns, hipStream_t s);
void launch_sketch_step(const Desc* d, int V, const int2* alist, int na, const int2* tlist, int nt,
                        const int2* ulist, int nu, const int2* wlist, int nw, const int* sys, int ns,
                        bool residual_column, int VT, const int2* cblist, int ncb, int VB, hipStream_t s);

}  // namespace plss

namespace plss {
// returns the flag bits of k_validate (0 = well formed)
int validate_csr_device(const long long* ptr, const int* idx, const double* val, int m, int n,
                        int* dflag, hipStream_t s);
}  // namespace plss

namespace plss {
void launch_check(const double* a, long long n, int positive, int* flag, hipStream_t s);
}  // namespace plss

namespace plss {
// row-blocked transpose: counts + per-block pointers, then one copy per block
void blk_build(const int* cp, const int* ri, int n, const int* d_rb, int nblk, int* d_cnt, int* d_bptr,
               void* scan_work, hipStream_t s);
void blk_copy(const int* cp, const int* ri, const void* cv, bool f32, int n, int b, const int* d_bptr, int* oi,
              void* ov, hipStream_t s);
void launch_ycomb(bool f32, const Desc* d, const int2* ulist, int n, hipStream_t s);
}  // namespace plss

namespace plss {
// striped store (stripe.hip): build steps and the product
void st_count(const int* ptr, const int* idx, int nunits, const int* d_urow, int S, int colbase, int sw, int* d_cnt,
              hipStream_t s);
void st_scatter(const int* ptr, const int* idx, const void* val, bool f32, int nunits, const int* d_urow,
                const int* d_seg, int S, int colbase, int sw, unsigned* opk, void* oval, hipStream_t s);
void st_split(const unsigned* pk, const int* d_seg, long long nseg, int* d_wsp, hipStream_t s);
void st_interleave(const unsigned* pk, const void* val, bool f32, const int* d_seg, const int* d_wsp, long long nseg,
                   int qmax, unsigned* rec, hipStream_t s);
void st_ysum(const double* ypart, int nblk, int n, double* y, hipStream_t s);
// A p from the column-block products (MODE_APB) over the CSR tile groups of alist
void launch_apcomb(const Desc* d, const int2* alist, int n, hipStream_t s);
void launch_sspmv(int mode, bool f32, const Desc* d, const int2* list, int n, int transposed, hipStream_t s);
// exclusive scan of n counts into out[0..n] (work: (n + 1023) / 1024 + 1 long longs)
void scan_counts(const int* cnt, int n, int* out, void* work, hipStream_t s);
}  // namespace plss

namespace plss {
// single-workgroup solve (small.hip): one workgroup per system in `sys`
bool small_fits(int m, int n, bool f32);
void launch_small(bool f32, const Desc* d, const int* sys, int n, hipStream_t s);
}  // namespace plss
