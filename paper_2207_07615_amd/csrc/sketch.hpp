// Identity and mixed sketches (one sketch column per step).
#pragma once
#include "runtime.hpp"
namespace plss {
void sketch_solve(plss_handle* h, const plss_matrix* A, const double* b, const plss_opts* o, double* x,
                  double* hist, long long hist_cap, plss_info* info, hipStream_t s);
void spmv_plain(const plss_matrix* A, bool transpose, const double* x, double* y, hipStream_t s);
void check_finite_inputs(const plss_matrix* A, const double* b, const plss_opts* o, hipStream_t s);
void autotune_matrix(plss_handle* h, plss_matrix* A, hipStream_t s);
// block sketches (block.cpp) and the randomized projection (randproj.cpp)
void block_solve(plss_handle* h, const plss_matrix* A, const double* b, const plss_opts* o, double* x,
                 double* hist, long long hist_cap_out, plss_info* info, hipStream_t s);
void randproj_solve(plss_handle* h, const plss_matrix* A, const double* b, const plss_opts* o, double* x,
                    double* hist, long long hist_cap_out, plss_info* info, hipStream_t s);
// plain product with its scratch in the fixed per-device array (noalloc.hip)
char* scratch_ptr(int device);
size_t spmv_noalloc_bytes(const plss_matrix* A, bool transpose, size_t* list_count);
void spmv_noalloc(plss_handle* h, const plss_matrix* A, bool transpose, const double* x, double* y,
                  hipStream_t s);
}  // namespace plss
