// Many right-hand sides on one matrix (sparse x dense block products).
#pragma once
#include "runtime.hpp"
namespace plss {
plss_status multi_solve(plss_handle* h, const plss_matrix* A, int nrhs, const double* B,
                        const plss_opts* o, double* X, plss_info* info, hipStream_t s);
}  // namespace plss
