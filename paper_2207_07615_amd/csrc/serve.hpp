// Request loop with continuous batching.
#pragma once
#include "runtime.hpp"
namespace plss {
plss_server* server_create(plss_handle* h, size_t budget, int max_slots);
plss_status server_submit(plss_server* s, const plss_csr* A, plss_dtype storage, const double* b,
                          const plss_opts* o, uint64_t* req);
plss_status server_poll(plss_server* s, uint64_t req, double* x, plss_info* info);
plss_status server_drain(plss_server* s);
plss_status server_cancel(plss_server* s, uint64_t req);
plss_status server_stats(plss_server* s, int64_t* submitted, int64_t* finished, int64_t* active,
                         int64_t* peak);
void server_destroy(plss_server* s);
}  // namespace plss
