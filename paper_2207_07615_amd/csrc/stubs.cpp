// Entry points still to be written.
#include "multi.hpp"
#include "serve.hpp"
#include "sketch.hpp"
namespace plss {
plss_server* server_create(plss_handle*, size_t, int) { throw InvalidArg{"server not built yet"}; }
plss_status server_submit(plss_server*, const plss_csr*, plss_dtype, const double*, const plss_opts*,
                          uint64_t*) {
  throw InvalidArg{"server not built yet"};
}
plss_status server_poll(plss_server*, uint64_t, double*, plss_info*) { throw InvalidArg{"no server"}; }
plss_status server_drain(plss_server*) { throw InvalidArg{"no server"}; }
plss_status server_cancel(plss_server*, uint64_t) { throw InvalidArg{"no server"}; }
plss_status server_stats(plss_server*, int64_t*, int64_t*, int64_t*, int64_t*) {
  throw InvalidArg{"no server"};
}
void server_destroy(plss_server*) {}
}  // namespace plss
