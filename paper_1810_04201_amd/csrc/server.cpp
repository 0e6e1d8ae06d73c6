// Continuous-batching solve server (placeholder until the scheduler lands).
#include "runtime.hpp"

using namespace wd;

extern "C" {

int wd_server_create(const wd_server_config *, wd_server **) {
    return fail(WD_ERR_STATE, "server not available in this build");
}
int wd_submit(wd_server *, wd_lattice *, const wd_solve_params *, const double *, double *,
              uint64_t *) {
    return fail(WD_ERR_STATE, "server not available in this build");
}
int wd_poll(wd_server *, uint64_t, wd_solve_info *) {
    return fail(WD_ERR_STATE, "server not available in this build");
}
int wd_server_stats(wd_server *, double *, double *, double *) {
    return fail(WD_ERR_STATE, "server not available in this build");
}
int wd_server_peak_bytes(wd_server *, size_t *) {
    return fail(WD_ERR_STATE, "server not available in this build");
}
int wd_server_destroy(wd_server *) {
    return fail(WD_ERR_STATE, "server not available in this build");
}

}  // extern "C"
