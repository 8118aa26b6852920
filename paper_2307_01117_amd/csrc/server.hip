// server.hip -- serving form (continuous batching).  Placeholder until the
// scheduler lands: every entry point reports HEAT_EINVAL.
#include "heat_internal.h"

using namespace heat;

extern "C" {
int heat_server_create(size_t, int32_t, int32_t, heat_server **out) {
    if (out) *out = nullptr;
    return fail(HEAT_EINVAL, "server not available in this build");
}
int heat_submit(heat_server *, heat_problem *, uint64_t *) { return fail(HEAT_EINVAL, "no server"); }
int heat_poll(heat_server *, uint64_t) { return fail(HEAT_ENOENT, "no server"); }
int heat_wait(heat_server *, uint64_t) { return fail(HEAT_ENOENT, "no server"); }
int heat_cancel(heat_server *, uint64_t) { return fail(HEAT_ENOENT, "no server"); }
int heat_server_get_stats(heat_server *, heat_server_stats *) { return fail(HEAT_EINVAL, "no server"); }
int heat_server_destroy(heat_server *) { return HEAT_OK; }
}
