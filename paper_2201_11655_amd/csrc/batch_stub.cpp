// Placeholder entry points, replaced by the batched and serving implementations.
#include "vdmc_internal.h"

extern "C" {
vdmc_status vdmc_count_batch(const vdmc_graph*, int32_t, int32_t, uint64_t* const*, void*) {
    return vdmc::guarded([] { throw vdmc::Error{VDMC_ERR_UNSUPPORTED, "not built yet"}; });
}
vdmc_status vdmc_tune(const vdmc_graph*, int32_t, int32_t, const char*) {
    return vdmc::guarded([] { throw vdmc::Error{VDMC_ERR_UNSUPPORTED, "not built yet"}; });
}
vdmc_status vdmc_serve_create(const vdmc_serve_config*, vdmc_server*) {
    return vdmc::guarded([] { throw vdmc::Error{VDMC_ERR_UNSUPPORTED, "not built yet"}; });
}
vdmc_status vdmc_serve_submit(vdmc_server, vdmc_graph, int32_t, uint64_t*, uint64_t*) {
    return vdmc::guarded([] { throw vdmc::Error{VDMC_ERR_UNSUPPORTED, "not built yet"}; });
}
vdmc_status vdmc_serve_poll(vdmc_server, uint64_t, int32_t*) {
    return vdmc::guarded([] { throw vdmc::Error{VDMC_ERR_UNSUPPORTED, "not built yet"}; });
}
vdmc_status vdmc_serve_wait(vdmc_server, uint64_t, int64_t) {
    return vdmc::guarded([] { throw vdmc::Error{VDMC_ERR_UNSUPPORTED, "not built yet"}; });
}
vdmc_status vdmc_serve_stats(vdmc_server, double*, double*, double*, uint64_t*) {
    return vdmc::guarded([] { throw vdmc::Error{VDMC_ERR_UNSUPPORTED, "not built yet"}; });
}
vdmc_status vdmc_serve_destroy(vdmc_server) {
    return vdmc::guarded([] { throw vdmc::Error{VDMC_ERR_UNSUPPORTED, "not built yet"}; });
}
}
