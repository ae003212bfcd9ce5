// Serving entry points (continuous batching).  Filled in by the serving scheduler.
#include "veg_internal.h"

extern "C" {
veg_status veg_serve_create(const veg_serve_config*, veg_server**) { return VEG_ERR_INVALID_ARG; }
veg_status veg_serve_add_model(veg_server*, const veg_gaussians*, int32_t*) { return VEG_ERR_INVALID_ARG; }
veg_status veg_serve_submit(veg_server*, const veg_request*, uint64_t*) { return VEG_ERR_INVALID_ARG; }
veg_status veg_serve_poll(veg_server*, uint64_t, int32_t*) { return VEG_ERR_INVALID_ARG; }
veg_status veg_serve_wait(veg_server*, uint64_t, int32_t) { return VEG_ERR_INVALID_ARG; }
veg_status veg_serve_stats_get(veg_server*, veg_serve_stats*) { return VEG_ERR_INVALID_ARG; }
veg_status veg_serve_stats_reset(veg_server*) { return VEG_ERR_INVALID_ARG; }
veg_status veg_serve_destroy(veg_server*) { return VEG_ERR_INVALID_ARG; }
}
