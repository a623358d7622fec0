// Serving entry points (continuous batching of polar requests).
#include "la_internal.h"

extern "C" {

la_status la_serve_create(la_context *, const la_serve_config *, void *, size_t, la_server **out)
{
    if (out)
        *out = nullptr;
    la::set_error("la_serve_create: serving is not available in this build");
    return LA_ERR_DEVICE;
}

la_status la_serve_submit(la_server *, int64_t, int64_t, const float *, int64_t,
                          const la_polar_opts *, uint64_t *)
{
    la::set_error("la_serve_submit: no server");
    return LA_ERR_INVALID_ARG;
}

la_status la_serve_poll(la_server *, uint64_t, float *, float *, la_polar_info *, la_status *)
{
    la::set_error("la_serve_poll: no server");
    return LA_ERR_INVALID_ARG;
}

la_status la_serve_stats_get(la_server *, la_serve_stats *)
{
    la::set_error("la_serve_stats_get: no server");
    return LA_ERR_INVALID_ARG;
}

la_status la_serve_destroy(la_server *) { return LA_OK; }

}  // extern "C"
