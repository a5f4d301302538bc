// Temporary entry points for paths not yet implemented.
#include "hsd_internal.hpp"

namespace hsd {
hsd_status nufft_transform_rule(hsd_ctx *, hipStream_t, const hsd_mesh *, const hsd_mesh *,
                                const hsd_rule *, const hsd_params *, double2 *, double *)
{
    set_error("NUFFT3 method not available");
    return HSD_EINVAL;
}
} // namespace hsd

extern "C" hsd_status hsd_distance_grad(hsd_ctx *, const hsd_mesh *, const hsd_mesh *, const hsd_rule *,
                                        const hsd_params *, double *, int32_t, hsd_result *)
{
    hsd::set_error("gradient not available");
    return HSD_EINVAL;
}

extern "C" {
hsd_status hsd_server_create(hsd_ctx *, const hsd_server_cfg *, hsd_server **)
{
    hsd::set_error("server not available");
    return HSD_EINVAL;
}
hsd_status hsd_submit(hsd_server *, const hsd_request *, uint64_t *) { return HSD_EINVAL; }
hsd_status hsd_poll(hsd_server *, uint64_t, hsd_result *, hsd_request_times *) { return HSD_EINVAL; }
hsd_status hsd_wait(hsd_server *, uint64_t, double, hsd_result *, hsd_request_times *) { return HSD_EINVAL; }
hsd_status hsd_cancel(hsd_server *, uint64_t) { return HSD_EINVAL; }
hsd_status hsd_release(hsd_server *, uint64_t) { return HSD_EINVAL; }
void hsd_server_destroy(hsd_server *) {}
}
