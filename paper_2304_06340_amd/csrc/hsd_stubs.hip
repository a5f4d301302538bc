// Temporary entry points for paths not yet implemented.
#include "hsd_internal.hpp"



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
