// Serving loop of the posterior engine (see include/qp.h): placeholder until
// the scheduler lands; every call reports that serving is unavailable.
#include "qp.h"

extern "C" {
qp_status qp_server_create(const qp_server_config*, qp_server** s) {
    if (s) *s = nullptr;
    return QP_EDEVICE;
}
qp_status qp_server_submit(qp_server*, const uint8_t* const*, const int32_t*, int32_t, const qp_params*, float,
                           uint64_t*) {
    return QP_EINVAL;
}
qp_status qp_server_wait(qp_server*, uint64_t, int32_t, qp_result** out, qp_request_times*) {
    if (out) *out = nullptr;
    return QP_EINVAL;
}
qp_status qp_server_cancel(qp_server*, uint64_t) { return QP_EINVAL; }
qp_status qp_server_stats(qp_server*, int64_t*, int64_t*, int64_t*, int64_t*) { return QP_EINVAL; }
qp_status qp_server_destroy(qp_server*) { return QP_EINVAL; }
}
