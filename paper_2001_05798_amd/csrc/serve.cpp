// Serving queue (continuous batching of flow + travel-time requests).
// Placeholder entry points until the scheduler lands.
#include "gw_internal.h"

struct gw_queue {
    int dummy;
};

extern "C" {

int queue_create(size_t, int32_t, gw_queue **q) {
    if (q) *q = nullptr;
    gw::set_last_error("queue: not implemented");
    return GW_EINVAL;
}
double queue_clock(const gw_queue *) { return 0.0; }
int queue_submit(gw_queue *, const gw_request *, uint64_t *) {
    gw::set_last_error("queue: not implemented");
    return GW_EINVAL;
}
int queue_poll(gw_queue *, uint64_t, gw_result *) {
    gw::set_last_error("queue: not implemented");
    return GW_EINVAL;
}
int queue_drain(gw_queue *) { return GW_OK; }
void queue_destroy(gw_queue *) {}

}  // extern "C"
