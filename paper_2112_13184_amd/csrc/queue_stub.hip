// placeholder, replaced by the serving queue
#include "../../include/ctm.h"
extern "C" {
ctm_status ctm_queue_create(size_t, int, ctm_queue** out) { if (out) *out = nullptr; return CTM_EINVAL; }
ctm_status ctm_queue_submit(ctm_queue*, const ctm_request*, uint64_t*) { return CTM_EINVAL; }
ctm_status ctm_queue_poll(ctm_queue*, uint64_t, ctm_result*) { return CTM_EINVAL; }
ctm_status ctm_queue_wait(ctm_queue*, uint64_t, int, ctm_result*) { return CTM_EINVAL; }
ctm_status ctm_queue_cancel(ctm_queue*, uint64_t) { return CTM_EINVAL; }
void ctm_queue_destroy(ctm_queue*) {}
}
