// Serving: continuous batching of independent requests (pms_stream_*).
#include <hip/hip_runtime.h>

#include "../../include/pms.h"

extern "C" {
int pms_stream_create(const pms_stream_config*, pms_stream**) { return PMS_E_UNSUPPORTED; }
int pms_stream_submit(pms_stream*, const pms_instance*, uint64_t*) { return PMS_E_UNSUPPORTED; }
int pms_stream_poll(pms_stream*, uint64_t, pms_result*) { return PMS_E_UNSUPPORTED; }
int pms_stream_wait(pms_stream*, uint64_t, pms_result*, int64_t) { return PMS_E_UNSUPPORTED; }
int pms_stream_destroy(pms_stream*) { return PMS_E_UNSUPPORTED; }
}
