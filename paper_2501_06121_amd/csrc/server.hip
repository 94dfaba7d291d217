// Continuous-batching server (placeholder until the serving loop lands).
#include <hip/hip_runtime.h>
#include "ann.h"

extern "C" {
int ann_server_create(const ann_index*, const ann_server_cfg*, ann_server**) { return ANN_EUNSUP; }
int ann_server_submit(ann_server*, const ann_request*) { return ANN_EUNSUP; }
int ann_server_poll(ann_server*, ann_completion*, int32_t) { return -ANN_EUNSUP; }
int ann_server_destroy(ann_server*) { return ANN_OK; }
}
