// Brute-force k-NN on matrix cores (placeholder until the MFMA tiles land).
#include <hip/hip_runtime.h>
#include "ann.h"
#include "search_kernels.h"

extern "C" int ann_bruteforce(const ann_index*, const float*, int64_t, int32_t, int64_t*, float*,
                              void*) {
  return ANN_EUNSUP;
}
