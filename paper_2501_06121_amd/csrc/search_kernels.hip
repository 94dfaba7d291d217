// Host-side dispatch of the search kernels: kernel choice per storage mode
// and launch shape, LDS size, launch.  The kernels themselves are in
// search_impl.h, instantiated by search_<mode>.hip.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "search_kernels.h"

namespace ann {

__global__ void reset_counter_kernel(int32_t* c) { *c = 0; }

__global__ void ring_rearm_kernel(uint64_t* head, uint64_t* activity) {
  __hip_atomic_fetch_and(head, ~kRingDrain, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);  // keeps a stop
  __hip_atomic_fetch_max(activity, (uint64_t)wall_clock64(), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

void ring_rearm(const RingArgs& r, hipStream_t st) {
  hipLaunchKernelGGL(ring_rearm_kernel, dim3(1), dim3(1), 0, st, r.head, r.activity);
}

bool dense_shape_supported(int mode, int nchunks, int L) {
  if (L != 16 && L != 32 && L != 64) return false;
  const int cpl = (nchunks + L - 1) / L;
  if (L == 64) return cpl <= 4;
  if (mode == MODE_F32) return cpl <= 4;
  if (L == 32 && mode != MODE_FP8) return cpl <= 3;
  return cpl <= 2;
}

const void* kernel_symbol(const SearchParams& p) {
  switch (p.mode) {
    case MODE_F32: return symbol_f32(p);
    case MODE_F16: return symbol_f16(p);
    case MODE_BF16: return symbol_bf16(p);
    case MODE_FP8: return symbol_fp8(p);
    case MODE_PQ: return symbol_pq(p);
    case MODE_SPARSE: return symbol_sparse(p);
  }
  return nullptr;
}

hipError_t launch_search(const SearchParams& p, int slots, size_t lds, hipStream_t st) {
  const void* fn = kernel_symbol(p);
  if (!fn) return hipErrorInvalidValue;
  hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, st, p.counter);
  SearchParams arg = p;
  void* args[] = {&arg};
  const hipError_t e = hipLaunchKernel(fn, dim3(slots), dim3(64 * p.waves_per_query), args, lds, st);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

size_t lds_bytes(const SearchParams& p) {
  auto al = [](size_t b) { return (b + 15) & ~size_t(15); };
  size_t b = 0;
  b += al(p.glist ? 0 : 4 * (size_t)p.ef_cap) * 2;
  b += al(4 * 64) * 3;
  b += al(4 * (size_t)p.wbuf) * 2;
  b += al(p.glist ? 4 * (size_t)kListTailCache * p.waves_per_query : 0) * 2;
  b += al(4 * (size_t)p.q_lds_floats);
  b += al(4 * (size_t)rerank_slots(p));
  b += al(p.mode == MODE_PQ ? 4 * (size_t)p.pq_m * 256 : 0);
  b += al(p.mode == MODE_SPARSE ? 4 * kSparseHashSlots : 0) * 2;
  b += al(p.mode == MODE_SPARSE ? 8 * 64 : 0) * 2;
  b += al(4 * 16);
  return b;
}

}  // namespace ann
