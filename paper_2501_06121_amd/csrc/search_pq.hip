// Search kernels over PQ codes (asymmetric distance from LDS tables), for
// 16, 32 or 64 lanes per candidate.
#include "search_impl.h"

namespace ann {

const void* symbol_pq(const SearchParams& p) {
  switch (p.lanes_per_row) {
    case 16: return pick_kernel<PQ<16>>(p);
    case 32: return pick_kernel<PQ<32>>(p);
    case 64: return pick_kernel<PQ<64>>(p);
  }
  return nullptr;
}

}  // namespace ann
