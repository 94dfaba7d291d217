// Search kernels over PQ codes (asymmetric distance from LDS tables).
#include "search_impl.h"

namespace ann {

const void* symbol_pq(const SearchParams& p) { return pick_kernel<PQ>(p); }

}  // namespace ann
