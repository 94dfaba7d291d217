// Search kernels over BF16 rows (every supported launch shape, beam
// list in LDS or in HBM).
#include "search_impl.h"

namespace ann {

const void* symbol_bf16(const SearchParams& p) { return dense_symbol<MODE_BF16>(p); }

}  // namespace ann
