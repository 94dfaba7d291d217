// Search kernels over FP8 rows (every supported launch shape, beam
// list in LDS or in HBM).
#include "search_impl.h"

namespace ann {

const void* symbol_fp8(const SearchParams& p) { return dense_symbol<MODE_FP8>(p); }

}  // namespace ann
