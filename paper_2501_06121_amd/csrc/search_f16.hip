// Search kernels over F16 rows (every supported launch shape, beam
// list in LDS or in HBM).
#include "search_impl.h"

namespace ann {

const void* symbol_f16(const SearchParams& p) { return dense_symbol<MODE_F16>(p); }

}  // namespace ann
