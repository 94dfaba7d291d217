// Search kernels over F32 rows (every supported launch shape, beam
// list in LDS or in HBM).
#include "search_impl.h"

namespace ann {

const void* symbol_f32(const SearchParams& p) { return dense_symbol<MODE_F32>(p); }

}  // namespace ann
