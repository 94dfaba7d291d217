// Search kernels over sparse rows (query terms in an LDS hash table).
#include "search_impl.h"

namespace ann {

const void* symbol_sparse(const SearchParams& p) { return pick_kernel<Sparse>(p); }

}  // namespace ann
