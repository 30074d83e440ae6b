// Generic row-marching kernel instantiations: Harris chain, groups starting at stage 6..8.
#include "tables_rowgen.h"

namespace fz {
RowGenFn lookup_rowgen_harris_hi(int a, int b)
{
    using S = std::make_integer_sequence<int, 9>;
    switch (a) {
    case 6: return pick_rowgen<CHAIN_HARRIS, 6>(b, S{});
    case 7: return pick_rowgen<CHAIN_HARRIS, 7>(b, S{});
    case 8: return pick_rowgen<CHAIN_HARRIS, 8>(b, S{});
    default: return nullptr;
    }
}
}  // namespace fz
