// Generic row-marching kernel instantiations: Harris chain, groups starting at stage 0..2.
#include "tables_rowgen.h"

namespace fz {
RowGenFn lookup_rowgen_harris_lo(int a, int b)
{
    using S = std::make_integer_sequence<int, 9>;
    switch (a) {
    case 0: return pick_rowgen<CHAIN_HARRIS, 0>(b, S{});
    case 1: return pick_rowgen<CHAIN_HARRIS, 1>(b, S{});
    case 2: return pick_rowgen<CHAIN_HARRIS, 2>(b, S{});
    default: return nullptr;
    }
}
}  // namespace fz
