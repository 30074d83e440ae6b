// Generic row-marching kernel instantiations: Harris chain, groups starting at stage 3..5.
#include "tables_rowgen.h"

namespace fz {
RowGenFn lookup_rowgen_harris_mid(int a, int b)
{
    using S = std::make_integer_sequence<int, 9>;
    switch (a) {
    case 3: return pick_rowgen<CHAIN_HARRIS, 3>(b, S{});
    case 4: return pick_rowgen<CHAIN_HARRIS, 4>(b, S{});
    case 5: return pick_rowgen<CHAIN_HARRIS, 5>(b, S{});
    default: return nullptr;
    }
}
}  // namespace fz
