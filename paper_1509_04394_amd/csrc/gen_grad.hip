// Generic row-marching kernel instantiations: gradient-magnitude chain.
#include "tables_rowgen.h"

namespace fz {
RowGenFn lookup_rowgen_grad(int a, int b)
{
    using S = std::make_integer_sequence<int, 3>;
    switch (a) {
    case 0: return pick_rowgen<CHAIN_GRAD, 0>(b, S{});
    case 1: return pick_rowgen<CHAIN_GRAD, 1>(b, S{});
    case 2: return pick_rowgen<CHAIN_GRAD, 2>(b, S{});
    default: return nullptr;
    }
}
}  // namespace fz
