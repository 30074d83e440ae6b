// Launch tables of the generic row-marching kernel, split over translation units.
#pragma once

#include "rowgen.h"

namespace fz {

RowGenFn lookup_rowgen_harris_lo(int a, int b);   // a in 0..2
RowGenFn lookup_rowgen_harris_mid(int a, int b);  // a in 3..5
RowGenFn lookup_rowgen_harris_hi(int a, int b);   // a in 6..8
RowGenFn lookup_rowgen_grad(int a, int b);

inline RowGenFn lookup_rowgen(int chain, int a, int b)
{
    if (chain == CHAIN_GRAD) return lookup_rowgen_grad(a, b);
    if (a <= 2) return lookup_rowgen_harris_lo(a, b);
    if (a <= 5) return lookup_rowgen_harris_mid(a, b);
    return lookup_rowgen_harris_hi(a, b);
}

template <int CH, int A, int... B>
inline RowGenFn pick_rowgen(int b, std::integer_sequence<int, B...>)
{
    static constexpr RowGenFn fns[] = {&launch_rowgen_t<CH, A, B, 2>...};
    return (b >= 0 && b < (int)sizeof...(B)) ? fns[b] : nullptr;
}

}  // namespace fz
