// Launch tables of the compiled chains, split over several translation units
// so they compile in parallel.
#pragma once

#include "engine.h"

namespace fz {

// Launch function of group [a..b] of the Harris chain / gradient chain.
LaunchFn lookup_harris_lo(int a, int b);  // a in 0..2
LaunchFn lookup_harris_mid(int a, int b); // a in 3..5
LaunchFn lookup_harris_hi(int a, int b);  // a in 6..8
LaunchFn lookup_grad(int a, int b);

inline LaunchFn lookup(int chain, int a, int b)
{
    if (chain == CHAIN_GRAD) return lookup_grad(a, b);
    if (a <= 2) return lookup_harris_lo(a, b);
    if (a <= 5) return lookup_harris_mid(a, b);
    return lookup_harris_hi(a, b);
}

template <int CH, int A, int... B>
inline LaunchFn pick_row(int b, std::integer_sequence<int, B...>)
{
    static constexpr LaunchFn fns[] = {&launch_group<CH, A, B>...};
    return (b >= 0 && b < (int)sizeof...(B)) ? fns[b] : nullptr;
}

}  // namespace fz
