// Instantiations and launch of the row-marching Harris-chain kernel.
#include "rowfuse.h"

namespace fz {

template <int K, bool RGB, bool DIFF>
static hipError_t go(const RowParams& rp, hipStream_t s)
{
    const int blocks = (rp.total + ROW_WAVES - 1) / ROW_WAVES;
    const size_t lds = DIFF ? (size_t)ROW_WAVES * rp.band_h * 64 : 0;
    hipLaunchKernelGGL((k_rowfuse<K, RGB, DIFF>), dim3(blocks), dim3(ROW_WAVES * 64), lds, s, rp);
    return hipGetLastError();
}

hipError_t launch_rowfuse(const RowParams& rp, int K, bool rgb, bool diff, hipStream_t s)
{
    if (K == 2) {
        if (rgb) return diff ? go<2, true, true>(rp, s) : go<2, true, false>(rp, s);
        return diff ? go<2, false, true>(rp, s) : go<2, false, false>(rp, s);
    }
    if (K == 3) {
        if (rgb) return diff ? go<3, true, true>(rp, s) : go<3, true, false>(rp, s);
        return diff ? go<3, false, true>(rp, s) : go<3, false, false>(rp, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace fz
