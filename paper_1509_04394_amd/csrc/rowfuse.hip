// Instantiations and launches of the row-marching Harris-chain kernels.
#include "rowfuse.h"

namespace fz {

// Zero the queue counter and every clip's point count (a kernel, so that the
// reset is an ordinary kernel node when the batch is captured into a graph).
__global__ void k_batch_reset(BatchParams bp)
{
    const int i = threadIdx.x;
    if (i == 0) *bp.queue = 0u;
    if (i < bp.n_clips && bp.clip[i].count != nullptr) *bp.clip[i].count = 0u;
}

// Zero n words (the frame-boundary arrival counters; a kernel, not a memset,
// so that it is an ordinary kernel node when a run is captured into a graph).
__global__ void k_zero_words(uint32_t* p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

template <int K, bool RGB, bool DIFF>
static hipError_t go(const RowParams& rp, hipStream_t s)
{
    const int blocks = (rp.total + ROW_WAVES - 1) / ROW_WAVES;
    const size_t lds = DIFF ? (size_t)ROW_WAVES * rp.band_h * 64 : 0;
    if (DIFF && rp.xcount != nullptr) {
        const int nb = row_boundaries(rp.nstrips, rp.nbands, rp.nchunks);
        if (nb > 0) {
            hipLaunchKernelGGL(k_zero_words, dim3((nb + 255) / 256), dim3(256), 0, s, rp.xcount, nb);
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
    }
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

template <int K, bool RGB, bool DIFF>
static hipError_t go_batch(const BatchParams& bp, int blocks, hipStream_t s)
{
    const size_t lds = DIFF ? (size_t)ROW_WAVES * BATCH_BAND_H * 64 : 0;
    hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, s, bp);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_rowfuse_batch<K, RGB, DIFF>), dim3(blocks), dim3(ROW_WAVES * 64), lds, s, bp);
    return hipGetLastError();
}

hipError_t launch_rowfuse_batch(const BatchParams& bp, int K, bool rgb, bool diff, int blocks, hipStream_t s)
{
    if (K != 2) return hipErrorInvalidValue;
    if (rgb) return diff ? go_batch<2, true, true>(bp, blocks, s) : go_batch<2, true, false>(bp, blocks, s);
    return diff ? go_batch<2, false, true>(bp, blocks, s) : go_batch<2, false, false>(bp, blocks, s);
}

template <int K, bool RGB, bool DIFF>
static int occ()
{
    int n = 0;
    const size_t lds = DIFF ? (size_t)ROW_WAVES * BATCH_BAND_H * 64 : 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_rowfuse_batch<K, RGB, DIFF>, ROW_WAVES * 64, lds) !=
        hipSuccess)
        return 0;
    return n;
}

int rowfuse_batch_blocks_per_cu(int K, bool rgb, bool diff)
{
    if (K != 2) return 0;
    if (rgb) return diff ? occ<2, true, true>() : occ<2, true, false>();
    return diff ? occ<2, false, true>() : occ<2, false, false>();
}

}  // namespace fz
