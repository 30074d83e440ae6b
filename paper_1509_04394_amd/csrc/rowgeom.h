// Geometry of the row-marching kernel, shared by the planner and the launcher.
#pragma once

#include <algorithm>

#include "fz_ops.h"

namespace fz {

constexpr int ROW_HX = 6;     // horizontal and vertical halo of the chain: 2 + 1 + 2 + 1
constexpr int ROW_WAVES = 4;  // independent wavefronts per workgroup
// Wavefronts per SIMD of the Harris row kernel, as its registers allow (512
// per lane, allocated in blocks of 8): two columns per lane take <= 85
// registers with RGB input (5 waves) and <= 80 with gray input (6 waves),
// three columns <= 128 (4 waves).
inline int row_waves(int K, bool rgb) { return K == 3 ? 4 : (rgb ? 5 : 6); }
// Wavefronts the 256 CUs (4 SIMDs each) hold at once; 4 per SIMD is assumed
// for the generic row kernel.
inline int row_slots(int K, bool rgb) { return 256 * 4 * row_waves(K, rgb); }
constexpr int ROW_SLOTS_GENERIC = 256 * 4 * 4;

// Groups the row kernel implements: gray conversion or Gaussian first, suppression
// or frame difference last, of the Harris chain.
inline bool row_group(int ch, int A, int B) { return ch == CHAIN_HARRIS && (A == 0 || A == 1) && (B == 7 || B == 8); }

// Strips of 64*K columns that overlap by 2*halo cover a frame of width W.
inline int row_strips(int W, int K, int halo = ROW_HX)
{
    const int span = 64 * K, S = span - 2 * halo;
    if (W < span) return 0;
    return 1 + (W - span + S - 1) / S;
}

// Groups the generic row kernel implements: any group with a window stage
// (one column per lane pair, K = 2).
inline bool rowgen_group(int ch, int A, int B) { return group_has_window(ch, A, B); }

// Columns per lane (2 or 3): the choice that computes the fewest columns per
// wavefront the SIMDs can hold; 0 if the frame is narrower than 128 columns.
inline int row_strips_best(int W, bool rgb)
{
    const int n2 = row_strips(W, 2), n3 = row_strips(W, 3);
    if (n2 == 0) return 0;
    if (n3 > 0 && n3 * 192 * row_waves(2, rgb) < n2 * 128 * row_waves(3, rgb)) return 3;
    return 2;
}

inline int row_lds_bytes(int band_h) { return ROW_WAVES * band_h * 64; }

// Frame boundaries between consecutive runs of one strip and band, and the
// device bytes of their exchange (two areas of band_h * K mask words and one
// counter each, 256-byte aligned), for a frame-difference row group.
FZ_HD inline int row_boundaries(int nstrips, int nbands, int nchunks)
{
    return nchunks > 1 ? nstrips * nbands * (nchunks - 1) : 0;
}
inline size_t row_exchange_bytes(int nstrips, int nbands, int nchunks, int band_h, int K)
{
    const size_t nb = (size_t)row_boundaries(nstrips, nbands, nchunks);
    const size_t words = ((2 * nb * band_h * K * 8) + 255) & ~(size_t)255;
    return nb == 0 ? 0 : words + ((nb * 4 + 255) & ~(size_t)255);
}

// A frame-difference group keeps one byte of previous-frame mask bits per lane
// and row in LDS: at most 256 rows per band keep that within 64 KB per
// workgroup of ROW_WAVES wavefronts.
constexpr int ROW_DIFF_MAX_BAND = 256;

// Rows per band and frames per work item.  A work item marches band_h + 2*HX
// rows per frame over tt frames (a frame-difference group takes the frame
// before them from the previous run's item, which costs about 0.45 of a
// frame per item); `slots` wavefronts run at once, fewer when the frame
// difference's LDS rows (one workgroup of ROW_WAVES wavefronts per SIMD slot)
// do not fit 160 KB per CU that many times.  The cost of a pair is its total
// work, items x (band_h + 2*HX) x (tt + exchange), times (1 + 1/r) for r =
// items / (wavefronts at once): a launch of few rounds of long items loses
// the tail of its last round, and on the 800x600x1000 RGB chain measured
// times fall from ~1.27 ms at 0.95 rounds (55 rows x 16 frames) to ~1.11 ms
// at 5-8 rounds (55-86 rows x 2 frames); and times slots / (wavefronts at
// once) where LDS holds fewer wavefronts than the registers allow.
// Explicit requests (> 0)
// are kept as given, except that a frame run longer than the video is the
// whole video and a band taller than the frame the whole frame; a request the
// kernel cannot run (a band over ROW_DIFF_MAX_BAND rows on a frame-difference
// group) gives band_h = 0 and is refused by the caller, never replaced.
struct RowShape {
    int band_h, tt;
};
inline RowShape row_shape(int H, int T, int nstrips, bool diff, int req_h, int req_tt, int slots)
{
    if (req_h > 0 && diff && std::min(req_h, H) > ROW_DIFF_MAX_BAND) return RowShape{0, 0};
    RowShape best{0, 0};
    double best_cost = -1.0;
    const int tts[] = {1, 2, 4, 8, 16, 32, 64};
    for (int tt : tts) {
        int t = tt;
        if (req_tt > 0) {
            if (tt != 1) break;
            t = std::min(req_tt, T);
        } else if ((!diff && t != 1) || (t > T && t != 1)) {
            continue;
        }
        for (int nb = 1; nb <= H; ++nb) {
            const int bh = req_h > 0 ? std::min(req_h, H) : (H + nb - 1) / nb;
            if (diff && bh > ROW_DIFF_MAX_BAND) continue;
            if (bh < 16 && req_h <= 0 && nb > 1) break;
            const long long items = (long long)nstrips * ((H + bh - 1) / bh) * ((T + t - 1) / t);
            long long fit = slots;
            if (diff) fit = std::min(fit, (long long)256 * ROW_WAVES * (163840 / row_lds_bytes(bh)));
            const double r = (double)items / (double)fit;
            const double cost = (double)items * (bh + 2 * ROW_HX) * (t + (diff && t < T ? 0.45 : 0.0)) *
                                (1.0 + 1.0 / r) * ((double)slots / (double)fit);
            if (best_cost < 0 || cost < best_cost) {
                best_cost = cost;
                best = RowShape{bh, t};
            }
            if (req_h > 0) break;
        }
    }
    return best;
}

}  // namespace fz
