/* Drives the oracle under the sanitizers: the fixed chain on small RGB and
 * gray volumes (with frame sizes down to one pixel), the generic chains
 * frame by frame and stage by stage (IIR, stencils over several frames), and
 * the tracker on seeded points.  Any sanitizer report aborts the run. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int or_chain(const int32_t* ops, int32_t n, const double* in, int32_t C, int32_t W, int32_t H, int32_t T, double* out,
             int32_t cout, double sigma, double k, double thr, double* pts, int64_t cap, int64_t* npts,
             int32_t nthreads);
int or_gchain(const int32_t* kind, const int32_t* rx, const int32_t* ry, const int32_t* pk, const double* pa,
              const double* pb, const double* w, int32_t n, const double* in, int32_t W, int32_t H, int32_t T,
              double* out, int32_t nthreads);
int or_gchain_seq(const int32_t* kind, const int32_t* rx, const int32_t* ry, const int32_t* rt, const int32_t* pk,
                  const double* pa, const double* pb, const double* w, int32_t n, const double* in, int32_t W,
                  int32_t H, int32_t T, double* out);
int64_t or_track(const int32_t* pts, int64_t n_pts, int32_t T, double q, double r, double gate, int32_t max_miss,
                 double v0, int32_t* out_i, double* out_d, int64_t cap);

static double urand(void) { return (double)rand() / RAND_MAX; }

int main(void)
{
    srand(11);
    const int sizes[][3] = {{37, 23, 4}, {1, 1, 2}, {3, 2, 3}, {64, 9, 2}};
    int fails = 0;
    for (int s = 0; s < 4; ++s) {
        const int W = sizes[s][0], H = sizes[s][1], T = sizes[s][2];
        const size_t P = (size_t)W * H * T;
        double* rgb = malloc(sizeof(double) * 3 * P);
        double* out = malloc(sizeof(double) * 3 * P);
        double* pts = malloc(sizeof(double) * 4 * 4096);
        for (size_t i = 0; i < 3 * P; ++i) rgb[i] = floor(urand() * 256.0);
        const int32_t ops[] = {1, 2, 3, 5, 6, 7, 8, 9, 10};
        int64_t np = 0;
        fails += or_chain(ops, 9, rgb, 3, W, H, T, out, 1, 1.0, 0.04, 1e3, pts, 4096, &np, 2) != 0;
        const int32_t grad[] = {2, 3, 4};
        fails += or_chain(grad, 3, rgb, 1, W, H, T, out, 1, 1.0, 0.04, 1e8, pts, 4096, &np, 1) != 0;
        /* generic: stencil 3x3, point sqrt|v|, box 2x1, affine */
        int32_t kind[] = {1, 0, 2, 0}, rx[] = {1, 0, 2, 0}, ry[] = {1, 0, 1, 0}, pk[] = {0, 3, 0, 0};
        double pa[] = {0, 0, 0, 0.5}, pb[] = {0, 0, 0, 2.0}, w[9];
        for (int q = 0; q < 9; ++q) w[q] = urand() - 0.5;
        fails += or_gchain(kind, rx, ry, pk, pa, pb, w, 4, rgb, W, H, T, out, 2) != 0;
        /* temporal: IIR, stencil over 3 frames, box */
        int32_t tk[] = {3, 1, 2}, trx[] = {0, 1, 1}, try_[] = {0, 1, 1}, trt[] = {0, 2, 0}, tpk[] = {0, 0, 0};
        double tpa[] = {0.3, 0, 0}, tpb[] = {0, 0, 0}, tw[27];
        for (int q = 0; q < 27; ++q) tw[q] = urand() / 27.0;
        fails += or_gchain_seq(tk, trx, try_, trt, tpk, tpa, tpb, tw, 3, rgb, W, H, T, out) != 0;
        free(rgb);
        free(out);
        free(pts);
    }
    /* tracker: 20 moving points over 50 frames, some dropping out */
    int32_t tp[3 * 1000];
    int n = 0;
    for (int t = 0; t < 50; ++t)
        for (int k = 0; k < 20; ++k) {
            if ((t + k) % 7 == 0) continue;
            tp[3 * n] = t;
            tp[3 * n + 1] = 10 + 13 * k + (t % 3);
            tp[3 * n + 2] = 5 + 2 * t + k;
            ++n;
        }
    int32_t* oi = malloc(sizeof(int32_t) * 3 * 8192);
    double* od = malloc(sizeof(double) * 4 * 8192);
    const int64_t m = or_track(tp, n, 50, 0.5, 1.0, 9.21, 3, 4.0, oi, od, 8192);
    fails += m <= 0 || m > 8192;
    free(oi);
    free(od);
    printf(fails ? "FAILED\n" : "ok\n");
    return fails ? 1 : 0;
}
