/*
 * CPU reference ("oracle") for the video kernel chain -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may call
 * this code.  It shares nothing with the GPU library: its own op codes, its own
 * weights, its own border handling, its own loops.
 *
 * What it computes (Sec. III): the chain I_out = K_n(...K_1(I_in)), each kernel
 * applied in sequence to the whole output of the previous one, here frame by
 * frame, unfused, in double precision.  Every window stage reads its input with
 * replicate (clamp-to-edge) borders on that stage's own input.
 *
 * Op codes (oracle-private):
 *   1 rgb2gray   point op (Table II row 1)      3 planes -> 1
 *   2 gauss5     5x5 sampled Gaussian, sigma     1 -> 1   (rectangular, Table II)
 *   3 sobel3     3x3 gradient Ix, Iy             1 -> 2   (rectangular, Table II)
 *   4 gradmag    sqrt(Ix^2 + Iy^2)               2 -> 1
 *   5 products   Ix^2, Ix*Iy, Iy^2               2 -> 3
 *   6 boxsum5    unweighted 5x5 window sums      c -> c
 *   7 harris     Sxx*Syy - Sxy^2 - k (Sxx+Syy)^2 3 -> 1
 *   8 threshold  R >= thr ? R : 0                1 -> 1   (Table III Threshold uses >=)
 *   9 nms3       255 iff v > 0 and v >= its 3x3 neighbours, else 0; emits points
 *  10 framediff  |m[t] - m[max(t-1,0)]|          1 -> 1   (multi-frame, Table I)
 *
 * Generic single-channel stages (or_gchain): the three access classes of
 * Table I with free parameters -- a point operation (affine, absolute value,
 * square, square root of the absolute value, clamp), a weighted
 * (2rx+1) x (2ry+1) stencil and an unweighted (2rx+1) x (2ry+1) window sum.
 *
 * Temporal generic stages (or_gchain_seq): an IIR filter (Table II, a
 * multi-frame point operation) and a stencil with a frame window (Table I,
 * spatio-temporal operation).
 *
 * Parity status of each function: pinned by tests/test_oracle.py and, for the
 * generic stages, tests/test_generic_oracle.py and tests/test_temporal_oracle.py
 * (closed forms, invariants, library routines, brute force); see the module
 * docstrings there.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum {
    OR_RGB2GRAY = 1, OR_GAUSS5 = 2, OR_SOBEL3 = 3, OR_GRADMAG = 4, OR_PRODUCTS = 5,
    OR_BOXSUM5 = 6, OR_HARRIS = 7, OR_THRESHOLD = 8, OR_NMS3 = 9, OR_FRAMEDIFF = 10
};

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* Pixel (x, y) of a W x H plane with replicate borders. */
static double px(const double* p, int W, int H, int x, int y)
{
    return p[(size_t)clampi(y, 0, H - 1) * W + clampi(x, 0, W - 1)];
}

/* Table II "Convert RGBA to Gray", a point operation.  Integer BT.601 luma
 * with round-half-up; exact in double because every term is an integer. */
void or_rgb2gray(const double* r, const double* g, const double* b, double* out, int W, int H)
{
    for (size_t i = 0; i < (size_t)W * H; ++i)
        out[i] = floor((299.0 * r[i] + 587.0 * g[i] + 114.0 * b[i] + 500.0) / 1000.0);
}

/* Table II "Gaussian Smooth Filter", a rectangular operation: the plain 2-D
 * 25-tap sum with normalised sampled weights exp(-i^2 / (2 sigma^2)). */
void or_gauss5(const double* in, double* out, int W, int H, double sigma)
{
    double w[5], s = 0.0;
    for (int i = -2; i <= 2; ++i) { w[i + 2] = exp(-(double)(i * i) / (2.0 * sigma * sigma)); s += w[i + 2]; }
    for (int i = 0; i < 5; ++i) w[i] /= s;
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            double acc = 0.0;
            for (int v = -2; v <= 2; ++v)
                for (int u = -2; u <= 2; ++u)
                    acc += w[v + 2] * w[u + 2] * px(in, W, H, x + u, y + v);
            out[(size_t)y * W + x] = acc;
        }
}

/* Table II "Gradient Filter", a rectangular operation: unnormalised Sobel.
 * Ix is the derivative along x (columns), positive for values increasing with x;
 * Iy the same along y (rows). */
void or_sobel3(const double* in, double* ix, double* iy, int W, int H)
{
    static const double kx[3][3] = {{-1, 0, 1}, {-2, 0, 2}, {-1, 0, 1}};
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            double gx = 0.0, gy = 0.0;
            for (int v = -1; v <= 1; ++v)
                for (int u = -1; u <= 1; ++u) {
                    double p = px(in, W, H, x + u, y + v);
                    gx += kx[v + 1][u + 1] * p;  /* row weight (1,2,1), column diff */
                    gy += kx[u + 1][v + 1] * p;  /* the transpose */
                }
            ix[(size_t)y * W + x] = gx;
            iy[(size_t)y * W + x] = gy;
        }
}

void or_gradmag(const double* ix, const double* iy, double* out, int W, int H)
{
    for (size_t i = 0; i < (size_t)W * H; ++i) out[i] = sqrt(ix[i] * ix[i] + iy[i] * iy[i]);
}

/* Structure-tensor entries, point operations. */
void or_products(const double* ix, const double* iy, double* pxx, double* pxy, double* pyy, int W, int H)
{
    for (size_t i = 0; i < (size_t)W * H; ++i) {
        pxx[i] = ix[i] * ix[i];
        pxy[i] = ix[i] * iy[i];
        pyy[i] = iy[i] * iy[i];
    }
}

/* Rectangular operation: unweighted (2rx+1) x (2ry+1) window sum, replicate
 * borders. */
void or_box(const double* in, double* out, int W, int H, int rx, int ry)
{
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            double acc = 0.0;
            for (int v = -ry; v <= ry; ++v)
                for (int u = -rx; u <= rx; ++u) acc += px(in, W, H, x + u, y + v);
            out[(size_t)y * W + x] = acc;
        }
}

void or_boxsum(const double* in, double* out, int W, int H, int r) { or_box(in, out, W, H, r, r); }

/* Rectangular operation with free weights: the correlation
 * out(x, y) = sum_{v,u} w[v + ry][u + rx] * in(x + u, y + v), replicate
 * borders, w row-major with 2rx+1 entries per row. */
void or_stencil(const double* in, double* out, int W, int H, int rx, int ry, const double* w)
{
    const int kw = 2 * rx + 1;
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            double acc = 0.0;
            for (int v = -ry; v <= ry; ++v)
                for (int u = -rx; u <= rx; ++u) acc += w[(v + ry) * kw + (u + rx)] * px(in, W, H, x + u, y + v);
            out[(size_t)y * W + x] = acc;
        }
}

/* Point operations of the generic chain. */
enum { OR_P_AFFINE = 0, OR_P_ABS = 1, OR_P_SQUARE = 2, OR_P_SQRTABS = 3, OR_P_CLAMP = 4 };

static double or_point_value(int kind, double a, double b, double v)
{
    switch (kind) {
    case OR_P_AFFINE: return a * v + b;
    case OR_P_ABS: return fabs(v);
    case OR_P_SQUARE: return v * v;
    case OR_P_SQRTABS: return sqrt(fabs(v));
    default: return fmin(fmax(v, a), b);  /* clamp to [a, b] */
    }
}

void or_point(const double* in, double* out, int W, int H, int kind, double a, double b)
{
    for (size_t i = 0; i < (size_t)W * H; ++i) out[i] = or_point_value(kind, a, b, in[i]);
}

/* Harris corner response from the window sums of the structure tensor. */
void or_harris(const double* sxx, const double* sxy, const double* syy, double* out, int W, int H, double k)
{
    for (size_t i = 0; i < (size_t)W * H; ++i) {
        double tr = sxx[i] + syy[i];
        out[i] = sxx[i] * syy[i] - sxy[i] * sxy[i] - k * tr * tr;
    }
}

/* Table III Threshold(): keep the value where it is >= TH, else 0. */
void or_threshold(const double* in, double* out, int W, int H, double thr)
{
    for (size_t i = 0; i < (size_t)W * H; ++i) out[i] = in[i] >= thr ? in[i] : 0.0;
}

/* 3x3 non-maximum suppression: 255 where the value is positive and no 3x3
 * neighbour (replicate borders) exceeds it.  Marked pixels are the features. */
void or_nms3(const double* in, double* out, int W, int H)
{
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            double c = in[(size_t)y * W + x];
            int keep = c > 0.0;
            for (int v = -1; v <= 1 && keep; ++v)
                for (int u = -1; u <= 1; ++u)
                    if (px(in, W, H, x + u, y + v) > c) { keep = 0; break; }
            out[(size_t)y * W + x] = keep ? 255.0 : 0.0;
        }
}

/* Multi-frame point operation (Table I): absolute temporal difference. */
void or_framediff(const double* cur, const double* prev, double* out, int W, int H)
{
    for (size_t i = 0; i < (size_t)W * H; ++i) out[i] = fabs(cur[i] - prev[i]);
}

static int op_in_ch(int op, int cur)
{
    switch (op) {
    case OR_RGB2GRAY: return 3;
    case OR_SOBEL3: return 1;
    case OR_GRADMAG: case OR_PRODUCTS: return 2;
    case OR_HARRIS: return 3;
    case OR_BOXSUM5: return cur;
    default: return 1;
    }
}

static int op_out_ch(int op, int in_ch)
{
    switch (op) {
    case OR_SOBEL3: return 2;
    case OR_PRODUCTS: return 3;
    case OR_BOXSUM5: return in_ch;
    default: return 1;
    }
}

typedef struct {
    const int32_t* ops; int n;
    const double* in; int in_ch;
    int W, H, T;
    double* out; int out_ch;
    double* prefd;         /* frame-local output before a trailing framediff */
    double sigma, k, thr;
    int t_begin, t_end;
    double* pts; int64_t pts_cap; int64_t npts;
    int status;
} job_t;

/* Run the frame-local part of the chain (every op except a trailing framediff)
 * on frame t; result planes go to res (out_ch planes). */
static int run_frame(const job_t* j, int n_local, int t, double* res, double* pts, int64_t cap, int64_t* npts)
{
    size_t P = (size_t)j->W * j->H;
    double* a = (double*)malloc(sizeof(double) * P * 3);
    double* b = (double*)malloc(sizeof(double) * P * 3);
    if (!a || !b) { free(a); free(b); return -1; }
    int ch = j->in_ch;
    for (int c = 0; c < ch; ++c)
        memcpy(a + c * P, j->in + ((size_t)c * j->T + t) * P, sizeof(double) * P);
    for (int s = 0; s < n_local; ++s) {
        int op = j->ops[s];
        if (op_in_ch(op, ch) != ch) { free(a); free(b); return -2; }
        int oc = op_out_ch(op, ch);
        switch (op) {
        case OR_RGB2GRAY: or_rgb2gray(a, a + P, a + 2 * P, b, j->W, j->H); break;
        case OR_GAUSS5: or_gauss5(a, b, j->W, j->H, j->sigma); break;
        case OR_SOBEL3: or_sobel3(a, b, b + P, j->W, j->H); break;
        case OR_GRADMAG: or_gradmag(a, a + P, b, j->W, j->H); break;
        case OR_PRODUCTS: or_products(a, a + P, b, b + P, b + 2 * P, j->W, j->H); break;
        case OR_BOXSUM5: for (int c = 0; c < ch; ++c) or_boxsum(a + c * P, b + c * P, j->W, j->H, 2); break;
        case OR_HARRIS: or_harris(a, a + P, a + 2 * P, b, j->W, j->H, j->k); break;
        case OR_THRESHOLD: or_threshold(a, b, j->W, j->H, j->thr); break;
        case OR_NMS3:
            or_nms3(a, b, j->W, j->H);
            for (int y = 0; y < j->H; ++y)
                for (int x = 0; x < j->W; ++x) {
                    size_t i = (size_t)y * j->W + x;
                    if (b[i] != 0.0) {
                        if (*npts < cap) {
                            double* q = pts + 4 * (*npts);
                            q[0] = t; q[1] = y; q[2] = x; q[3] = a[i];
                        }
                        ++*npts;
                    }
                }
            break;
        default: free(a); free(b); return -3;
        }
        double* tmp = a; a = b; b = tmp;
        ch = oc;
    }
    memcpy(res, a, sizeof(double) * P * ch);
    free(a); free(b);
    return ch;
}

static void* worker(void* arg)
{
    job_t* j = (job_t*)arg;
    size_t P = (size_t)j->W * j->H;
    int has_fd = j->n > 0 && j->ops[j->n - 1] == OR_FRAMEDIFF;
    int n_local = has_fd ? j->n - 1 : j->n;
    int lch = j->out_ch;
    double* res = (double*)malloc(sizeof(double) * P * 3);
    if (!res) { j->status = -1; return NULL; }
    for (int t = j->t_begin; t < j->t_end; ++t) {
        int ch = run_frame(j, n_local, t, res, j->pts, j->pts_cap, &j->npts);
        if (ch < 0) { j->status = ch; break; }
        if (has_fd && ch != 1) { j->status = -4; break; }
        if (!has_fd && ch != lch) { j->status = -5; break; }
        double* dst = has_fd ? j->prefd : j->out;
        for (int c = 0; c < ch; ++c)
            memcpy(dst + ((size_t)c * j->T + t) * P, res + c * P, sizeof(double) * P);
    }
    free(res);
    return NULL;
}

/*
 * Run ops[0..n) over the volume in[in_ch][T][H][W] (double planes) and write
 * the last op's output to out[out_ch][T][H][W].  Feature points from nms3 are
 * written as rows (t, y, x, response) into pts (capacity pts_cap rows); the
 * total count is returned in *n_pts (it may exceed the capacity).  Frames are
 * split into contiguous ranges over nthreads threads; this changes no
 * arithmetic.  framediff is supported as the last op only and reads the
 * previous frame of its input, the first frame being its own predecessor.
 * Returns 0 on success, a negative code on a malformed chain.
 */
int or_chain(const int32_t* ops, int32_t n, const double* in, int32_t in_ch, int32_t W, int32_t H,
             int32_t T, double* out, int32_t out_ch, double sigma, double k, double thr,
             double* pts, int64_t pts_cap, int64_t* n_pts, int32_t nthreads)
{
    if (n <= 0 || W <= 0 || H <= 0 || T <= 0) return -10;
    for (int s = 0; s < n - 1; ++s)
        if (ops[s] == OR_FRAMEDIFF) return -11;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > T) nthreads = T;
    size_t P = (size_t)W * H;
    int has_fd = ops[n - 1] == OR_FRAMEDIFF;
    double* prefd = NULL;
    if (has_fd) {
        if (n == 1) prefd = (double*)in;
        else {
            prefd = (double*)malloc(sizeof(double) * P * T);
            if (!prefd) return -1;
        }
    }
    job_t* jobs = (job_t*)calloc(nthreads, sizeof(job_t));
    pthread_t* th = (pthread_t*)calloc(nthreads, sizeof(pthread_t));
    int64_t per_cap = nthreads > 0 ? pts_cap / nthreads : 0;
    double** jpts = (double**)calloc(nthreads, sizeof(double*));
    for (int i = 0; i < nthreads; ++i) {
        job_t* j = &jobs[i];
        j->ops = ops; j->n = n; j->in = in; j->in_ch = in_ch; j->W = W; j->H = H; j->T = T;
        j->out = out; j->out_ch = out_ch; j->prefd = prefd;
        j->sigma = sigma; j->k = k; j->thr = thr;
        j->t_begin = (int)((int64_t)T * i / nthreads);
        j->t_end = (int)((int64_t)T * (i + 1) / nthreads);
        /* each thread collects points privately; merged in frame order below */
        j->pts_cap = pts_cap;
        jpts[i] = pts_cap > 0 ? (double*)malloc(sizeof(double) * 4 * pts_cap) : NULL;
        j->pts = jpts[i];
    }
    (void)per_cap;
    if (!(has_fd && n == 1)) {
        for (int i = 0; i < nthreads; ++i) pthread_create(&th[i], NULL, worker, &jobs[i]);
        for (int i = 0; i < nthreads; ++i) pthread_join(th[i], NULL);
    }
    int status = 0;
    int64_t total = 0;
    for (int i = 0; i < nthreads; ++i) {
        if (jobs[i].status) status = jobs[i].status;
        for (int64_t q = 0; q < jobs[i].npts; ++q) {
            if (total < pts_cap && q < pts_cap) memcpy(pts + 4 * total, jobs[i].pts + 4 * q, sizeof(double) * 4);
            ++total;
        }
        free(jpts[i]);
    }
    *n_pts = total;
    if (status == 0 && has_fd) {
        if (out_ch != 1) status = -6;
        else
            for (int t = 0; t < T; ++t)
                or_framediff(prefd + (size_t)t * P, prefd + (size_t)(t > 0 ? t - 1 : 0) * P,
                             out + (size_t)t * P, W, H);
    }
    if (has_fd && n > 1) free(prefd);
    free(jobs); free(th); free(jpts);
    return status;
}

/* ------------------------------------------------------------------ generic chains */

enum { OR_G_POINT = 0, OR_G_STENCIL = 1, OR_G_BOX = 2 };

typedef struct {
    const int32_t* kind; const int32_t* rx; const int32_t* ry; const int32_t* pk;
    const double* pa; const double* pb; const double* w;
    int n;
    const double* in; double* out;
    int W, H, T, t_begin, t_end, status;
} gjob_t;

static void* gworker(void* arg)
{
    gjob_t* j = (gjob_t*)arg;
    size_t P = (size_t)j->W * j->H;
    double* a = (double*)malloc(sizeof(double) * P);
    double* b = (double*)malloc(sizeof(double) * P);
    if (!a || !b) { free(a); free(b); j->status = -1; return NULL; }
    for (int t = j->t_begin; t < j->t_end; ++t) {
        memcpy(a, j->in + (size_t)t * P, sizeof(double) * P);
        size_t woff = 0;
        for (int s = 0; s < j->n; ++s) {
            switch (j->kind[s]) {
            case OR_G_POINT: or_point(a, b, j->W, j->H, j->pk[s], j->pa[s], j->pb[s]); break;
            case OR_G_STENCIL:
                or_stencil(a, b, j->W, j->H, j->rx[s], j->ry[s], j->w + woff);
                woff += (size_t)(2 * j->rx[s] + 1) * (2 * j->ry[s] + 1);
                break;
            case OR_G_BOX: or_box(a, b, j->W, j->H, j->rx[s], j->ry[s]); break;
            default: j->status = -3; free(a); free(b); return NULL;
            }
            double* tmp = a; a = b; b = tmp;
        }
        memcpy(j->out + (size_t)t * P, a, sizeof(double) * P);
    }
    free(a); free(b);
    return NULL;
}

/*
 * Generic chain: stages 0..n-1 of kinds OR_G_*, applied in order to every
 * frame of in[T][H][W] (frames are independent: no generic stage looks at
 * other frames), result in out[T][H][W].  rx/ry are the window radii of the
 * window stages; pk/pa/pb the kind and parameters of the point stages; w the
 * weights of the stencil stages, concatenated in stage order.
 */
int or_gchain(const int32_t* kind, const int32_t* rx, const int32_t* ry, const int32_t* pk, const double* pa,
              const double* pb, const double* w, int32_t n, const double* in, int32_t W, int32_t H, int32_t T,
              double* out, int32_t nthreads)
{
    if (n <= 0 || W <= 0 || H <= 0 || T <= 0) return -10;
    for (int s = 0; s < n; ++s)
        if (kind[s] != OR_G_POINT && (rx[s] < 0 || ry[s] < 0)) return -12;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > T) nthreads = T;
    gjob_t* jobs = (gjob_t*)calloc(nthreads, sizeof(gjob_t));
    pthread_t* th = (pthread_t*)calloc(nthreads, sizeof(pthread_t));
    if (!jobs || !th) { free(jobs); free(th); return -1; }
    for (int i = 0; i < nthreads; ++i) {
        gjob_t* j = &jobs[i];
        j->kind = kind; j->rx = rx; j->ry = ry; j->pk = pk; j->pa = pa; j->pb = pb; j->w = w; j->n = n;
        j->in = in; j->out = out; j->W = W; j->H = H; j->T = T;
        j->t_begin = (int)((int64_t)T * i / nthreads);
        j->t_end = (int)((int64_t)T * (i + 1) / nthreads);
        pthread_create(&th[i], NULL, gworker, j);
    }
    int status = 0;
    for (int i = 0; i < nthreads; ++i) {
        pthread_join(th[i], NULL);
        if (jobs[i].status) status = jobs[i].status;
    }
    free(jobs); free(th);
    return status;
}

/* ------------------------------------------------------------------ temporal generic chains */

/*
 * Generic chains whose stages may look at earlier frames: besides the point,
 * stencil and window-sum stages above,
 *   - a stencil with a frame window (Table I, spatio-temporal operation): rt
 *     frames back, weights w[tau][v + ry][u + rx] for tau = 0..rt (tau = frames
 *     back), out(x, y, t) = sum_{tau, v, u} w[tau][v][u] * in(x + u, y + v,
 *     max(t - tau, 0)): replicate borders in space and, before the first
 *     frame, in time;
 *   - an IIR filter (Table II "IIR Filter", a multi-frame point operation):
 *     y[t] = a * x[t] + (1 - a) * y[t - 1] per pixel, with y[-1] := x[0] (so
 *     y[0] = x[0]).
 * Frames are no longer independent, so the chain runs stage by stage over the
 * whole volume: every stage's output for all frames is formed from its input
 * for all frames before the next stage starts.
 */
enum { OR_G_IIR = 3 };

int or_gchain_seq(const int32_t* kind, const int32_t* rx, const int32_t* ry, const int32_t* rt, const int32_t* pk,
                  const double* pa, const double* pb, const double* w, int32_t n, const double* in, int32_t W,
                  int32_t H, int32_t T, double* out)
{
    if (n <= 0 || W <= 0 || H <= 0 || T <= 0) return -10;
    const size_t P = (size_t)W * H, V = P * T;
    double* a = (double*)malloc(sizeof(double) * V);
    double* b = (double*)malloc(sizeof(double) * V);
    double* tmp = (double*)malloc(sizeof(double) * P);
    if (!a || !b || !tmp) { free(a); free(b); free(tmp); return -1; }
    memcpy(a, in, sizeof(double) * V);
    size_t woff = 0;
    int status = 0;
    for (int s = 0; s < n && status == 0; ++s) {
        switch (kind[s]) {
        case OR_G_POINT:
            for (int t = 0; t < T; ++t) or_point(a + t * P, b + t * P, W, H, pk[s], pa[s], pb[s]);
            break;
        case OR_G_BOX:
            if (rx[s] < 0 || ry[s] < 0) { status = -12; break; }
            for (int t = 0; t < T; ++t) or_box(a + t * P, b + t * P, W, H, rx[s], ry[s]);
            break;
        case OR_G_STENCIL: {
            if (rx[s] < 0 || ry[s] < 0 || rt[s] < 0) { status = -12; break; }
            const size_t nw = (size_t)(2 * rx[s] + 1) * (2 * ry[s] + 1);
            for (int t = 0; t < T; ++t) {
                double* o = b + t * P;
                for (size_t i = 0; i < P; ++i) o[i] = 0.0;
                for (int tau = 0; tau <= rt[s]; ++tau) {
                    const int tf = t - tau < 0 ? 0 : t - tau;
                    or_stencil(a + tf * P, tmp, W, H, rx[s], ry[s], w + woff + tau * nw);
                    for (size_t i = 0; i < P; ++i) o[i] += tmp[i];
                }
            }
            woff += nw * (rt[s] + 1);
            break;
        }
        case OR_G_IIR: {
            const double c = pa[s];
            for (size_t i = 0; i < P; ++i) {
                double y = a[i];  /* y[-1] := x[0] */
                for (int t = 0; t < T; ++t) {
                    y = c * a[t * P + i] + (1.0 - c) * y;
                    b[t * P + i] = y;
                }
            }
            break;
        }
        default: status = -3;
        }
        double* sw = a; a = b; b = sw;
    }
    if (status == 0) memcpy(out, a, sizeof(double) * V);
    free(a); free(b); free(tmp);
    return status;
}
