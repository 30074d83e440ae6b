/*
 * Oracle of the tracking stage -- TEST INFRASTRUCTURE ONLY (used by tests/,
 * the smoke check and the benchmark's CPU baseline; never by the library).
 *
 * The paper's pipeline ends by applying a Kalman filter to the extracted
 * feature points (Sec. III; Table II "Apply Kalman Filter": a single-point,
 * multi-frame operation; Table IV: kernel-to-kernel dependent, so never fused
 * with the kernels before it).  The paper gives no model, so this is the
 * textbook discrete Kalman filter with a constant-velocity model and greedy
 * nearest-neighbour association:
 *
 *   state s = (x, y, vx, vy) (column, row, pixels per frame), covariance P;
 *   F = [[1,0,1,0],[0,1,0,1],[0,0,1,0],[0,0,0,1]],
 *   Q = q [[1/4,0,1/2,0],[0,1/4,0,1/2],[1/2,0,1,0],[0,1/2,0,1]]
 *       (white acceleration noise over one frame),
 *   H = [[1,0,0,0],[0,1,0,0]], R = r I.
 *
 * Per frame t (points of the frame ordered by (y, x), measurement z = (x, y)):
 *   1. predict every live track: s- = F s, P- = F P F^T + Q;
 *   2. for every track and point: innovation nu = z - H s-, S = H P- H^T + R,
 *      S^-1 = [[S11, -S01], [-S10, S00]] / det, det = S00 S11 - S01 S10,
 *      d2 = nu^T S^-1 nu; the pair is a candidate when d2 <= gate;
 *   3. candidates are taken in increasing (d2, track id, point index) order
 *      when neither the track nor the point is taken yet (greedy nearest
 *      neighbour);
 *   4. a matched track is updated: K = P- H^T S^-1, s = s- + K nu,
 *      P = (I - K H) P-; an unmatched one keeps s-, P- and counts a miss, and
 *      is dropped once it has missed more than max_miss frames in a row;
 *   5. every unmatched point starts a track, s = (x, y, 0, 0),
 *      P = diag(r, r, v0, v0), with the next id (in point order).
 * Output: one record per live track and frame after step 5:
 *   (t, id, status, x, y, vx, vy), status 0 = predicted only, 1 = updated,
 *   2 = started.
 *
 * Every matrix product is the plain sum over k = 0, 1, ... from 0.0, in
 * double precision; the library's tracking kernel evaluates the same sums in
 * the same order, so the two agree to the bit.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t id, miss;
    double s[4];
    double P[4][4];
} otrack;

typedef struct {
    double d2;
    int32_t id, ti, pj;
} ocand;

static int cand_cmp(const void* a, const void* b)
{
    const ocand* x = (const ocand*)a;
    const ocand* y = (const ocand*)b;
    if (x->d2 != y->d2) return x->d2 < y->d2 ? -1 : 1;
    if (x->id != y->id) return x->id < y->id ? -1 : 1;
    return x->pj < y->pj ? -1 : (x->pj > y->pj);
}

static int pt_cmp(const void* a, const void* b)
{
    const int32_t* x = (const int32_t*)a;
    const int32_t* y = (const int32_t*)b;
    if (x[0] != y[0]) return x[0] < y[0] ? -1 : 1; /* frame */
    if (x[1] != y[1]) return x[1] < y[1] ? -1 : 1; /* row */
    return x[2] < y[2] ? -1 : (x[2] > y[2]);       /* column */
}

static void matmul(int n, int m, int p, const double* A, const double* B, double* C)
{
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < p; ++j) {
            double acc = 0.0;
            for (int k = 0; k < m; ++k) acc = acc + A[i * m + k] * B[k * p + j];
            C[i * p + j] = acc;
        }
}

static void transpose(int n, int m, const double* A, double* At)
{
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < m; ++j) At[j * n + i] = A[i * m + j];
}

/*
 * pts: n_pts records (t, y, x) as int32 triples, any order; frames 0..T-1.
 * out: capacity rows of (t, id, status) int32 + (x, y, vx, vy) double, i.e.
 * out_i[3 * k + 0..2] and out_d[4 * k + 0..3].  Returns the number of
 * records (may exceed the capacity: only the first `cap` are written), or a
 * negative error.
 */
int64_t or_track(const int32_t* pts, int64_t n_pts, int32_t T, double q, double r, double gate, int32_t max_miss,
                 double v0, int32_t* out_i, double* out_d, int64_t cap)
{
    if (T <= 0 || n_pts < 0 || max_miss < 0) return -1;
    int32_t* p = (int32_t*)malloc(sizeof(int32_t) * 3 * (n_pts > 0 ? n_pts : 1));
    otrack* tr = (otrack*)malloc(sizeof(otrack) * (n_pts + 1));
    otrack* nt = (otrack*)malloc(sizeof(otrack) * (n_pts + 1));
    if (!p || !tr || !nt) { free(p); free(tr); free(nt); return -2; }
    memcpy(p, pts, sizeof(int32_t) * 3 * n_pts);
    qsort(p, (size_t)n_pts, sizeof(int32_t) * 3, pt_cmp);

    const double F[16] = {1, 0, 1, 0, 0, 1, 0, 1, 0, 0, 1, 0, 0, 0, 0, 1};
    const double Q[16] = {0.25 * q, 0, 0.5 * q, 0, 0, 0.25 * q, 0, 0.5 * q, 0.5 * q, 0, q, 0, 0, 0.5 * q, 0, q};
    const double Hm[8] = {1, 0, 0, 0, 0, 1, 0, 0};
    double Ft[16], Ht[8];
    transpose(4, 4, F, Ft);
    transpose(2, 4, Hm, Ht);

    int64_t ntr = 0, nrec = 0, k0 = 0;
    int32_t next_id = 0;
    for (int32_t t = 0; t < T; ++t) {
        int64_t k1 = k0;
        while (k1 < n_pts && p[3 * k1] == t) ++k1;
        const int64_t np = k1 - k0;
        const int32_t* fp = p + 3 * k0;
        /* 1. predict */
        double (*Sinv)[4] = (double(*)[4])malloc(sizeof(double) * 4 * (ntr > 0 ? ntr : 1));
        double (*Spr)[4] = (double(*)[4])malloc(sizeof(double) * 4 * (ntr > 0 ? ntr : 1));
        for (int64_t i = 0; i < ntr; ++i) {
            double sp[4], FP[16], Pp[16], HP[8], S[4];
            matmul(4, 4, 1, F, tr[i].s, sp);
            matmul(4, 4, 4, F, &tr[i].P[0][0], FP);
            matmul(4, 4, 4, FP, Ft, Pp);
            for (int e = 0; e < 16; ++e) Pp[e] = Pp[e] + Q[e];
            memcpy(tr[i].s, sp, sizeof sp);
            memcpy(&tr[i].P[0][0], Pp, sizeof Pp);
            matmul(2, 4, 4, Hm, Pp, HP);
            matmul(2, 4, 2, HP, Ht, S);
            S[0] = S[0] + r;
            S[3] = S[3] + r;
            const double det = S[0] * S[3] - S[1] * S[2];
            Sinv[i][0] = S[3] / det;
            Sinv[i][1] = -S[1] / det;
            Sinv[i][2] = -S[2] / det;
            Sinv[i][3] = S[0] / det;
            memcpy(Spr[i], S, sizeof S);
        }
        /* 2. candidates */
        ocand* c = (ocand*)malloc(sizeof(ocand) * (size_t)(ntr * np > 0 ? ntr * np : 1));
        int64_t nc = 0;
        for (int64_t i = 0; i < ntr; ++i)
            for (int64_t j = 0; j < np; ++j) {
                double z[2] = {(double)fp[3 * j + 2], (double)fp[3 * j + 1]}, hs[2], nu[2];
                matmul(2, 4, 1, Hm, tr[i].s, hs);
                nu[0] = z[0] - hs[0];
                nu[1] = z[1] - hs[1];
                double d2 = 0.0;
                for (int a = 0; a < 2; ++a)
                    for (int b = 0; b < 2; ++b) d2 = d2 + nu[a] * Sinv[i][2 * a + b] * nu[b];
                if (d2 <= gate) {
                    c[nc].d2 = d2;
                    c[nc].id = tr[i].id;
                    c[nc].ti = (int32_t)i;
                    c[nc].pj = (int32_t)j;
                    ++nc;
                }
            }
        /* 3. greedy association */
        qsort(c, (size_t)nc, sizeof(ocand), cand_cmp);
        int32_t* tmatch = (int32_t*)malloc(sizeof(int32_t) * (ntr > 0 ? ntr : 1));
        char* ptaken = (char*)calloc((size_t)(np > 0 ? np : 1), 1);
        for (int64_t i = 0; i < ntr; ++i) tmatch[i] = -1;
        for (int64_t k = 0; k < nc; ++k)
            if (tmatch[c[k].ti] < 0 && !ptaken[c[k].pj]) {
                tmatch[c[k].ti] = c[k].pj;
                ptaken[c[k].pj] = 1;
            }
        /* 4. update or count a miss; 5. start tracks; output */
        int64_t n_new = 0;
        for (int64_t i = 0; i < ntr; ++i) {
            otrack* o = &tr[i];
            int status = 0;
            if (tmatch[i] >= 0) {
                const int64_t j = tmatch[i];
                double z[2] = {(double)fp[3 * j + 2], (double)fp[3 * j + 1]}, hs[2], nu[2];
                double PHt[8], K[8], Knu[4], KH[16], IKH[16], Pn[16];
                matmul(2, 4, 1, Hm, o->s, hs);
                nu[0] = z[0] - hs[0];
                nu[1] = z[1] - hs[1];
                matmul(4, 4, 2, &o->P[0][0], Ht, PHt);
                matmul(4, 2, 2, PHt, Sinv[i], K);
                matmul(4, 2, 1, K, nu, Knu);
                for (int e = 0; e < 4; ++e) o->s[e] = o->s[e] + Knu[e];
                matmul(4, 2, 4, K, Hm, KH);
                for (int a = 0; a < 4; ++a)
                    for (int b = 0; b < 4; ++b) IKH[4 * a + b] = (a == b ? 1.0 : 0.0) - KH[4 * a + b];
                matmul(4, 4, 4, IKH, &o->P[0][0], Pn);
                memcpy(&o->P[0][0], Pn, sizeof Pn);
                o->miss = 0;
                status = 1;
            } else {
                o->miss += 1;
                if (o->miss > max_miss) continue; /* dropped */
            }
            nt[n_new] = *o;
            if (nrec < cap) {
                out_i[3 * nrec] = t;
                out_i[3 * nrec + 1] = o->id;
                out_i[3 * nrec + 2] = status;
                memcpy(out_d + 4 * nrec, o->s, sizeof o->s);
            }
            ++nrec;
            ++n_new;
        }
        for (int64_t j = 0; j < np; ++j) {
            if (ptaken[j]) continue;
            otrack* o = &nt[n_new++];
            memset(o, 0, sizeof *o);
            o->id = next_id++;
            o->s[0] = (double)fp[3 * j + 2];
            o->s[1] = (double)fp[3 * j + 1];
            o->P[0][0] = r;
            o->P[1][1] = r;
            o->P[2][2] = v0;
            o->P[3][3] = v0;
            if (nrec < cap) {
                out_i[3 * nrec] = t;
                out_i[3 * nrec + 1] = o->id;
                out_i[3 * nrec + 2] = 2;
                memcpy(out_d + 4 * nrec, o->s, sizeof o->s);
            }
            ++nrec;
        }
        otrack* sw = tr; tr = nt; nt = sw;
        ntr = n_new;
        free(Sinv); free(Spr); free(c); free(tmatch); free(ptaken);
        k0 = k1;
    }
    free(p); free(tr); free(nt);
    return nrec;
}
