// Drives the host planner under the sanitizers: every operation's descriptor,
// every contiguous part of the fixed chains in every partition mode, random
// generic chains read from a file (stage kind, radii, frames back, parameters,
// weights) planned with every partition mode, kernel-configuration overrides,
// the Eq. 6 box, the partition model on random price tables and learned
// planning with the shipped network.  Any sanitizer report aborts the run;
// the driver prints a line per stage and "ok" at the end.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include <vector>

#include "fz.h"

static int fails = 0;
#define CHECK(c)                                                           \
    do {                                                                   \
        if (!(c)) {                                                        \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            ++fails;                                                       \
        }                                                                  \
    } while (0)

static void plan_all_partitions(const fz_stage* st, int n, int W, int H, int T, int engine)
{
    fz_plan_opts o = {};
    o.width = W;
    o.height = H;
    o.frames = T;
    o.engine = engine;
    for (int mode = 0; mode < 2; ++mode) {
        o.partition = mode;
        fz_plan* p = nullptr;
        if (fz_plan_chain(st, n, &o, &p) == FZ_OK) {
            const int ns = fz_plan_num_segments(p);
            std::vector<int32_t> sl(ns);
            CHECK(fz_plan_segments(p, sl.data(), ns) == FZ_OK);
            for (int i = 0; i < ns; ++i) {
                fz_segment_info si;
                CHECK(fz_plan_segment_info(p, i, &si) == FZ_OK);
                float f[64];
                CHECK(fz_plan_segment_features(p, i, f, 64) == fz_cost_n_features());
                (void)fz_plan_set_segment_config(p, i, FZ_ENGINE_TILE, 32, 32, 0);
                (void)fz_plan_set_segment_config(p, i, FZ_ENGINE_AUTO, 0, 0, 4);
            }
            (void)fz_workspace_bytes(p);
            fz_plan_destroy(p);
        }
    }
    // explicit cuts: every single cut
    for (int c = 0; c + 1 < n; ++c) {
        o.partition = FZ_PART_EXPLICIT;
        o.n_cuts = 1;
        o.cuts = &c;
        fz_plan* p = nullptr;
        if (fz_plan_chain(st, n, &o, &p) == FZ_OK) fz_plan_destroy(p);
    }
}

int main(int argc, char** argv)
{
    // 1. descriptors, fixed chains
    const int harris[] = {FZ_OP_RGB2GRAY, FZ_OP_GAUSS5, FZ_OP_SOBEL3, FZ_OP_PRODUCTS, FZ_OP_BOXSUM5,
                          FZ_OP_HARRIS, FZ_OP_THRESHOLD, FZ_OP_NMS3, FZ_OP_FRAMEDIFF};
    for (int op = 0; op < 20; ++op) {
        fz_stage s;
        (void)fz_stage_describe(op, &s);
    }
    const int sizes[][3] = {{800, 600, 1000}, {192, 432, 600}, {7, 5, 3}, {1, 1, 1}, {130, 9, 40}};
    for (auto& sz : sizes)
        for (int a = 0; a < 9; ++a)
            for (int b = a; b < 9; ++b) {
                fz_stage st[9];
                for (int k = a; k <= b; ++k) fz_stage_describe(harris[k], &st[k - a]);
                plan_all_partitions(st, b - a + 1, sz[0], sz[1], sz[2], FZ_ENGINE_AUTO);
            }
    printf("fixed chains done\n");
    // 2. random generic chains from the file written by the test
    if (argc > 1) {
        FILE* f = fopen(argv[1], "r");
        CHECK(f != nullptr);
        int nchains = 0;
        while (f && fscanf(f, "%d", &nchains) == 1) {
            std::vector<fz_stage> st(nchains);
            std::vector<std::vector<float>> ws(nchains);
            for (int i = 0; i < nchains; ++i) {
                int op, rx, ry, rt, nw;
                float a, b, c;
                if (fscanf(f, "%d %d %d %d %f %f %f %d", &op, &rx, &ry, &rt, &a, &b, &c, &nw) != 8) return 2;
                fz_stage_describe(op, &st[i]);
                st[i].rx = rx;
                st[i].ry = ry;
                st[i].rt = rt;
                st[i].param[0] = a;
                st[i].param[1] = b;
                st[i].param[2] = c;
                if (i == 0) st[i].in_dtype = FZ_U8;
                ws[i].resize(nw);
                for (int q = 0; q < nw; ++q)
                    if (fscanf(f, "%f", &ws[i][q]) != 1) return 2;
                st[i].weights = nw ? ws[i].data() : nullptr;
            }
            plan_all_partitions(st.data(), nchains, 800, 600, 64, FZ_ENGINE_AUTO);
            plan_all_partitions(st.data(), nchains, 13, 7, 9, FZ_ENGINE_AUTO);
            plan_all_partitions(st.data(), nchains, 320, 240, 100, FZ_ENGINE_JIT);
        }
        if (f) fclose(f);
        printf("generic chains done\n");
    }
    // 3. Eq. 6, partition model on random tables
    double x, t;
    CHECK(fz_box_eq6(4096, 1, 1, &x, &t) == FZ_OK && fabs(x * x * t - 4096) < 1e-6);
    CHECK(fz_box_eq6(-1, 1, 1, &x, &t) == FZ_E_INVALID);
    srand(7);
    for (int n = 1; n <= 64; n += 7) {
        std::vector<double> c((size_t)n * n);
        for (auto& v : c) v = (rand() % 10 == 0) ? INFINITY : (double)(rand() % 1000);
        std::vector<int32_t> sl(n);
        int32_t ns = 0;
        double tot = 0;
        CHECK(fz_partition_min(c.data(), n, sl.data(), &ns, &tot) == FZ_OK);
    }
    // 4. learned planning with the shipped network (parameters from a file)
    if (argc > 2) {
        FILE* f = fopen(argv[2], "rb");
        CHECK(f != nullptr);
        const int F = fz_cost_n_features();
        std::vector<float> prm((size_t)F * 64 + 64 + 64 * 64 + 64 + 64 + 1);
        CHECK(f && fread(prm.data(), sizeof(float), prm.size(), f) == prm.size());
        if (f) fclose(f);
        fz_plan_opts o = {};
        o.width = 640;
        o.height = 480;
        o.frames = 64;
        o.cost_model = FZ_COST_LEARNED;
        o.cost_weights = prm.data();
        o.cost_n_features = fz_cost_n_features();
        fz_stage st[9];
        for (int k = 0; k < 9; ++k) fz_stage_describe(harris[k], &st[k]);
        fz_plan* p = nullptr;
        CHECK(fz_plan_chain(st, 9, &o, &p) == FZ_OK);
        fz_plan_destroy(p);
        printf("learned planning done\n");
    }
    printf(fails ? "FAILED\n" : "ok\n");
    return fails ? 1 : 0;
}
