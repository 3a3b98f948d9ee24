/*
 * Driver for the AddressSanitizer / UndefinedBehaviorSanitizer build of the
 * oracle (test infrastructure: built and run by tests/test_asan.py on the
 * CPU).  The oracle source is compiled into this translation unit.
 *
 * It draws a small particle set from a fixed 64-bit LCG (positions around the
 * camera target, some behind the camera, a few screen-filling footprints,
 * every species, one fixed-size species) and calls every oracle entry point
 * in the modes the tests use: palette and vector colour, window, centre
 * counts, prefilter, the ordered transfer, projection, an empty set and the
 * argument checks.  Inputs and outputs are written as raw little-endian
 * arrays to the directory named by argv[1], so that the test can re-run the
 * same cases through the ordinary oracle build and compare the bits.
 */
#include "../../oracle/splotch_oracle.c"

#include <stdio.h>

enum { N = 700, M = 5, W = 37, H = 23 };

static uint64_t lcg_state = 0x853c49e6748fea9bull;
static double uniform01(void) {
    lcg_state = lcg_state * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(lcg_state >> 11) * (1.0 / 9007199254740992.0);
}

static int write_array(const char* dir, const char* name, const void* p, size_t bytes) {
    char path[4096];
    snprintf(path, sizeof path, "%s/%s.bin", dir, name);
    FILE* f = fopen(path, "wb");
    if (!f) return -1;
    const size_t w = bytes ? fwrite(p, 1, bytes, f) : 0;
    fclose(f);
    return w == bytes ? 0 : -1;
}

static void camera_of(oracle_camera* c) {
    const double eye[3] = {0.3, -0.2, 3.0}, target[3] = {0.0, 0.1, 0.0}, up[3] = {0.1, 1.0, 0.0};
    /* every value is a float32 widened to double, as the library receives */
    for (int k = 0; k < 3; ++k) {
        c->eye[k] = (float)eye[k];
        c->target[k] = (float)target[k];
        c->up[k] = (float)up[k];
    }
    c->fov_deg = 40.0;
    c->z_near = (float)0.05;
    c->width = W;
    c->height = H;
}

static void params_of(oracle_params* p, int colour_mode, double prefilter) {
    memset(p, 0, sizeof *p);
    p->chi = 2.0;
    const double br[4] = {0.4, 0.15, 0.9, 0.05}, ab[4] = {0.7, 0.3, 0.05, 1.2};
    for (int k = 0; k < 4; ++k) {
        p->brightness[k] = (float)br[k];
        p->absorption[k] = (float)ab[k];
    }
    p->fixed_sigma_frac[3] = (float)0.02;
    p->scalar_min = colour_mode ? -0.5 : -1.0;
    p->scalar_max = colour_mode ? 1.5 : 1.0;
    p->scalar_log10 = colour_mode ? 0 : 1;
    p->col_norm = colour_mode ? 0 : 1;
    p->colour_mode = colour_mode;
    p->prefilter = (float)prefilter;
}

int main(int argc, char** argv) {
    if (argc != 2) {
        fprintf(stderr, "usage: %s OUTDIR\n", argv[0]);
        return 2;
    }
    const char* dir = argv[1];
    float* x = malloc(N * sizeof(float));
    float* y = malloc(N * sizeof(float));
    float* z = malloc(N * sizeof(float));
    float* h = malloc(N * sizeof(float));
    float* in = malloc(N * sizeof(float));
    float* s = malloc(N * sizeof(float));
    float* vx = malloc(N * sizeof(float));
    float* vy = malloc(N * sizeof(float));
    float* vz = malloc(N * sizeof(float));
    uint8_t* sp = malloc(N);
    float cmap[3 * M];
    for (int i = 0; i < 3 * M; ++i) cmap[i] = (float)uniform01();
    for (int p = 0; p < N; ++p) {
        x[p] = (float)(uniform01() * 2.4 - 1.2);
        y[p] = (float)(uniform01() * 1.6 - 0.7);
        z[p] = (float)(uniform01() * 7.0 - 3.5);   /* some behind the camera */
        h[p] = (float)(p % 97 == 0 ? 0.8 : 0.004 + 0.05 * uniform01());
        in[p] = (float)(0.2 + uniform01());
        s[p] = (float)(0.01 + 20.0 * uniform01());
        vx[p] = (float)(uniform01() * 2.0 - 0.5);
        vy[p] = (float)(uniform01() * 2.0 - 0.5);
        vz[p] = (float)(uniform01() * 2.0 - 0.5);
        sp[p] = (uint8_t)(p % 5);                  /* 4 is read as species 3 */
    }
    int bad = 0;
    bad |= write_array(dir, "x", x, N * sizeof(float));
    bad |= write_array(dir, "y", y, N * sizeof(float));
    bad |= write_array(dir, "z", z, N * sizeof(float));
    bad |= write_array(dir, "h", h, N * sizeof(float));
    bad |= write_array(dir, "intensity", in, N * sizeof(float));
    bad |= write_array(dir, "scalar", s, N * sizeof(float));
    bad |= write_array(dir, "vx", vx, N * sizeof(float));
    bad |= write_array(dir, "vy", vy, N * sizeof(float));
    bad |= write_array(dir, "vz", vz, N * sizeof(float));
    bad |= write_array(dir, "species", sp, N);
    bad |= write_array(dir, "cmap", cmap, sizeof cmap);

    oracle_camera cam;
    camera_of(&cam);
    oracle_params prm;
    oracle_stats st;
    const size_t full3 = (size_t)W * H * 3;
    double* L = malloc(full3 * sizeof(double));
    double* I = malloc(full3 * sizeof(double));
    int32_t* cnt = malloc((size_t)W * H * sizeof(int32_t));
    int64_t stats[2 * 8];
    int rc;

    /* palette colours, log10 scalar, centre counts, whole image */
    params_of(&prm, 0, 0.0);
    rc = oracle_render(N, x, y, z, h, in, s, NULL, NULL, NULL, sp, &cam, M, cmap, &prm, NULL, 1,
                       L, I, cnt, &st);
    bad |= rc != 0;
    stats[0] = st.samples;
    stats[1] = st.active;
    bad |= write_array(dir, "palette_L", L, full3 * sizeof(double));
    bad |= write_array(dir, "palette_I", I, full3 * sizeof(double));
    bad |= write_array(dir, "palette_count", cnt, (size_t)W * H * sizeof(int32_t));

    /* a window touching the right and bottom edges, with counts */
    const int32_t win[4] = {20, 9, 17, 14};
    const size_t win3 = (size_t)win[2] * win[3] * 3;
    rc = oracle_render(N, x, y, z, h, in, s, NULL, NULL, NULL, sp, &cam, M, cmap, &prm, win, 1,
                       L, I, cnt, &st);
    bad |= rc != 0;
    stats[2] = st.samples;
    stats[3] = st.active;
    bad |= write_array(dir, "window_L", L, win3 * sizeof(double));
    bad |= write_array(dir, "window_count", cnt, (size_t)win[2] * win[3] * sizeof(int32_t));

    /* vector colours */
    params_of(&prm, 1, 0.0);
    rc = oracle_render(N, x, y, z, h, in, NULL, vx, vy, vz, sp, &cam, 0, NULL, &prm, NULL, 1, L,
                       NULL, NULL, &st);
    bad |= rc != 0;
    stats[4] = st.samples;
    stats[5] = st.active;
    bad |= write_array(dir, "vector_L", L, full3 * sizeof(double));

    /* prefiltered (anti-aliased) render */
    params_of(&prm, 0, 0.75);
    rc = oracle_render(N, x, y, z, h, in, s, NULL, NULL, NULL, sp, &cam, M, cmap, &prm, NULL, 1,
                       L, NULL, NULL, &st);
    bad |= rc != 0;
    stats[6] = st.samples;
    stats[7] = st.active;
    bad |= write_array(dir, "prefilter_L", L, full3 * sizeof(double));

    /* ordered transfer (E != A), whole image and a window at the origin */
    params_of(&prm, 0, 0.0);
    rc = oracle_render_ordered(N, x, y, z, h, in, s, NULL, NULL, NULL, sp, &cam, M, cmap, &prm,
                               NULL, 1, L, I, &st);
    bad |= rc != 0;
    stats[8] = st.samples;
    stats[9] = st.active;
    bad |= write_array(dir, "ordered_L", L, full3 * sizeof(double));
    bad |= write_array(dir, "ordered_I", I, full3 * sizeof(double));
    const int32_t win0[4] = {0, 0, 11, 23};
    const size_t win03 = (size_t)win0[2] * win0[3] * 3;
    rc = oracle_render_ordered(N, x, y, z, h, in, s, NULL, NULL, NULL, sp, &cam, M, cmap, &prm,
                               win0, 1, L, I, &st);
    bad |= rc != 0;
    stats[10] = st.samples;
    stats[11] = st.active;
    bad |= write_array(dir, "ordered_window_I", I, win03 * sizeof(double));

    /* projection */
    double* X = malloc(N * sizeof(double));
    double* Y = malloc(N * sizeof(double));
    double* S = malloc(N * sizeof(double));
    double* D = malloc(N * sizeof(double));
    rc = oracle_project(N, x, y, z, h, sp, &cam, &prm, X, Y, S, D);
    bad |= rc != 0;
    bad |= write_array(dir, "project_X", X, N * sizeof(double));
    bad |= write_array(dir, "project_depth", D, N * sizeof(double));

    /* an empty set clears the image */
    rc = oracle_render(0, x, y, z, h, in, s, NULL, NULL, NULL, sp, &cam, M, cmap, &prm, NULL, 1, L,
                       I, cnt, &st);
    bad |= rc != 0 || st.samples != 0 || L[0] != 0.0 || cnt[W * H - 1] != 0;
    stats[12] = st.samples;

    /* argument checks: each returns -1 before touching the outputs */
    const int32_t win_out[4] = {30, 0, 8, 23};    /* leaves the image */
    int nbad = 0;
    nbad += oracle_render(N, x, y, z, h, in, s, NULL, NULL, NULL, sp, &cam, M, cmap, &prm,
                          win_out, 1, L, I, cnt, &st) == -1;
    nbad += oracle_render(N, x, y, z, h, in, s, NULL, NULL, NULL, sp, &cam, 1, cmap, &prm, NULL,
                          1, L, I, cnt, &st) == -1;
    nbad += oracle_render(-1, x, y, z, h, in, s, NULL, NULL, NULL, sp, &cam, M, cmap, &prm, NULL,
                          1, L, I, cnt, &st) == -1;
    params_of(&prm, 1, 0.0);
    nbad += oracle_render(N, x, y, z, h, in, s, NULL, NULL, NULL, sp, &cam, M, cmap, &prm, NULL,
                          1, L, I, cnt, &st) == -1;   /* vector mode without vectors */
    oracle_camera flat = cam;
    memcpy(flat.target, flat.eye, sizeof flat.eye);     /* degenerate camera */
    params_of(&prm, 0, 0.0);
    nbad += oracle_render_ordered(N, x, y, z, h, in, s, NULL, NULL, NULL, sp, &flat, M, cmap,
                                  &prm, NULL, 1, L, I, &st) == -1;
    nbad += oracle_project(N, x, y, z, h, sp, &flat, &prm, X, Y, S, D) == -1;
    stats[13] = nbad;
    stats[14] = bad;
    stats[15] = N;
    bad |= write_array(dir, "stats", stats, sizeof stats);

    free(x); free(y); free(z); free(h); free(in); free(s);
    free(vx); free(vy); free(vz); free(sp);
    free(L); free(I); free(cnt);
    free(X); free(Y); free(S); free(D);
    if (bad || nbad != 6) {
        fprintf(stderr, "oracle driver: bad=%d argument checks=%d of 6\n", bad, nbad);
        return 1;
    }
    return 0;
}
