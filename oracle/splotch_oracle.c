/*
 * FP64 reference renderer for the Splotch emission = absorption path.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the HIP library is
 * checked against.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load or call it; the product library never does, and
 * the two share no code, headers or tables.
 *
 * It computes the plain definition of the image, particle by particle, with
 * no size classes, no tiles and no sorting, in double precision:
 *
 *   O1  camera basis: forward = (target-eye)/|target-eye|,
 *       right = forward x up / |forward x up|, up' = right x forward;
 *       focal length in pixels f = (W/2) / tan(fov/2), fov horizontal.
 *   O2  camera coordinates c = (right.(x-eye), up'.(x-eye), forward.(x-eye))
 *       (roto-translation, Section "Splotch Overview", processing stage).
 *   O3  a particle with c_z <= z_near is behind the camera and is skipped.
 *   O4  perspective projection X = W/2 + f c_x/c_z, Y = H/2 - f c_y/c_z;
 *       pixel (i,j) (column i, row j counted from the top) has its centre at
 *       (i+1/2, j+1/2).
 *   O5  screen smoothing length sigma = f h / c_z (the smoothing length is
 *       projected with the positions; Eq. 7's r(p) is chi*sigma), or
 *       sigma = fixed_sigma_frac[species] * W for a fixed-size species.
 *  O5p screen-plane prefilter (an anti-aliased render): with s > 0 the
 *       optical depth is convolved with the normalised Gaussian
 *       exp(-d^2/s^2)/(pi s^2) before the pixel centres sample it.  The
 *       convolution of two Gaussians is a Gaussian: sigma becomes
 *       sqrt(sigma^2 + s^2) and the coefficients are multiplied by
 *       sigma^2/(sigma^2 + s^2), which keeps each particle's integral.
 *   O6  colour: s' = clamp((g(s) - s_min)/(s_max - s_min), 0, 1) with
 *       g = log10 when requested (min/max normalisation, Section
 *       "CUDA Implementation" footnote); u = s'(M-1), m = min(floor u, M-2),
 *       t = u - m, colour = (1-t) C[m] + t C[m+1] (palette look-up).
 *  O6v colour by vector (Section "Splotch Overview": the three colour
 *       components taken from a vector quantity such as the velocity):
 *       colour_c = clamp((v_c - s_min)/(s_max - s_min), 0, 1), c = R, G, B,
 *       with the same min/max normalisation and no logarithm.
 *   O7  peak optical depth tau0 = brightness[species] * intensity * colour
 *       (times sqrt(pi) h when col_norm is set: the column of a 3-D Gaussian
 *       of unit central density, Eq. 2).  E = A = this coefficient.
 *   O8  every pixel centre at screen distance d with d^2 <= (chi sigma)^2
 *       receives L_c += tau0_c exp(-d^2/sigma^2): the Gaussian of Eq. 2,
 *       clipped at chi*sigma.
 *   O9  with E = A the solution of Eq. 1 along each ray is independent of
 *       the order of the particles and equals I_c = 1 - exp(-L_c) for a
 *       black background.
 *
 * Parallelism: particles are split statically over OpenMP threads, each with
 * a private FP64 image; the private images are summed in thread order.
 *
 * oracle_render_ordered() is the general E != A case of Eq. 1 (emission and
 * absorption coefficients set independently, Section "Splotch Overview"),
 * where the order along the ray matters:
 *   O10 coefficients: E_c = brightness[k] * intensity * colour_c and
 *       A_c = absorption[k] * intensity * colour_c (each times sqrt(pi) h
 *       with col_norm);
 *   O11 each particle is a thin slab at its camera depth c_z: crossing it
 *       with column weight w = exp(-d^2/sigma^2) (d^2 <= R^2) solves Eq. 1
 *       with constant coefficients, I -> I exp(-A w) + E w g(A w),
 *       g(t) = (1 - exp(-t))/t, g(0) = 1;
 *   O12 along each pixel ray the slabs are crossed from the far end (I = 0
 *       behind everything) toward the eye: decreasing c_z, and for equal c_z
 *       decreasing particle index (the ray order is (c_z, index), nearest
 *       first).
 * With A = E this gives 1 - exp(-sum E w), the image of O9; with A = 0 it
 * gives sum E w.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double eye[3], target[3], up[3];
    double fov_deg;
    double z_near;
    int32_t width, height;
} oracle_camera;

typedef struct {
    double chi;
    double brightness[4];
    double fixed_sigma_frac[4];
    double scalar_min, scalar_max;
    int32_t scalar_log10;
    int32_t col_norm;
    int32_t colour_mode; /* 0: palette of the scalar (O6); 1: vector (O6v) */
    double absorption[4]; /* O10: absorption scale per species (ordered render) */
    double prefilter;     /* O5p: prefilter sigma s (pixels), 0 = none */
} oracle_params;

typedef struct {
    int64_t samples;  /* (particle, pixel) pairs with d^2 <= R^2 in the image */
    int64_t active;   /* particles in front of the camera whose bounding box
                         [floor(X-R-1/2), ceil(X+R-1/2)] x [...] meets the image */
    int32_t threads_used;
} oracle_stats;

static void cross3(const double a[3], const double b[3], double o[3]) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

static double dot3(const double a[3], const double b[3]) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

/* O1: returns 0 on success, -1 for a degenerate camera. */
int oracle_camera_basis(const oracle_camera* cam, double right[3], double upv[3],
                        double fwd[3], double* focal) {
    double d[3] = {cam->target[0] - cam->eye[0], cam->target[1] - cam->eye[1],
                   cam->target[2] - cam->eye[2]};
    double nd = sqrt(dot3(d, d));
    if (!(nd > 0)) return -1;
    for (int k = 0; k < 3; ++k) fwd[k] = d[k] / nd;
    double r[3];
    cross3(fwd, cam->up, r);
    double nr = sqrt(dot3(r, r));
    if (!(nr > 0)) return -1;
    for (int k = 0; k < 3; ++k) right[k] = r[k] / nr;
    cross3(right, fwd, upv);
    *focal = 0.5 * cam->width / tan(0.5 * cam->fov_deg * M_PI / 180.0);
    return 0;
}

/* O5p: widens *sig by the prefilter and returns the factor that keeps the
   particle's integral (1 without a prefilter). */
static double prefilter_sigma(const oracle_params* p, double* sig) {
    if (!(p->prefilter > 0.0)) return 1.0;
    const double s2 = (*sig) * (*sig);
    const double t2 = s2 + p->prefilter * p->prefilter;
    *sig = sqrt(t2);
    return s2 / t2;
}

/* O6: palette look-up with linear interpolation between entries. */
static void colour_of(double s, const oracle_params* p, int32_t ncmap,
                      const float* cmap, double col[3]) {
    double g = p->scalar_log10 ? log10(s) : s;
    double sn = (g - p->scalar_min) / (p->scalar_max - p->scalar_min);
    if (!(sn > 0.0)) sn = 0.0; /* also catches NaN */
    if (sn > 1.0) sn = 1.0;
    double u = sn * (ncmap - 1);
    int m = (int)floor(u);
    if (m > ncmap - 2) m = ncmap - 2;
    double t = u - m;
    for (int c = 0; c < 3; ++c)
        col[c] = (1.0 - t) * (double)cmap[3 * m + c] + t * (double)cmap[3 * (m + 1) + c];
}

/* O6v: each colour channel is its own normalised vector component. */
static void colour_of_vector(double vx, double vy, double vz, const oracle_params* p,
                             double col[3]) {
    const double v[3] = {vx, vy, vz};
    for (int c = 0; c < 3; ++c) {
        double sn = (v[c] - p->scalar_min) / (p->scalar_max - p->scalar_min);
        if (!(sn > 0.0)) sn = 0.0; /* also catches NaN */
        if (sn > 1.0) sn = 1.0;
        col[c] = sn;
    }
}

/*
 * Render the window of columns [wx, wx+ww) and rows [wy, wy+wh) of the
 * image (window = NULL: the whole image).  L (wh*ww*3 doubles, row-major,
 * RGB interleaved) is overwritten with the accumulated optical depth; I
 * (same layout, optional) with 1-exp(-L); center_count (wh*ww, optional)
 * with the number of particles in front of the camera whose projected
 * centre lies in the pixel.  Samples and active particles are counted
 * inside the window.  The colour input is scalar (palette mode, cmap with
 * ncmap >= 2 entries) or vx, vy, vz (vector mode; cmap is not read).
 * Returns 0, or -1 on bad arguments, -2 if memory for the per-thread images
 * is not available.
 */
int oracle_render(int64_t n, const float* x, const float* y, const float* z,
                  const float* h, const float* intensity, const float* scalar,
                  const float* vx, const float* vy, const float* vz,
                  const uint8_t* species, const oracle_camera* cam,
                  int32_t ncmap, const float* cmap, const oracle_params* prm,
                  const int32_t* window, int32_t nthreads, double* L, double* I,
                  int32_t* center_count, oracle_stats* stats) {
    if (!cam || !prm || !L || n < 0) return -1;
    if (prm->colour_mode == 0 && (ncmap < 2 || !cmap || (n > 0 && !scalar))) return -1;
    if (prm->colour_mode == 1 && (prm->scalar_log10 || (n > 0 && (!vx || !vy || !vz))))
        return -1;
    if (prm->colour_mode != 0 && prm->colour_mode != 1) return -1;
    if (cam->width <= 0 || cam->height <= 0) return -1;
    double right[3], upv[3], fwd[3], f;
    if (oracle_camera_basis(cam, right, upv, fwd, &f) != 0) return -1;
    const int64_t Wimg = cam->width;
    const int64_t wx = window ? window[0] : 0, wy = window ? window[1] : 0;
    const int64_t W = window ? window[2] : cam->width, H = window ? window[3] : cam->height;
    if (W <= 0 || H <= 0 || wx < 0 || wy < 0 || wx + W > cam->width || wy + H > cam->height)
        return -1;
    const int64_t npix3 = W * H * 3;

    int nt = 1;
#ifdef _OPENMP
    nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#endif
    /* keep the private images under ~12 GB */
    while (nt > 1 && (double)nt * npix3 * 8.0 > 12e9) nt--;
    double* priv = (double*)calloc((size_t)nt * (size_t)npix3, sizeof(double));
    if (!priv) return -2;
    int32_t* ccount = NULL;
    if (center_count) {
        memset(center_count, 0, sizeof(int32_t) * (size_t)(W * H));
        ccount = center_count;
    }
    int64_t tot_samples = 0, tot_active = 0;
    const double sqrt_pi = sqrt(M_PI);

#pragma omp parallel num_threads(nt) reduction(+ : tot_samples, tot_active)
    {
        int tid = 0, nth = 1;
#ifdef _OPENMP
        tid = omp_get_thread_num();
        nth = omp_get_num_threads();
#endif
        double* Lt = priv + (size_t)tid * (size_t)npix3;
        int64_t lo = n * tid / nth, hi = n * (tid + 1) / nth;
        for (int64_t p = lo; p < hi; ++p) {
            double xp[3] = {(double)x[p] - cam->eye[0], (double)y[p] - cam->eye[1],
                            (double)z[p] - cam->eye[2]};
            double cx = dot3(right, xp), cy = dot3(upv, xp), cz = dot3(fwd, xp);
            if (!(cz > cam->z_near)) continue;                      /* O3 */
            double X = 0.5 * Wimg + f * cx / cz;                    /* O4 */
            double Y = 0.5 * cam->height - f * cy / cz;
            int k = species ? species[p] : 0;
            if (k > 3) k = 3;
            double sig = prm->fixed_sigma_frac[k] > 0.0
                             ? prm->fixed_sigma_frac[k] * (double)Wimg
                             : f * (double)h[p] / cz;               /* O5 */
            if (!(sig > 0.0) || !isfinite(sig) || !isfinite(X) || !isfinite(Y)) continue;
            const double keep = prefilter_sigma(prm, &sig);           /* O5p */
            double R = prm->chi * sig;
            /* pixel box of the footprint in window coordinates (a superset
               of the pixel centres with d^2 <= R^2), clipped to the window */
            double bx0 = floor(X - R - 0.5) - (double)wx, bx1 = ceil(X + R - 0.5) - (double)wx;
            double by0 = floor(Y - R - 0.5) - (double)wy, by1 = ceil(Y + R - 0.5) - (double)wy;
            if (bx0 < 0) bx0 = 0;
            if (by0 < 0) by0 = 0;
            if (bx1 > (double)(W - 1)) bx1 = (double)(W - 1);
            if (by1 > (double)(H - 1)) by1 = (double)(H - 1);
            double Xw = X - (double)wx, Yw = Y - (double)wy;
            if (ccount && Xw >= 0.0 && Xw < (double)W && Yw >= 0.0 && Yw < (double)H) {
                int64_t pix = (int64_t)floor(Yw) * W + (int64_t)floor(Xw);
#pragma omp atomic
                ccount[pix] += 1;
            }
            if (bx0 > bx1 || by0 > by1) continue;
            int64_t i0 = (int64_t)bx0, i1 = (int64_t)bx1, j0 = (int64_t)by0, j1 = (int64_t)by1;
            tot_active += 1;
            double col[3];
            if (prm->colour_mode == 1)
                colour_of_vector((double)vx[p], (double)vy[p], (double)vz[p], prm, col); /* O6v */
            else
                colour_of((double)scalar[p], prm, ncmap, cmap, col);    /* O6 */
            double amp = prm->brightness[k] * (double)intensity[p]; /* O7 */
            if (prm->col_norm) amp *= sqrt_pi * (double)h[p];
            amp *= keep;
            double tau0[3] = {amp * col[0], amp * col[1], amp * col[2]};
            double R2 = R * R, s2 = sig * sig;
            for (int64_t j = j0; j <= j1; ++j) {
                double dy = (double)(j + wy) + 0.5 - Y;
                for (int64_t i = i0; i <= i1; ++i) {
                    double dx = (double)(i + wx) + 0.5 - X;
                    double d2 = dx * dx + dy * dy;
                    if (d2 <= R2) {                                 /* O8 */
                        double e = exp(-d2 / s2);
                        double* px = Lt + (j * W + i) * 3;
                        px[0] += tau0[0] * e;
                        px[1] += tau0[1] * e;
                        px[2] += tau0[2] * e;
                        tot_samples += 1;
                    }
                }
            }
        }
    }

    /* sum the private images in thread order */
#pragma omp parallel for num_threads(nt) schedule(static)
    for (int64_t q = 0; q < npix3; ++q) {
        double acc = 0.0;
        for (int t = 0; t < nt; ++t) acc += priv[(size_t)t * (size_t)npix3 + q];
        L[q] = acc;
        if (I) I[q] = -expm1(-acc);                                  /* O9 */
    }
    free(priv);
    if (stats) {
        stats->samples = tot_samples;
        stats->active = tot_active;
        stats->threads_used = nt;
    }
    return 0;
}

/* One fragment of a pixel ray: a particle's slab and its column weight. */
typedef struct {
    double depth;
    int64_t index;
    double w;
} oracle_fragment;

/* Ray order (O12): nearest first, i.e. increasing (depth, index). */
static int fragment_cmp(const void* a, const void* b) {
    const oracle_fragment* x = (const oracle_fragment*)a;
    const oracle_fragment* y = (const oracle_fragment*)b;
    if (x->depth != y->depth) return x->depth < y->depth ? -1 : 1;
    if (x->index != y->index) return x->index < y->index ? -1 : 1;
    return 0;
}

/* g(t) = (1 - exp(-t))/t with g(0) = 1 (O11). */
static double slab_gain(double t) { return t == 0.0 ? 1.0 : -expm1(-t) / t; }

/*
 * Ordered (E != A) render of the window (as oracle_render).  L receives the
 * total absorption depth sum A_c w of each pixel (order-free), I the
 * intensity of O11-O12.  Fragments are collected per pixel, sorted into ray
 * order and crossed from the far end.  Returns 0, -1 on bad arguments, -2
 * when memory for the fragments is not available.
 */
int oracle_render_ordered(int64_t n, const float* x, const float* y, const float* z,
                          const float* h, const float* intensity, const float* scalar,
                          const float* vx, const float* vy, const float* vz,
                          const uint8_t* species, const oracle_camera* cam, int32_t ncmap,
                          const float* cmap, const oracle_params* prm, const int32_t* window,
                          int32_t nthreads, double* L, double* I, oracle_stats* stats) {
    if (!cam || !prm || !L || !I || n < 0) return -1;
    if (prm->colour_mode == 0 && (ncmap < 2 || !cmap || (n > 0 && !scalar))) return -1;
    if (prm->colour_mode == 1 && (prm->scalar_log10 || (n > 0 && (!vx || !vy || !vz))))
        return -1;
    if (prm->colour_mode != 0 && prm->colour_mode != 1) return -1;
    if (cam->width <= 0 || cam->height <= 0) return -1;
    double right[3], upv[3], fwd[3], f;
    if (oracle_camera_basis(cam, right, upv, fwd, &f) != 0) return -1;
    const int64_t Wimg = cam->width;
    const int64_t wx = window ? window[0] : 0, wy = window ? window[1] : 0;
    const int64_t W = window ? window[2] : cam->width, H = window ? window[3] : cam->height;
    if (W <= 0 || H <= 0 || wx < 0 || wy < 0 || wx + W > cam->width || wy + H > cam->height)
        return -1;
    const double sqrt_pi = sqrt(M_PI);

    /* per particle: projection (O1-O5), coefficients (O10) */
    double* X = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * 10);
    if (!X) return -2;
    double *Y = X + n, *S = X + 2 * n, *D = X + 3 * n, *Ec = X + 4 * n, *Ac = X + 7 * n;
    int64_t* start = (int64_t*)calloc((size_t)(W * H + 1), sizeof(int64_t));
    if (!start) { free(X); return -2; }
    int64_t tot_active = 0;
    for (int64_t p = 0; p < n; ++p) {
        D[p] = -1.0;
        double xp[3] = {(double)x[p] - cam->eye[0], (double)y[p] - cam->eye[1],
                        (double)z[p] - cam->eye[2]};
        double cx = dot3(right, xp), cy = dot3(upv, xp), cz = dot3(fwd, xp);
        if (!(cz > cam->z_near)) continue;
        X[p] = 0.5 * Wimg + f * cx / cz;
        Y[p] = 0.5 * cam->height - f * cy / cz;
        int k = species ? species[p] : 0;
        if (k > 3) k = 3;
        S[p] = prm->fixed_sigma_frac[k] > 0.0 ? prm->fixed_sigma_frac[k] * (double)Wimg
                                              : f * (double)h[p] / cz;
        if (!(S[p] > 0.0) || !isfinite(S[p]) || !isfinite(X[p]) || !isfinite(Y[p])) continue;
        const double keep = prefilter_sigma(prm, &S[p]);             /* O5p */
        D[p] = cz;
        double col[3];
        if (prm->colour_mode == 1)
            colour_of_vector((double)vx[p], (double)vy[p], (double)vz[p], prm, col);
        else
            colour_of((double)scalar[p], prm, ncmap, cmap, col);
        double amp = (double)intensity[p] * keep;
        if (prm->col_norm) amp *= sqrt_pi * (double)h[p];
        for (int c = 0; c < 3; ++c) {
            Ec[3 * p + c] = prm->brightness[k] * amp * col[c];
            Ac[3 * p + c] = prm->absorption[k] * amp * col[c];
        }
    }
    /* two sweeps over the footprints: count the fragments of each pixel,
       then fill them in */
    oracle_fragment* frag = NULL;
    int64_t tot_samples = 0;
    for (int sweep = 0; sweep < 2; ++sweep) {
        int64_t* fill = NULL;
        if (sweep == 1) {
            for (int64_t q = 0; q < W * H; ++q) start[q + 1] += start[q];
            tot_samples = start[W * H];
            frag = (oracle_fragment*)malloc(sizeof(oracle_fragment) * (size_t)(tot_samples + 1));
            fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(W * H));
            if (!frag || !fill) { free(frag); free(fill); free(start); free(X); return -2; }
            memcpy(fill, start, sizeof(int64_t) * (size_t)(W * H));
        }
        for (int64_t p = 0; p < n; ++p) {
            if (D[p] < 0.0) continue;
            double R = prm->chi * S[p];
            double bx0 = floor(X[p] - R - 0.5) - (double)wx, bx1 = ceil(X[p] + R - 0.5) - (double)wx;
            double by0 = floor(Y[p] - R - 0.5) - (double)wy, by1 = ceil(Y[p] + R - 0.5) - (double)wy;
            if (bx0 < 0) bx0 = 0;
            if (by0 < 0) by0 = 0;
            if (bx1 > (double)(W - 1)) bx1 = (double)(W - 1);
            if (by1 > (double)(H - 1)) by1 = (double)(H - 1);
            if (bx0 > bx1 || by0 > by1) continue;
            if (sweep == 0) tot_active += 1;
            double R2 = R * R, s2 = S[p] * S[p];
            for (int64_t j = (int64_t)by0; j <= (int64_t)by1; ++j) {
                double dy = (double)(j + wy) + 0.5 - Y[p];
                for (int64_t i = (int64_t)bx0; i <= (int64_t)bx1; ++i) {
                    double dx = (double)(i + wx) + 0.5 - X[p];
                    double d2 = dx * dx + dy * dy;
                    if (!(d2 <= R2)) continue;
                    int64_t q = j * W + i;
                    if (sweep == 0) {
                        start[q + 1] += 1;
                    } else {
                        oracle_fragment* fr = frag + fill[q]++;
                        fr->depth = D[p];
                        fr->index = p;
                        fr->w = exp(-d2 / s2);
                    }
                }
            }
        }
        free(fill);
    }
    int nt = 1;
#ifdef _OPENMP
    nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#endif
    (void)nt;
#pragma omp parallel for num_threads(nt) schedule(dynamic, 64)
    for (int64_t q = 0; q < W * H; ++q) {
        oracle_fragment* fr = frag + start[q];
        const int64_t m = start[q + 1] - start[q];
        qsort(fr, (size_t)m, sizeof(oracle_fragment), fragment_cmp);
        double Ip[3] = {0.0, 0.0, 0.0}, Lp[3] = {0.0, 0.0, 0.0};
        for (int64_t e = m - 1; e >= 0; --e) {           /* far end first (O12) */
            const int64_t p = fr[e].index;
            const double w = fr[e].w;
            for (int c = 0; c < 3; ++c) {
                const double t = Ac[3 * p + c] * w;
                Ip[c] = Ip[c] * exp(-t) + Ec[3 * p + c] * w * slab_gain(t);   /* O11 */
                Lp[c] += t;
            }
        }
        for (int c = 0; c < 3; ++c) {
            I[3 * q + c] = Ip[c];
            L[3 * q + c] = Lp[c];
        }
    }
    free(frag);
    free(start);
    free(X);
    if (stats) {
        stats->samples = tot_samples;
        stats->active = tot_active;
        stats->threads_used = nt;
    }
    return 0;
}

/* Projection only (O1-O5, O5p), for tests that inspect screen positions:
   sigma is the one drawn (after the prefilter). */
int oracle_project(int64_t n, const float* x, const float* y, const float* z,
                   const float* h, const uint8_t* species, const oracle_camera* cam,
                   const oracle_params* prm, double* X, double* Y, double* sigma,
                   double* depth) {
    double right[3], upv[3], fwd[3], f;
    if (oracle_camera_basis(cam, right, upv, fwd, &f) != 0) return -1;
    for (int64_t p = 0; p < n; ++p) {
        double xp[3] = {(double)x[p] - cam->eye[0], (double)y[p] - cam->eye[1],
                        (double)z[p] - cam->eye[2]};
        double cx = dot3(right, xp), cy = dot3(upv, xp), cz = dot3(fwd, xp);
        int k = species ? species[p] : 0;
        if (k > 3) k = 3;
        X[p] = 0.5 * cam->width + f * cx / cz;
        Y[p] = 0.5 * cam->height - f * cy / cz;
        sigma[p] = prm->fixed_sigma_frac[k] > 0.0 ? prm->fixed_sigma_frac[k] * cam->width
                                                  : f * (double)h[p] / cz;
        (void)prefilter_sigma(prm, &sigma[p]);                        /* O5p */
        depth[p] = cz;
    }
    return 0;
}

int oracle_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
