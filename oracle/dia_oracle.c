/*
 * FP64 matrix-free oracle for the SFSeg adjacency -- TEST INFRASTRUCTURE ONLY.
 *
 * Burceanu & Leordeanu, "A 3D Convolutional Approach to Spectral Object
 * Segmentation in Space and Time" (arXiv 1907.02731).
 *
 * Applies exactly the entries of M from Eq. (2),
 *     M_ij = w_i w_j [1 - alpha (F_i - F_j)^2] G(j - i),
 * row by row, visiting every neighbour offset of the box neighbourhood and
 * skipping neighbours outside the volume.  It never uses the convolution
 * factorisation of Eq. (7), so it stays independent of the GPU route; it is
 * the explicit scipy CSR matrix of the Python oracle evaluated without
 * storing it, for volumes too large to hold M (a 70x480x854 clip with a
 * 5x11x11 box has ~1.7e10 non-zeros).
 *
 * w (= S^p), F and x are float64 arrays in (t, y, x) row-major order,
 * W fastest.  Only tests, the smoke check and the benchmark's CPU baseline
 * load this library.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

static double *offset_weights(int rt, int rs, double sigma_t, double sigma_s)
{
    const int nt = 2 * rt + 1, ns = 2 * rs + 1;
    double *g = (double *)malloc(sizeof(double) * (size_t)nt * ns * ns);
    if (!g) return NULL;
    for (int a = 0; a < nt; ++a)
        for (int b = 0; b < ns; ++b)
            for (int c = 0; c < ns; ++c) {
                const double dt = a - rt, dy = b - rs, dx = c - rs;
                g[((size_t)a * ns + b) * ns + c] =
                    exp(-(dt * dt) / (2.0 * sigma_t * sigma_t)
                        - (dy * dy + dx * dx) / (2.0 * sigma_s * sigma_s));
            }
    return g;
}

/* (M x)_i for the single voxel i = (t, y, x). */
static double row_apply(int64_t T, int64_t H, int64_t W, int rt, int rs, double alpha,
                        const double *g, const double *w, const double *f,
                        const double *xv, int64_t t, int64_t y, int64_t x)
{
    const int ns = 2 * rs + 1;
    const int64_t i = (t * H + y) * W + x;
    const double wi = w[i], fi = f[i];
    if (wi == 0.0) return 0.0;
    double acc = 0.0;
    for (int a = -rt; a <= rt; ++a) {
        const int64_t tj = t + a;
        if (tj < 0 || tj >= T) continue;
        for (int b = -rs; b <= rs; ++b) {
            const int64_t yj = y + b;
            if (yj < 0 || yj >= H) continue;
            const double *grow = g + ((size_t)(a + rt) * ns + (b + rs)) * ns + rs;
            const int64_t base = (tj * H + yj) * W;
            for (int c = -rs; c <= rs; ++c) {
                const int64_t xj = x + c;
                if (xj < 0 || xj >= W) continue;
                const int64_t j = base + xj;
                const double d = fi - f[j];
                acc += wi * w[j] * (1.0 - alpha * d * d) * grow[c] * xv[j];
            }
        }
    }
    return acc;
}

/* y = M x over the whole volume.  Returns 0, or -1 on bad arguments. */
int oracle_apply(int64_t T, int64_t H, int64_t W, int rt, int rs,
                 double sigma_t, double sigma_s, double alpha,
                 const double *w, const double *f, const double *x, double *y)
{
    if (T < 1 || H < 1 || W < 1 || rt < 0 || rs < 0 || !w || !f || !x || !y) return -1;
    double *g = offset_weights(rt, rs, sigma_t, sigma_s);
    if (!g) return -1;
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t t = 0; t < T; ++t)
        for (int64_t yy = 0; yy < H; ++yy)
            for (int64_t xx = 0; xx < W; ++xx)
                y[(t * H + yy) * W + xx] =
                    row_apply(T, H, W, rt, rs, alpha, g, w, f, x, t, yy, xx);
    free(g);
    return 0;
}

/* out[k] = (M x)_{rows[k]} for k < nrows: sampled rows of the product. */
int oracle_apply_rows(int64_t T, int64_t H, int64_t W, int rt, int rs,
                      double sigma_t, double sigma_s, double alpha,
                      const double *w, const double *f, const double *x,
                      const int64_t *rows, int64_t nrows, double *out)
{
    if (T < 1 || H < 1 || W < 1 || rt < 0 || rs < 0 || !w || !f || !x || !rows || !out)
        return -1;
    const int64_t N = T * H * W;
    for (int64_t k = 0; k < nrows; ++k)
        if (rows[k] < 0 || rows[k] >= N) return -1;
    double *g = offset_weights(rt, rs, sigma_t, sigma_s);
    if (!g) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nrows; ++k) {
        const int64_t i = rows[k];
        const int64_t t = i / (H * W), rem = i % (H * W);
        out[k] = row_apply(T, H, W, rt, rs, alpha, g, w, f, x, t, rem / W, rem % W);
    }
    free(g);
    return 0;
}

/* Number of OpenMP threads the parallel loops above use. */
int oracle_num_threads(void)
{
    int n = 1;
#pragma omp parallel
    {
#pragma omp single
        {
#ifdef _OPENMP
            extern int omp_get_num_threads(void);
            n = omp_get_num_threads();
#endif
        }
    }
    return n;
}
