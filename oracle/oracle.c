/*
 * oracle.c -- plain, slow FP64 CPU reference for the volumetric filters that
 * the Harpia library offers (Section III-C: Gaussian smoothing in the
 * filtering suite; erosion, dilation and opening in the label-editing
 * module) and for the gradients of those filters.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may load, call or
 * link this file: only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no source, header, table or helper
 * with the GPU library.
 *
 * Conventions
 *   - volumes are C-ordered [nz][ny][nx] arrays of double, x contiguous;
 *   - shape[0..2] = {nz, ny, nx}; per-axis parameters are ordered {z, y, x};
 *   - every value is computed in IEEE double, no fast-math.
 *
 * The paper gives no formulas for these filters (it names them only), so
 * each function writes out the textbook definition that the build adopts:
 *   - boundary: half-sample symmetric reflection of the index (the edge
 *     voxel is repeated: ... 2 1 0 | 0 1 2 ... n-1 | n-1 n-2 ...), taken
 *     modulo 2n so that radii larger than the volume reflect repeatedly;
 *   - Gaussian taps: sampled exp(-k^2 / (2 sigma^2)) for k = -r..r,
 *     normalised to sum 1, with r = (int)(truncate * sigma + 0.5);
 *   - erosion / dilation: min / max of the input over the structuring
 *     element placed at the voxel, counting only offsets inside the volume;
 *   - structuring elements: box |d_a| <= r_a, ball dz^2 + dy^2 + dx^2 <= r^2.
 *
 * Parity pins: every function here is checked in tests/test_oracle_pins.py
 * against scipy.ndimage, pure-Python brute force, closed forms and
 * invariants (constant volume, impulse, linearity, adjointness, duality,
 * order, idempotence, finite differences).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define IDX(z, y, x, ny, nx) ((((int64_t)(z) * (ny)) + (y)) * (nx) + (x))

/* Half-sample symmetric reflection of index i into [0, n). */
int64_t oracle_reflect(int64_t i, int64_t n)
{
    int64_t period = 2 * n;
    int64_t m = i % period;
    if (m < 0)
        m += period;
    return (m < n) ? m : (period - 1 - m);
}

/* Truncation radius of a Gaussian: (int)(truncate * sigma + 0.5). */
int oracle_gauss_radius(double sigma, double truncate)
{
    return (int)(truncate * sigma + 0.5);
}

/* w[k + r] = exp(-k^2 / (2 sigma^2)) / sum_j exp(-j^2 / (2 sigma^2)),
 * k = -r..r.  Returns 0, or -1 for sigma <= 0 or r < 0. */
int oracle_gauss_taps(double sigma, int r, double *w)
{
    if (!(sigma > 0.0) || r < 0)
        return -1;
    double total = 0.0;
    for (int k = -r; k <= r; ++k) {
        double e = exp(-((double)k * k) / (2.0 * sigma * sigma));
        w[k + r] = e;
        total += e;
    }
    for (int k = -r; k <= r; ++k)
        w[k + r] /= total;
    return 0;
}

/* Derivative of the normalised taps with respect to sigma, radius held
 * fixed.  With e_k = exp(-k^2/(2 s^2)), de_k/ds = e_k k^2 / s^3 and
 * w_k = e_k / S, the quotient rule gives
 *   dw_k/ds = w_k (k^2 - sum_j w_j j^2) / s^3. */
int oracle_gauss_dtaps(double sigma, int r, double *dw)
{
    if (!(sigma > 0.0) || r < 0)
        return -1;
    double *w = (double *)malloc(sizeof(double) * (size_t)(2 * r + 1));
    if (!w)
        return -2;
    oracle_gauss_taps(sigma, r, w);
    double m2 = 0.0;
    for (int k = -r; k <= r; ++k)
        m2 += w[k + r] * (double)k * (double)k;
    double s3 = sigma * sigma * sigma;
    for (int k = -r; k <= r; ++k)
        dw[k + r] = w[k + r] * ((double)k * k - m2) / s3;
    free(w);
    return 0;
}

/* Direct 3D convolution with the outer product of three 1D tap vectors:
 *   y[z,y,x] = sum_{a,b,c} wz[a] wy[b] wx[c] v[R(z+a), R(y+b), R(x+c)].
 * This is the definition itself (a triple loop over taps per voxel). */
void oracle_conv3d_direct(const double *v, double *out, const int64_t *shape,
                          const double *wz, int rz, const double *wy, int ry,
                          const double *wx, int rx)
{
    int64_t nz = shape[0], ny = shape[1], nx = shape[2];
#pragma omp parallel for schedule(dynamic)
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x) {
                double acc = 0.0;
                for (int a = -rz; a <= rz; ++a) {
                    int64_t zz = oracle_reflect(z + a, nz);
                    for (int b = -ry; b <= ry; ++b) {
                        int64_t yy = oracle_reflect(y + b, ny);
                        for (int c = -rx; c <= rx; ++c) {
                            int64_t xx = oracle_reflect(x + c, nx);
                            acc += wz[a + rz] * wy[b + ry] * wx[c + rx] *
                                   v[IDX(zz, yy, xx, ny, nx)];
                        }
                    }
                }
                out[IDX(z, y, x, ny, nx)] = acc;
            }
}

/* One 1D pass along `axis` (0 = z, 1 = y, 2 = x):
 *   out[p] = sum_k w[k + r] in[p with coordinate c -> R(c + k)]. */
void oracle_conv1d(const double *in, double *out, const int64_t *shape,
                   int axis, const double *w, int r)
{
    int64_t nz = shape[0], ny = shape[1], nx = shape[2];
    int64_t n = shape[axis];
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x) {
                int64_t c = (axis == 0) ? z : (axis == 1) ? y : x;
                double acc = 0.0;
                for (int k = -r; k <= r; ++k) {
                    int64_t s = oracle_reflect(c + k, n);
                    int64_t zz = (axis == 0) ? s : z;
                    int64_t yy = (axis == 1) ? s : y;
                    int64_t xx = (axis == 2) ? s : x;
                    acc += w[k + r] * in[IDX(zz, yy, xx, ny, nx)];
                }
                out[IDX(z, y, x, ny, nx)] = acc;
            }
}

/* Literal transpose of oracle_conv1d: every product w[k] * in[p] is added
 * back onto the source voxel that the forward pass read it from,
 *   out[p with c -> R(c + k)] += w[k + r] in[p].
 * Each 1D line is independent, so lines run in parallel and the scatter
 * inside one line stays serial. */
void oracle_conv1d_transpose(const double *in, double *out,
                             const int64_t *shape, int axis, const double *w,
                             int r)
{
    int64_t nz = shape[0], ny = shape[1], nx = shape[2];
    int64_t n = shape[axis];
    int64_t total = nz * ny * nx;
    memset(out, 0, sizeof(double) * (size_t)total);
    /* enumerate lines by the two coordinates other than `axis` */
    int64_t n1 = (axis == 0) ? ny : nz;
    int64_t n2 = (axis == 2) ? ny : nx;
#pragma omp parallel for schedule(static)
    for (int64_t i1 = 0; i1 < n1; ++i1)
        for (int64_t i2 = 0; i2 < n2; ++i2)
            for (int64_t c = 0; c < n; ++c) {
                int64_t z, y, x;
                if (axis == 0) { z = c; y = i1; x = i2; }
                else if (axis == 1) { z = i1; y = c; x = i2; }
                else { z = i1; y = i2; x = c; }
                double g = in[IDX(z, y, x, ny, nx)];
                for (int k = -r; k <= r; ++k) {
                    int64_t s = oracle_reflect(c + k, n);
                    int64_t zz = (axis == 0) ? s : z;
                    int64_t yy = (axis == 1) ? s : y;
                    int64_t xx = (axis == 2) ? s : x;
                    out[IDX(zz, yy, xx, ny, nx)] += w[k + r] * g;
                }
            }
}

/* Separable form of oracle_conv3d_direct: an x pass, then y, then z. */
int oracle_conv3d_separable(const double *v, double *out, const int64_t *shape,
                            const double *wz, int rz, const double *wy, int ry,
                            const double *wx, int rx)
{
    int64_t total = shape[0] * shape[1] * shape[2];
    double *t1 = (double *)malloc(sizeof(double) * (size_t)total);
    double *t2 = (double *)malloc(sizeof(double) * (size_t)total);
    if (!t1 || !t2) {
        free(t1);
        free(t2);
        return -2;
    }
    oracle_conv1d(v, t1, shape, 2, wx, rx);
    oracle_conv1d(t1, t2, shape, 1, wy, ry);
    oracle_conv1d(t2, out, shape, 0, wz, rz);
    free(t1);
    free(t2);
    return 0;
}

/* Transpose of the separable operator G = Gz Gy Gx: G^T = Gx^T Gy^T Gz^T,
 * each factor the literal scatter above. */
int oracle_conv3d_transpose(const double *g, double *out, const int64_t *shape,
                            const double *wz, int rz, const double *wy, int ry,
                            const double *wx, int rx)
{
    int64_t total = shape[0] * shape[1] * shape[2];
    double *t1 = (double *)malloc(sizeof(double) * (size_t)total);
    double *t2 = (double *)malloc(sizeof(double) * (size_t)total);
    if (!t1 || !t2) {
        free(t1);
        free(t2);
        return -2;
    }
    oracle_conv1d_transpose(g, t1, shape, 0, wz, rz);
    oracle_conv1d_transpose(t1, t2, shape, 1, wy, ry);
    oracle_conv1d_transpose(t2, out, shape, 2, wx, rx);
    free(t1);
    free(t2);
    return 0;
}

/* Is offset (dz, dy, dx) in the structuring element?
 * se 0 = box |d_a| <= r_a; se 1 = ball dz^2 + dy^2 + dx^2 <= r^2 with the
 * single radius r = r[0] (the ball is isotropic). */
static int in_se(int se, const int *r, int dz, int dy, int dx)
{
    if (se == 0)
        return abs(dz) <= r[0] && abs(dy) <= r[1] && abs(dx) <= r[2];
    return dz * dz + dy * dy + dx * dx <= r[0] * r[0];
}

/* Erosion (op 0, min) or dilation (op 1, max) by brute force over the
 * structuring element.  Offsets whose voxel falls outside the volume are
 * skipped; the centre is always inside, so the set is never empty.
 * If `arg` is not NULL it receives the flat index of the extremum that
 * comes first in lexicographic (dz, dy, dx) order (a later offset replaces
 * the running extremum only when it is strictly better). */
int oracle_morph3d(const double *v, double *out, int64_t *arg,
                   const int64_t *shape, int op, int se, const int *radius)
{
    if ((op != 0 && op != 1) || (se != 0 && se != 1))
        return -1;
    if (radius[0] < 0 || radius[1] < 0 || radius[2] < 0)
        return -1;
    if (se == 1 && (radius[1] != radius[0] || radius[2] != radius[0]))
        return -1;
    int64_t nz = shape[0], ny = shape[1], nx = shape[2];
    int rz = radius[0], ry = radius[1], rx = radius[2];
#pragma omp parallel for schedule(dynamic)
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x) {
                int64_t best_i = IDX(z, y, x, ny, nx);
                double best = v[best_i];
                int have = 0;
                for (int dz = -rz; dz <= rz; ++dz)
                    for (int dy = -ry; dy <= ry; ++dy)
                        for (int dx = -rx; dx <= rx; ++dx) {
                            if (!in_se(se, radius, dz, dy, dx))
                                continue;
                            int64_t zz = z + dz, yy = y + dy, xx = x + dx;
                            if (zz < 0 || zz >= nz || yy < 0 || yy >= ny ||
                                xx < 0 || xx >= nx)
                                continue;
                            int64_t i = IDX(zz, yy, xx, ny, nx);
                            double s = v[i];
                            int better = !have || (op == 0 ? (s < best)
                                                           : (s > best));
                            if (better) {
                                best = s;
                                best_i = i;
                                have = 1;
                            }
                        }
                out[IDX(z, y, x, ny, nx)] = best;
                if (arg)
                    arg[IDX(z, y, x, ny, nx)] = best_i;
            }
    return 0;
}

/* Subgradient routing of erosion / dilation: every output voxel p sends its
 * upstream gradient to the voxel arg[p] that supplied its value,
 *   gin[j] = sum over p with arg[p] = j of g[p]   (serial, in order of p). */
void oracle_route(const double *g, const int64_t *arg, double *gin, int64_t n)
{
    memset(gin, 0, sizeof(double) * (size_t)n);
    for (int64_t p = 0; p < n; ++p)
        gin[arg[p]] += g[p];
}

/* Fixed threshold: b = 1 where v > t (strict), else 0. */
void oracle_threshold(const double *v, double *b, int64_t n, double t)
{
    for (int64_t i = 0; i < n; ++i)
        b[i] = (v[i] > t) ? 1.0 : 0.0;
}

/* Number of worker threads OpenMP will use (reported by the CPU baseline). */
int oracle_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
