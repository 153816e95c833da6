/* Host sanitizer check of the oracle: every entry point on small volumes,
 * including radii beyond the volume (repeated reflection), 1-voxel axes and
 * anisotropic boxes, built with AddressSanitizer and UndefinedBehavior-
 * Sanitizer by tests/test_oracle_sanitized.py.  Prints "ok" on success. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int64_t oracle_reflect(int64_t i, int64_t n);
int oracle_gauss_radius(double sigma, double truncate);
int oracle_gauss_taps(double sigma, int r, double *w);
int oracle_gauss_dtaps(double sigma, int r, double *dw);
void oracle_conv3d_direct(const double *v, double *out, const int64_t *shape, const double *wz, int rz,
                          const double *wy, int ry, const double *wx, int rx);
void oracle_conv1d(const double *in, double *out, const int64_t *shape, int axis, const double *w, int r);
void oracle_conv1d_transpose(const double *in, double *out, const int64_t *shape, int axis, const double *w, int r);
int oracle_conv3d_separable(const double *v, double *out, const int64_t *shape, const double *wz, int rz,
                            const double *wy, int ry, const double *wx, int rx);
int oracle_conv3d_transpose(const double *g, double *out, const int64_t *shape, const double *wz, int rz,
                            const double *wy, int ry, const double *wx, int rx);
int oracle_morph3d(const double *v, double *out, int64_t *arg, const int64_t *shape, int op, int se,
                   const int *radius);
void oracle_route(const double *g, const int64_t *arg, double *gin, int64_t n);
void oracle_threshold(const double *v, double *b, int64_t n, double t);

static int fail(const char *what)
{
    printf("FAIL %s\n", what);
    return 1;
}

int main(void)
{
    static const int64_t shapes[4][3] = {{5, 6, 7}, {1, 9, 4}, {3, 1, 1}, {2, 3, 8}};
    for (int s = 0; s < 4; ++s) {
        const int64_t *sh = shapes[s];
        const int64_t n = sh[0] * sh[1] * sh[2];
        double *v = malloc(n * sizeof(double)), *a = malloc(n * sizeof(double));
        double *b = malloc(n * sizeof(double)), *c = malloc(n * sizeof(double));
        int64_t *arg = malloc(n * sizeof(int64_t));
        for (int64_t i = 0; i < n; ++i) v[i] = (double)((i * 7919) % 13) - 6.0;
        for (int si = 0; si < 3; ++si) {
            const double sigma = 0.6 + 1.7 * si;  /* radii 2, 7, 12: beyond every extent */
            const int r = oracle_gauss_radius(sigma, 3.0);
            double *w = malloc((2 * r + 1) * sizeof(double)), *dw = malloc((2 * r + 1) * sizeof(double));
            if (oracle_gauss_taps(sigma, r, w) != 0 || oracle_gauss_dtaps(sigma, r, dw) != 0) return fail("taps");
            oracle_conv3d_direct(v, a, sh, w, r, w, r, w, r);
            if (oracle_conv3d_separable(v, b, sh, w, r, w, r, w, r) != 0) return fail("separable");
            for (int64_t i = 0; i < n; ++i)
                if (fabs(a[i] - b[i]) > 1e-12 * (1.0 + fabs(a[i]))) return fail("separable != direct");
            if (oracle_conv3d_transpose(v, c, sh, w, r, dw, r, w, r) != 0) return fail("transpose");
            for (int axis = 0; axis < 3; ++axis) {
                oracle_conv1d(v, a, sh, axis, w, r);
                oracle_conv1d_transpose(v, b, sh, axis, dw, r);
            }
            free(w);
            free(dw);
        }
        static const int radii[4][3] = {{1, 1, 1}, {2, 0, 3}, {4, 4, 4}, {3, 3, 3}};
        for (int k = 0; k < 4; ++k)
            for (int se = 0; se < 2; ++se) {
                if (se == 1 && !(radii[k][0] == radii[k][1] && radii[k][1] == radii[k][2])) continue;
                for (int op = 0; op < 2; ++op) {
                    if (oracle_morph3d(v, a, arg, sh, op, se, radii[k]) != 0) return fail("morph");
                    for (int64_t i = 0; i < n; ++i)
                        if ((op == 0 && a[i] > v[i]) || (op == 1 && a[i] < v[i])) return fail("morph order");
                    oracle_route(v, arg, b, n);
                }
            }
        oracle_threshold(v, a, n, 0.5);
        for (int64_t i = -3 * sh[2]; i < 3 * sh[2]; ++i) {
            const int64_t m = oracle_reflect(i, sh[2]);
            if (m < 0 || m >= sh[2]) return fail("reflect");
        }
        free(v);
        free(a);
        free(b);
        free(c);
        free(arg);
    }
    printf("ok\n");
    return 0;
}
