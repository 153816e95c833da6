// The Hessian's two three-component passes, float32 input.
#include "hess_impl.h"

namespace harpia {

bool launch_hessian_fused(const ChunkArgs &a, harpia_dtype in_t, const double sigma[3], const int r[3],
                          int64_t cstride, hipStream_t s)
{
    if (in_t != HARPIA_F32 || !(r[0] == r[1] && r[1] == r[2])) return false;
    if (r[0] < 1 || r[0] > gauss_detail::kHessMaxR || !gauss_detail::fused_ok_extent(a)) return false;
    gauss_detail::HessTaps ht;
    static const int ord[3][3] = {{0, 0, 0}, {1, 1, 1}, {2, 2, 2}};
    GaussTaps t[3];
    for (int o = 0; o < 3; ++o) make_gauss_deriv_taps(sigma, r, ord[o], t[o]);
    for (int ax = 0; ax < 3; ++ax)
        for (int k = 0; k <= gauss_detail::kHessMaxR; ++k) {
            ht.g[ax][k] = t[0].w[ax][k];
            ht.d1[ax][k] = t[1].w[ax][k];
            ht.d2[ax][k] = t[2].w[ax][k];
        }
    return hess_run<float>(a, ht, r[0], cstride, s);
}

}  // namespace harpia
