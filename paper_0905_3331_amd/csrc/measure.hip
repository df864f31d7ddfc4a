// measure.hip -- contractions of solver output (consumers of the solver).
//
// Time-slice sums of spin bilinears psi^+ Gamma psi of a full-lattice field,
// the contraction of the one-end-trick correlators of the online
// measurements (eqs. (source), (oneend)): with phi = M^-1 xi for a noise
// source xi on one time slice, sum over the spatial sites of phi^+ Gamma phi
// estimates tr[G G^+ Gamma]-type correlators.
#include "devutil.h"
#include "views.h"

namespace tmq {

// One thread per site of the slice (12 complex loaded contiguously); grid
// (blocks per slice, T); per-block partial sums of the real and imaginary
// parts at pre / pim [t * gridDim.x + block].
__global__ __launch_bounds__(BLAS_BLOCK) void k_ts_bilinear(const double2 *psi, long S, SpinMat g, double *pre,
                                                           double *pim)
{
    const int t = blockIdx.y;
    double re = 0.0, im = 0.0;
    for (long i = (long)blockIdx.x * BLAS_BLOCK + threadIdx.x; i < S; i += (long)gridDim.x * BLAS_BLOCK) {
        const double2 *q = psi + ((long)t * S + i) * 12;
        cx<double> v[4][3];
#pragma unroll
        for (int k = 0; k < 12; k++) v[k / 3][k % 3] = cx<double>{q[k].x, q[k].y};
#pragma unroll
        for (int c = 0; c < 3; c++)
#pragma unroll
            for (int s = 0; s < 4; s++) {
                cx<double> w = {0.0, 0.0};
#pragma unroll
                for (int u = 0; u < 4; u++) w = fma(cx<double>{g.m[s][u].x, g.m[s][u].y}, v[u][c], w);
                // conj(v) w
                re = fmad(v[s][c].re, w.re, fmad(v[s][c].im, w.im, re));
                im = fmad(v[s][c].re, w.im, fmad(-v[s][c].im, w.re, im));
            }
    }
    __shared__ double sh[2][BLAS_BLOCK / 64];
    const double a = block_sum(re, sh[0]);
    const double b = block_sum(im, sh[1]);
    if (threadIdx.x == 0) {
        pre[(long)t * gridDim.x + blockIdx.x] = a;
        pim[(long)t * gridDim.x + blockIdx.x] = b;
    }
}

int ts_bilinear_blocks(const Geom &g)
{
    const long S = (long)g.LZ * g.LY * g.LX;
    const long nb = (S + BLAS_BLOCK - 1) / BLAS_BLOCK;
    return (int)(nb < 64 ? nb : 64);
}

hipError_t launch_ts_bilinear(const Geom &g, const double2 *psi, const SpinMat &m, double *pre, double *pim,
                              hipStream_t st)
{
    const long S = (long)g.LZ * g.LY * g.LX;
    hipLaunchKernelGGL(k_ts_bilinear, dim3(ts_bilinear_blocks(g), g.T), dim3(BLAS_BLOCK), 0, st, psi, S, m, pre, pim);
    return hipGetLastError();
}

}  // namespace tmq
