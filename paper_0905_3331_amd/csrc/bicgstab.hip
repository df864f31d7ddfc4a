// bicgstab.hip -- vector and scalar kernels of BiCGstab on an odd-site system.
//
// BiCGstab (one of the solvers the paper lists for D chi = phi, Sec. 4.4;
// van der Vorst's algorithm) solves Qhat^{+-} x = b with the operator itself,
// two applications per iteration, instead of CG on the normal equations.
// Complex scalars live on the device and are formed from per-block FP64
// partial sums in a fixed order, as for CG; every kernel of an iteration does
// nothing once the device has flagged the solve done, so the host can enqueue
// an iteration before it has read whether the previous one converged.
// Inner products are <a, b> = sum conj(a) b.  FP64 fields, one right-hand side.
#include "devutil.h"
#include "views.h"

namespace tmq {

namespace {

// per-block sums of up to three reals (written to three partial arrays)
__device__ __forceinline__ void write3(double a, double b, double c, double *pa, double *pb, double *pc)
{
    __shared__ double sh[3][BLAS_BLOCK / 64];
    const double sa = block_sum(a, sh[0]);
    const double sb = block_sum(b, sh[1]);
    const double sc = block_sum(c, sh[2]);
    if (threadIdx.x == 0) {
        if (pa) pa[blockIdx.x] = sa;
        if (pb) pb[blockIdx.x] = sb;
        if (pc) pc[blockIdx.x] = sc;
    }
}

__device__ __forceinline__ cx<double> cplx(const double (&v)[2]) { return {v[0], v[1]}; }

// <a, b> accumulated over one site, and |w|^2 of w (a or b)
__device__ __forceinline__ void site_dot(const spinor<double> &a, const spinor<double> &b, const spinor<double> &w,
                                        double &re, double &im, double &nw)
{
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int c = 0; c < 3; c++) {
            const cx<double> x = a.c[i][c], y = b.c[i][c], z = w.c[i][c];
            re = fmad(x.re, y.re, fmad(x.im, y.im, re));
            im = fmad(x.re, y.im, fmad(-x.im, y.re, im));
            nw = fmad(z.re, z.re, fmad(z.im, z.im, nw));
        }
}

}  // namespace

// <a, b> -> partial 0 (re), 1 (im); |a|^2 -> partial 2
__global__ __launch_bounds__(BLAS_BLOCK) void k_bi_dot(SpF64 a, SpF64 b, long n, const BicgScalars *sc,
                                                      double *p0, double *p1, double *p2)
{
    if (sc && sc->done) return;
    const long h = (long)blockIdx.x * BLAS_BLOCK + threadIdx.x;
    double re = 0.0, im = 0.0, nb = 0.0;
    if (h < n) {
        spinor<double> x, y;
        a.load(h, x);
        b.load(h, y);
        site_dot(x, y, x, re, im, nb);
    }
    write3(re, im, nb, p0, p1, p2);
}

// p = r + beta (p - omega v)
__global__ __launch_bounds__(BLAS_BLOCK) void k_bi_p(SpF64 r, SpF64 p, SpF64 v, long n, const BicgScalars *sc)
{
    if (sc->done) return;
    const long h = (long)blockIdx.x * BLAS_BLOCK + threadIdx.x;
    if (h >= n) return;
    const cx<double> be = cplx(sc->beta), om = cplx(sc->omega);
    spinor<double> rs, ps, vs;
    r.load(h, rs);
    p.load(h, ps);
    v.load(h, vs);
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int c = 0; c < 3; c++) {
            const cx<double> w = fma(-om, vs.c[i][c], ps.c[i][c]);
            ps.c[i][c] = fma(be, w, rs.c[i][c]);
        }
    p.store(h, ps);
}

// s = r - alpha v
__global__ __launch_bounds__(BLAS_BLOCK) void k_bi_s(SpF64 r, SpF64 v, SpF64 s, long n, const BicgScalars *sc)
{
    if (sc->done) return;
    const long h = (long)blockIdx.x * BLAS_BLOCK + threadIdx.x;
    if (h >= n) return;
    const cx<double> al = cplx(sc->alpha);
    spinor<double> rs, vs;
    r.load(h, rs);
    v.load(h, vs);
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int c = 0; c < 3; c++) rs.c[i][c] = fma(-al, vs.c[i][c], rs.c[i][c]);
    s.store(h, rs);
}

// x += alpha p + omega s ; r = s - omega t ; partials <rhat, r> (0, 1) and |r|^2 (2)
__global__ __launch_bounds__(BLAS_BLOCK) void k_bi_xr(SpF64 x, SpF64 p, SpF64 s, SpF64 t, SpF64 r, SpF64 rhat,
                                                     long n, const BicgScalars *sc, double *p0, double *p1,
                                                     double *p2)
{
    if (sc->done) return;
    const long h = (long)blockIdx.x * BLAS_BLOCK + threadIdx.x;
    double re = 0.0, im = 0.0, nr = 0.0;
    if (h < n) {
        const cx<double> al = cplx(sc->alpha), om = cplx(sc->omega);
        spinor<double> xs, ps, ss, ts, rh;
        x.load(h, xs);
        p.load(h, ps);
        s.load(h, ss);
        t.load(h, ts);
        rhat.load(h, rh);
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int c = 0; c < 3; c++) {
                xs.c[i][c] = fma(om, ss.c[i][c], fma(al, ps.c[i][c], xs.c[i][c]));
                ts.c[i][c] = fma(-om, ts.c[i][c], ss.c[i][c]);  // the new r
            }
        x.store(h, xs);
        r.store(h, ts);
        site_dot(rh, ts, ts, re, im, nr);
    }
    write3(re, im, nr, p0, p1, p2);
}

constexpr int BI_THREADS = 1024;

__device__ __forceinline__ double bi_sum(const double *partial, int n, double *sh)
{
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += BI_THREADS) v += partial[i];
    return block_sum(v, sh);
}

__device__ __forceinline__ cx<double> cdiv(cx<double> a, cx<double> b)
{
    const double d = b.re * b.re + b.im * b.im;
    return {(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}

__global__ __launch_bounds__(BI_THREADS) void k_bi_scalar(int op, const double *p0, const double *p1,
                                                         const double *p2, int nparts, BicgScalars *s, double tol2,
                                                         int relative, BicgScalars *publish)
{
    if (op != BI_START && s->done) {
        if (publish && threadIdx.x == 0) *publish = *s;
        return;
    }
    __shared__ double sh[3][BI_THREADS / 64];
    const double a = bi_sum(p0, nparts, sh[0]);
    const double b = bi_sum(p1, nparts, sh[1]);
    const double c = bi_sum(p2, nparts, sh[2]);
    if (threadIdx.x != 0) return;
    const cx<double> dot = {a, b};
    switch (op) {
    case BI_START:  // r = rhat: <rhat, r> = |r|^2 = c ; a restart keeps |b|^2 and the counters
        if (s->iter == 0 && s->restarts == 0) {
            s->bb = c;
            s->target = tol2 * (relative ? c : 1.0);
        }
        s->rr = c;
        s->rho[0] = a, s->rho[1] = b;
        s->alpha[0] = 1.0, s->alpha[1] = 0.0;
        s->omega[0] = 1.0, s->omega[1] = 0.0;
        s->beta[0] = 0.0, s->beta[1] = 0.0;
        s->breakdown = 0;
        s->nan = isfinite(c) ? 0 : 1;
        s->done = (c < s->target || c == 0.0 || s->nan) ? 1 : 0;
        break;
    case BI_ALPHA: {  // <rhat, v>
        if (dot.re == 0.0 && dot.im == 0.0) {
            s->breakdown = 1, s->done = 1;
            break;
        }
        const cx<double> al = cdiv(cplx(s->rho), dot);
        s->alpha[0] = al.re, s->alpha[1] = al.im;
        if (!isfinite(al.re) || !isfinite(al.im)) s->nan = 1, s->done = 1;
        break;
    }
    case BI_OMEGA: {  // <t, s> and |t|^2
        const cx<double> om = c > 0.0 ? cx<double>{a / c, b / c} : cx<double>{0.0, 0.0};
        s->omega[0] = om.re, s->omega[1] = om.im;
        if (!isfinite(om.re) || !isfinite(om.im)) s->nan = 1, s->done = 1;
        break;
    }
    case BI_UPDATE: {  // <rhat, r> and |r|^2 of the new residual
        s->rr = c;
        s->iter += 1;
        if (s->iter >= s->max_iter) s->done = 1;
        if (!isfinite(c) || !isfinite(a) || !isfinite(b)) {
            s->nan = 1, s->done = 1;
            break;
        }
        if (c < s->target) {
            s->done = 1;
            break;
        }
        const cx<double> om = cplx(s->omega);
        if ((om.re == 0.0 && om.im == 0.0) || (dot.re == 0.0 && dot.im == 0.0)) {
            s->breakdown = 1, s->done = 1;
            break;
        }
        const cx<double> be = cdiv(dot, cplx(s->rho)) * cdiv(cplx(s->alpha), om);
        s->beta[0] = be.re, s->beta[1] = be.im;
        s->rho[0] = dot.re, s->rho[1] = dot.im;
        break;
    }
    }
    if (publish) *publish = *s;
}

hipError_t launch_bi_dot(const FieldDesc &a, const FieldDesc &b, const BicgScalars *sc, double *p0, double *p1,
                         double *p2, hipStream_t st)
{
    if (a.prec != P64 || b.prec != P64 || a.n != b.n) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_bi_dot, dim3(blas_grid(a.n)), dim3(BLAS_BLOCK), 0, st, make_sp<SpF64>(a),
                       make_sp<SpF64>(b), a.n, sc, p0, p1, p2);
    return hipGetLastError();
}

hipError_t launch_bi_p(const FieldDesc &r, const FieldDesc &p, const FieldDesc &v, const BicgScalars *sc,
                       hipStream_t st)
{
    hipLaunchKernelGGL(k_bi_p, dim3(blas_grid(r.n)), dim3(BLAS_BLOCK), 0, st, make_sp<SpF64>(r), make_sp<SpF64>(p),
                       make_sp<SpF64>(v), r.n, sc);
    return hipGetLastError();
}

hipError_t launch_bi_s(const FieldDesc &r, const FieldDesc &v, const FieldDesc &s, const BicgScalars *sc,
                       hipStream_t st)
{
    hipLaunchKernelGGL(k_bi_s, dim3(blas_grid(r.n)), dim3(BLAS_BLOCK), 0, st, make_sp<SpF64>(r), make_sp<SpF64>(v),
                       make_sp<SpF64>(s), r.n, sc);
    return hipGetLastError();
}

hipError_t launch_bi_xr(const FieldDesc &x, const FieldDesc &p, const FieldDesc &s, const FieldDesc &t,
                        const FieldDesc &r, const FieldDesc &rhat, const BicgScalars *sc, double *p0, double *p1,
                        double *p2, hipStream_t st)
{
    hipLaunchKernelGGL(k_bi_xr, dim3(blas_grid(r.n)), dim3(BLAS_BLOCK), 0, st, make_sp<SpF64>(x), make_sp<SpF64>(p),
                       make_sp<SpF64>(s), make_sp<SpF64>(t), make_sp<SpF64>(r), make_sp<SpF64>(rhat), r.n, sc, p0,
                       p1, p2);
    return hipGetLastError();
}

hipError_t launch_bi_scalar(int op, const double *p0, const double *p1, const double *p2, int nparts,
                            BicgScalars *s, double tol2, int relative, BicgScalars *publish, hipStream_t st)
{
    hipLaunchKernelGGL(k_bi_scalar, dim3(1), dim3(BI_THREADS), 0, st, op, p0, p1, p2, nparts, s, tol2, relative,
                       publish);
    return hipGetLastError();
}

}  // namespace tmq
