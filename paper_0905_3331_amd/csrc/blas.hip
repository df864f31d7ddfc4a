// blas.hip -- site-parallel vector kernels of the CG solvers and their scalars.
//
// One lane per lattice site (all 12 spin-colour components), so that the
// per-site scaled 16-bit formats can be decoded and re-encoded in registers.
// Grid: x over the sites, y over the RHS of the launch.  Every reduction
// writes one FP64 partial per block; a single-block-per-RHS scalar kernel
// sums the partials in a fixed order, which makes norms, inner products and
// therefore iteration counts bit-reproducible from run to run and
// independent of the batch an RHS is solved in.
#include "devutil.h"
#include "views.h"

namespace tmq {

int blas_grid(long n) { return (int)((n + BLAS_BLOCK - 1) / BLAS_BLOCK); }

RhsList rhs_all(int n)
{
    RhsList l;
    l.n = n < 0 ? 0 : (n > MAX_RHS ? MAX_RHS : n);
    for (int i = 0; i < l.n; i++) l.idx[i] = (unsigned char)i;
    return l;
}

template <typename R>
__device__ __forceinline__ R site_norm2(const spinor<R> &s)
{
    R n = R(0);
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) n += norm2(s.c[i][j]);
    return n;
}

// RHS of this block (grid y)
#define BLOCK_RHS(rl) const int rhs = (rl).idx[blockIdx.y]

#define WRITE_PARTIAL(ptr, pstride, part)                                   \
    {                                                                       \
        __shared__ double sh[BLAS_BLOCK / 64];                              \
        const double s_ = block_sum(part, sh);                              \
        if (threadIdx.x == 0) (ptr)[rhs * (pstride) + blockIdx.x] = s_;     \
    }

template <class F>
__global__ __launch_bounds__(BLAS_BLOCK) void k_norm2(BatchView<F> v, long n, RhsList rl, double *partial,
                                                      long pstride)
{
    using R = typename F::real;
    BLOCK_RHS(rl);
    const long h = (long)blockIdx.x * BLAS_BLOCK + threadIdx.x;
    double part = 0.0;
    if (h < n) {
        spinor<R> s;
        v.at(rhs).load(h, s);
        part = (double)site_norm2(s);
    }
    WRITE_PARTIAL(partial, pstride, part)
}

template <class FI, class FO>
__global__ __launch_bounds__(BLAS_BLOCK) void k_convert(BatchView<FI> in, BatchView<FO> out, long n, RhsList rl)
{
    using R = typename FI::real;
    BLOCK_RHS(rl);
    const long h = (long)blockIdx.x * BLAS_BLOCK + threadIdx.x;
    if (h < n) {
        spinor<R> s;
        in.at(rhs).load(h, s);
        out.at(rhs).store(h, s);
    }
}

template <class F>
__global__ __launch_bounds__(BLAS_BLOCK) void k_zero(BatchView<F> v, long n, RhsList rl)
{
    using R = typename F::real;
    BLOCK_RHS(rl);
    const long h = (long)blockIdx.x * BLAS_BLOCK + threadIdx.x;
    if (h < n) {
        spinor<R> s;
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int j = 0; j < 3; j++) s.c[i][j] = cx<R>{R(0), R(0)};
        v.at(rhs).store(h, s);
    }
}

// x += alpha p ; r -= alpha ap ; partial |r|^2
template <class FX, class F>
__global__ __launch_bounds__(BLAS_BLOCK) void k_axpy_norm(BatchView<FX> x, BatchView<F> p, BatchView<F> r,
                                                           BatchView<F> ap, long n, RhsList rl,
                                                           const CgScalars *sc, double *partial, long pstride,
                                                           int skip_done)
{
    using R = typename F::real;
    using RX = typename FX::real;
    BLOCK_RHS(rl);
    if (skip_done && sc[rhs].done) return;
    const double alpha = sc[rhs].alpha;
    const long h = (long)blockIdx.x * BLAS_BLOCK + threadIdx.x;
    double part = 0.0;
    if (h < n) {
        spinor<R> ps, rs, as;
        spinor<RX> xs;
        p.at(rhs).load(h, ps);
        r.at(rhs).load(h, rs);
        ap.at(rhs).load(h, as);
        x.at(rhs).load(h, xs);
        const R a = (R)alpha;
        const RX ax = (RX)alpha;
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int j = 0; j < 3; j++) {
                xs.c[i][j].re = fmad(ax, (RX)ps.c[i][j].re, xs.c[i][j].re);
                xs.c[i][j].im = fmad(ax, (RX)ps.c[i][j].im, xs.c[i][j].im);
                rs.c[i][j].re = fmad(-a, as.c[i][j].re, rs.c[i][j].re);
                rs.c[i][j].im = fmad(-a, as.c[i][j].im, rs.c[i][j].im);
            }
        x.at(rhs).store(h, xs);
        r.at(rhs).store(h, rs);
        part = (double)site_norm2(rs);
    }
    WRITE_PARTIAL(partial, pstride, part)
}

// out = cu * in on spins 0, 1 and cd * in on spins 2, 3 (a site-local
// a + i b gamma_5, FP64)
__global__ __launch_bounds__(BLAS_BLOCK) void k_twist(BatchView<SpF64> in, BatchView<SpF64> out, long n, RhsList rl,
                                                      double2 cu, double2 cd)
{
    BLOCK_RHS(rl);
    const long h = (long)blockIdx.x * BLAS_BLOCK + threadIdx.x;
    if (h < n) {
        spinor<double> s;
        in.at(rhs).load(h, s);
        const cx<double> u = {cu.x, cu.y}, d = {cd.x, cd.y};
#pragma unroll
        for (int c = 0; c < 3; c++) {
            s.c[0][c] = u * s.c[0][c];
            s.c[1][c] = u * s.c[1][c];
            s.c[2][c] = d * s.c[2][c];
            s.c[3][c] = d * s.c[3][c];
        }
        out.at(rhs).store(h, s);
    }
}

// p = r + beta p
template <class F>
__global__ __launch_bounds__(BLAS_BLOCK) void k_xpay(BatchView<F> r, BatchView<F> p, long n, RhsList rl,
                                                     const CgScalars *sc, int skip_done)
{
    using R = typename F::real;
    BLOCK_RHS(rl);
    if (skip_done && sc[rhs].done) return;
    const R b = (R)sc[rhs].beta;
    const long h = (long)blockIdx.x * BLAS_BLOCK + threadIdx.x;
    if (h < n) {
        spinor<R> rs, ps;
        r.at(rhs).load(h, rs);
        p.at(rhs).load(h, ps);
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int j = 0; j < 3; j++) {
                ps.c[i][j].re = fmad(b, ps.c[i][j].re, rs.c[i][j].re);
                ps.c[i][j].im = fmad(b, ps.c[i][j].im, rs.c[i][j].im);
            }
        p.at(rhs).store(h, ps);
    }
}

__global__ __launch_bounds__(BLAS_BLOCK) void k_residual(BatchView<SpF64> b, BatchView<SpF64> ax,
                                                         BatchView<SpF64> r, long n, RhsList rl, double *partial,
                                                         long pstride)
{
    BLOCK_RHS(rl);
    const long h = (long)blockIdx.x * BLAS_BLOCK + threadIdx.x;
    double part = 0.0;
    if (h < n) {
        spinor<double> bs, as;
        b.at(rhs).load(h, bs);
        ax.at(rhs).load(h, as);
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int j = 0; j < 3; j++) bs.c[i][j] = bs.c[i][j] - as.c[i][j];
        r.at(rhs).store(h, bs);
        part = site_norm2(bs);
    }
    WRITE_PARTIAL(partial, pstride, part)
}

template <class FS>
__global__ __launch_bounds__(BLAS_BLOCK) void k_accumulate(BatchView<SpF64> x, BatchView<FS> xs, long n,
                                                           RhsList rl)
{
    using RS = typename FS::real;
    BLOCK_RHS(rl);
    const long h = (long)blockIdx.x * BLAS_BLOCK + threadIdx.x;
    if (h < n) {
        spinor<double> a;
        spinor<RS> d, z;
        x.at(rhs).load(h, a);
        xs.at(rhs).load(h, d);
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int j = 0; j < 3; j++) {
                a.c[i][j].re += (double)d.c[i][j].re;
                a.c[i][j].im += (double)d.c[i][j].im;
                z.c[i][j] = cx<RS>{RS(0), RS(0)};
            }
        x.at(rhs).store(h, a);
        xs.at(rhs).store(h, z);
    }
}

// ------------------------------------------------------------- scalars

constexpr int SC_THREADS = 1024;

__device__ __forceinline__ double det_sum(const double *partial, int n, double *sh)
{
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += SC_THREADS) v += partial[i];
    return block_sum(v, sh);  // valid in thread 0
}

__device__ __forceinline__ int finite(double v) { return isfinite(v) ? 1 : 0; }

// one block per RHS of rl (grid x)
__global__ __launch_bounds__(SC_THREADS) void k_scalar(int op, RhsList rl, const double *partial, long pstride,
                                                       int nparts, CgScalars *sc, double tol2, int relative,
                                                       int skip_done, CgScalars *publish)
{
    const int rhs = rl.idx[blockIdx.x];
    CgScalars *s = sc + rhs;
    if (skip_done && s->done) {
        if (publish && threadIdx.x == 0) publish[rhs] = *s;
        return;
    }
    __shared__ double sh[SC_THREADS / 64];
    const double sum = det_sum(partial + rhs * pstride, nparts, sh);
    if (threadIdx.x != 0) return;
    switch (op) {
    case SC_INIT:  // sum = ||b||^2 = ||r_0||^2 (x_0 = 0)
        s->bb = sum;
        s->rr = s->rr_prev = sum;
        s->target = tol2 * (relative ? sum : 1.0);
        s->alpha = s->beta = s->pAp = 0.0;
        s->iter = 0;
        s->reliable = 0;
        s->last_true = 1;
        s->nan = !finite(sum);
        s->done = (sum < s->target || sum == 0.0 || s->nan) ? 1 : 0;
        break;
    case SC_ALPHA:  // sum = <p, A p>
        s->pAp = sum;
        s->alpha = s->rr / sum;
        if (!finite(s->alpha)) s->nan = 1, s->done = 1;
        break;
    case SC_BETA:  // sum = ||r||^2 of the updated iterated residual
        s->rr_prev = s->rr;
        s->rr = sum;
        s->beta = sum / s->rr_prev;
        s->iter += 1;
        s->last_true = 0;
        if (!finite(sum) || !finite(s->beta)) s->nan = 1;
        s->done = (sum < s->target || s->nan) ? 1 : 0;
        break;
    case SC_RELIABLE:  // sum = ||b - A x||^2 recomputed in FP64; replaces the iterated residual
        s->rr = sum;
        s->beta = s->rr_prev > 0.0 ? sum / s->rr_prev : 0.0;
        s->reliable += 1;
        s->last_true = 1;
        if (!finite(sum)) s->nan = 1;
        s->done = (sum < s->target || sum == 0.0 || s->nan) ? 1 : 0;
        break;
    }
    if (publish) publish[rhs] = *s;
}

constexpr int SUM_THREADS = 1024;

__global__ __launch_bounds__(SUM_THREADS) void k_max(const double *partial, int n, double *out)
{
    __shared__ double sh[SUM_THREADS / 64];
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += SUM_THREADS) v = fmax(v, partial[i]);
    const double m = block_max(v, sh);
    if (threadIdx.x == 0) *out = m;
}

// plain streaming copy, 16 bytes per lane, for bandwidth calibration
__global__ __launch_bounds__(256) void k_stream_copy(const float4 *__restrict__ a, float4 *__restrict__ b, long n)
{
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) b[i] = a[i];
}

// ------------------------------------------------------------- dispatch

#define DISPATCH_SP TMQ_DISPATCH_SP

static dim3 grid2(long n, const RhsList &rl) { return dim3((unsigned)blas_grid(n), (unsigned)rl.n); }

#define LAUNCH(KERNEL, NSITES, RL, STREAM, ...)                                                          \
    do {                                                                                                  \
        if ((RL).n > 0 && (NSITES) > 0)                                                                   \
            hipLaunchKernelGGL(KERNEL, grid2(NSITES, RL), dim3(BLAS_BLOCK), 0, STREAM, __VA_ARGS__);      \
    } while (0)

hipError_t launch_norm2(const FieldDesc &v, const RhsList &rl, double *partial, long pstride, hipStream_t st)
{
    DISPATCH_SP(v.prec, F, LAUNCH(k_norm2<F>, v.n, rl, st, make_bv<F>(v), v.n, rl, partial, pstride));
    return hipGetLastError();
}

hipError_t launch_zero(const FieldDesc &v, const RhsList &rl, hipStream_t st)
{
    DISPATCH_SP(v.prec, F, LAUNCH(k_zero<F>, v.n, rl, st, make_bv<F>(v), v.n, rl));
    return hipGetLastError();
}

hipError_t launch_twist(const FieldDesc &in, const FieldDesc &out, const RhsList &rl, double2 cu, double2 cd,
                        hipStream_t st)
{
    if (in.prec != P64 || out.prec != P64 || in.n != out.n) return hipErrorInvalidValue;
    LAUNCH(k_twist, in.n, rl, st, make_bv<SpF64>(in), make_bv<SpF64>(out), in.n, rl, cu, cd);
    return hipGetLastError();
}

hipError_t launch_convert(const FieldDesc &in, const FieldDesc &out, const RhsList &rl, hipStream_t st)
{
    if (in.n != out.n) return hipErrorInvalidValue;
    DISPATCH_SP(in.prec, FI,
                DISPATCH_SP(out.prec, FO,
                            LAUNCH((k_convert<FI, FO>), in.n, rl, st, make_bv<FI>(in), make_bv<FO>(out), in.n, rl)));
    return hipGetLastError();
}

hipError_t launch_axpy_norm(const FieldDesc &x, const FieldDesc &p, const FieldDesc &r, const FieldDesc &ap,
                            const RhsList &rl, const CgScalars *s, double *partial, long pstride, bool skip_done,
                            hipStream_t st)
{
    if (p.prec != r.prec || p.prec != ap.prec) return hipErrorInvalidValue;
    const long n = p.n;
    const int sk = skip_done ? 1 : 0;
    if (x.prec == P64 && p.prec == P64)
        LAUNCH((k_axpy_norm<SpF64, SpF64>), n, rl, st, make_bv<SpF64>(x), make_bv<SpF64>(p), make_bv<SpF64>(r),
               make_bv<SpF64>(ap), n, rl, s, partial, pstride, sk);
    else if (x.prec == P32) {
        DISPATCH_SP(p.prec, F,
                    LAUNCH((k_axpy_norm<SpF32, F>), n, rl, st, make_bv<SpF32>(x), make_bv<F>(p), make_bv<F>(r),
                           make_bv<F>(ap), n, rl, s, partial, pstride, sk));
    } else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_xpay(const FieldDesc &r, const FieldDesc &p, const RhsList &rl, const CgScalars *s,
                       bool skip_done, hipStream_t st)
{
    if (r.prec != p.prec) return hipErrorInvalidValue;
    DISPATCH_SP(p.prec, F,
                LAUNCH(k_xpay<F>, p.n, rl, st, make_bv<F>(r), make_bv<F>(p), p.n, rl, s, skip_done ? 1 : 0));
    return hipGetLastError();
}

hipError_t launch_residual(const FieldDesc &b, const FieldDesc &ax, const FieldDesc &r, const RhsList &rl,
                           double *partial, long pstride, hipStream_t st)
{
    if (b.prec != P64 || ax.prec != P64 || r.prec != P64) return hipErrorInvalidValue;
    LAUNCH(k_residual, b.n, rl, st, make_bv<SpF64>(b), make_bv<SpF64>(ax), make_bv<SpF64>(r), b.n, rl, partial,
           pstride);
    return hipGetLastError();
}

hipError_t launch_accumulate(const FieldDesc &x64, const FieldDesc &xs, const RhsList &rl, hipStream_t st)
{
    if (x64.prec != P64) return hipErrorInvalidValue;
    DISPATCH_SP(xs.prec, F,
                LAUNCH(k_accumulate<F>, x64.n, rl, st, make_bv<SpF64>(x64), make_bv<F>(xs), x64.n, rl));
    return hipGetLastError();
}

hipError_t launch_scalar(int op, const RhsList &rl, const double *partial, long pstride, int nparts,
                         CgScalars *s, double tol2, int relative, bool skip_done, CgScalars *publish,
                         hipStream_t st)
{
    if (rl.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scalar, dim3(rl.n), dim3(SC_THREADS), 0, st, op, rl, partial, pstride, nparts, s, tol2,
                       relative, skip_done ? 1 : 0, publish);
    return hipGetLastError();
}

hipError_t launch_max(const double *partial, int n, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_max, dim3(1), dim3(SUM_THREADS), 0, st, partial, n, out);
    return hipGetLastError();
}

hipError_t launch_stream_copy(const void *src, void *dst, size_t bytes, hipStream_t st)
{
    const long n = (long)(bytes / 16);
    hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, (const float4 *)src,
                       (float4 *)dst, n);
    return hipGetLastError();
}

FieldDesc field_sub(const FieldDesc &f, long off, long n)
{
    FieldDesc o = f;
    o.data = (char *)f.data + off * (long)field_blocks(f.prec) * (long)field_elem_bytes(f.prec);
    o.scale = f.scale ? f.scale + off : nullptr;
    o.n = n;
    return o;
}

FieldDesc field_rhs(const FieldDesc &f, int r)
{
    FieldDesc o = f;
    o.data = (char *)f.data + (long)r * f.rhs_elems * (long)field_elem_bytes(f.prec);
    o.scale = f.scale ? f.scale + (long)r * f.rhs_sites : nullptr;
    o.nrhs = 1;
    return o;
}

size_t field_elem_bytes(int) { return 16; }  // double2, float4, uint4
int field_blocks(int prec) { return prec == P64 ? 12 : prec == P32 ? 6 : 3; }

}  // namespace tmq
