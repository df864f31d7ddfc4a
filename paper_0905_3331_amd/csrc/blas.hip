// blas.hip -- site-parallel vector kernels of the CG solvers and their scalars.
//
// One lane per lattice site (all 12 spin-colour components), so that the
// per-site scaled 16-bit formats can be decoded and re-encoded in registers.
// Every reduction writes one FP64 partial per block; a single-block scalar
// kernel sums the partials in a fixed order, which makes norms, inner products
// and therefore iteration counts bit-reproducible from run to run.
#include "devutil.h"
#include "views.h"

namespace tmq {

int blas_grid(long n) { return (int)((n + BLAS_BLOCK - 1) / BLAS_BLOCK); }

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

#define SITE_LOOP_BEGIN                                   \
    const long h = (long)blockIdx.x * BLAS_BLOCK + threadIdx.x; \
    double part = 0.0;                                    \
    if (h < n) {
#define SITE_LOOP_END }

#define WRITE_PARTIAL(ptr)                                \
    {                                                     \
        __shared__ double sh[BLAS_BLOCK / 64];            \
        double s_ = block_sum(part, sh);                  \
        if (threadIdx.x == 0) (ptr)[blockIdx.x] = s_;     \
    }

template <class F>
__global__ __launch_bounds__(BLAS_BLOCK) void k_norm2(F v, long n, double *partial)
{
    using R = typename F::real;
    SITE_LOOP_BEGIN
    spinor<R> s;
    v.load(h, s);
    part = (double)site_norm2(s);
    SITE_LOOP_END
    WRITE_PARTIAL(partial)
}

template <class FI, class FO>
__global__ __launch_bounds__(BLAS_BLOCK) void k_convert(FI in, FO out, long n)
{
    using R = typename FI::real;
    const long h = (long)blockIdx.x * BLAS_BLOCK + threadIdx.x;
    if (h < n) {
        spinor<R> s;
        in.load(h, s);
        out.store(h, s);
    }
}

template <class F>
__global__ __launch_bounds__(BLAS_BLOCK) void k_zero(F v, long n)
{
    using R = typename F::real;
    const long h = (long)blockIdx.x * BLAS_BLOCK + threadIdx.x;
    if (h < n) {
        spinor<R> s;
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int j = 0; j < 3; j++) s.c[i][j] = cx<R>{R(0), R(0)};
        v.store(h, s);
    }
}

// x += alpha p ; r -= alpha ap ; partial |r|^2
template <class FX, class F>
__global__ __launch_bounds__(BLAS_BLOCK) void k_axpy_norm(FX x, F p, F r, F ap, long n, const CgScalars *sc,
                                                           double *partial, const int *skip)
{
    using R = typename F::real;
    using RX = typename FX::real;
    if (skip && *skip) return;
    const double alpha = sc->alpha;
    SITE_LOOP_BEGIN
    spinor<R> ps, rs, as;
    spinor<RX> xs;
    p.load(h, ps);
    r.load(h, rs);
    ap.load(h, as);
    x.load(h, xs);
    const R a = (R)alpha;
    const RX ax = (RX)alpha;
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            xs.c[i][j].re += ax * (RX)ps.c[i][j].re;
            xs.c[i][j].im += ax * (RX)ps.c[i][j].im;
            rs.c[i][j].re -= a * as.c[i][j].re;
            rs.c[i][j].im -= a * as.c[i][j].im;
        }
    x.store(h, xs);
    r.store(h, rs);
    part = (double)site_norm2(rs);
    SITE_LOOP_END
    WRITE_PARTIAL(partial)
}

// p = r + beta p
template <class F>
__global__ __launch_bounds__(BLAS_BLOCK) void k_xpay(F r, F p, long n, const CgScalars *sc, const int *skip)
{
    using R = typename F::real;
    if (skip && *skip) return;
    const R b = (R)sc->beta;
    const long h = (long)blockIdx.x * BLAS_BLOCK + threadIdx.x;
    if (h < n) {
        spinor<R> rs, ps;
        r.load(h, rs);
        p.load(h, ps);
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int j = 0; j < 3; j++) {
                ps.c[i][j].re = rs.c[i][j].re + b * ps.c[i][j].re;
                ps.c[i][j].im = rs.c[i][j].im + b * ps.c[i][j].im;
            }
        p.store(h, ps);
    }
}

__global__ __launch_bounds__(BLAS_BLOCK) void k_residual(SpF64 b, SpF64 ax, SpF64 r, long n, double *partial)
{
    SITE_LOOP_BEGIN
    spinor<double> bs, as;
    b.load(h, bs);
    ax.load(h, as);
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) bs.c[i][j] = bs.c[i][j] - as.c[i][j];
    r.store(h, bs);
    part = site_norm2(bs);
    SITE_LOOP_END
    WRITE_PARTIAL(partial)
}

template <class FS>
__global__ __launch_bounds__(BLAS_BLOCK) void k_accumulate(SpF64 x, FS xs, long n)
{
    using RS = typename FS::real;
    const long h = (long)blockIdx.x * BLAS_BLOCK + threadIdx.x;
    if (h < n) {
        spinor<double> a;
        spinor<RS> d, z;
        x.load(h, a);
        xs.load(h, d);
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int j = 0; j < 3; j++) {
                a.c[i][j].re += (double)d.c[i][j].re;
                a.c[i][j].im += (double)d.c[i][j].im;
                z.c[i][j] = cx<RS>{RS(0), RS(0)};
            }
        x.store(h, a);
        xs.store(h, z);
    }
}

__global__ __launch_bounds__(BLAS_BLOCK) void k_axpy_host(double a, SpF64 x, SpF64 y, long n)
{
    const long h = (long)blockIdx.x * BLAS_BLOCK + threadIdx.x;
    if (h < n) {
        spinor<double> xs, ys;
        x.load(h, xs);
        y.load(h, ys);
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int j = 0; j < 3; j++) {
                ys.c[i][j].re += a * xs.c[i][j].re;
                ys.c[i][j].im += a * xs.c[i][j].im;
            }
        y.store(h, ys);
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

// publish != nullptr: thread 0 finally copies the scalars to that (host-mapped)
// slot, also when the kernel is skipped, so the host always sees the state.
__global__ __launch_bounds__(SC_THREADS) void k_scalar(int op, const double *partial, int n, CgScalars *s,
                                                       double tol2, int relative, const int *skip,
                                                       CgScalars *publish)
{
    if (skip && *skip) {
        if (publish && threadIdx.x == 0) *publish = *s;
        return;
    }
    __shared__ double sh[SC_THREADS / 64];
    const double sum = det_sum(partial, n, sh);
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
    if (publish) *publish = *s;
}

constexpr int SUM_THREADS = 1024;

__global__ __launch_bounds__(SUM_THREADS) void k_sum(const double *partial, int n, double *out)
{
    __shared__ double sh[SUM_THREADS / 64];
    const double s = det_sum(partial, n, sh);
    if (threadIdx.x == 0) *out = s;
}

__global__ __launch_bounds__(SUM_THREADS) void k_max(const double *partial, int n, double *out)
{
    __shared__ double sh[SUM_THREADS / 64];
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += SUM_THREADS) v = fmax(v, partial[i]);
    const double m = block_max(v, sh);
    if (threadIdx.x == 0) *out = m;
}

// ------------------------------------------------------------- dispatch

#define DISPATCH_SP TMQ_DISPATCH_SP

#define LAUNCH(kernel, n, st, ...) \
    hipLaunchKernelGGL(kernel, dim3(blas_grid(n)), dim3(BLAS_BLOCK), 0, st, __VA_ARGS__)

hipError_t launch_norm2(const FieldDesc &v, double *partial, hipStream_t st)
{
    DISPATCH_SP(v.prec, F, LAUNCH(k_norm2<F>, v.n, st, make_sp<F>(v), v.n, partial));
    return hipGetLastError();
}

hipError_t launch_zero(const FieldDesc &v, hipStream_t st)
{
    DISPATCH_SP(v.prec, F, LAUNCH(k_zero<F>, v.n, st, make_sp<F>(v), v.n));
    return hipGetLastError();
}

hipError_t launch_convert(const FieldDesc &in, const FieldDesc &out, hipStream_t st)
{
    if (in.n != out.n) return hipErrorInvalidValue;
    DISPATCH_SP(in.prec, FI, DISPATCH_SP(out.prec, FO, LAUNCH((k_convert<FI, FO>), in.n, st, make_sp<FI>(in), make_sp<FO>(out), in.n)));
    return hipGetLastError();
}

hipError_t launch_axpy_norm(const FieldDesc &x, const FieldDesc &p, const FieldDesc &r, const FieldDesc &ap,
                            const CgScalars *s, double *partial, const int *skip, hipStream_t st)
{
    if (p.prec != r.prec || p.prec != ap.prec) return hipErrorInvalidValue;
    const long n = p.n;
    if (x.prec == P64 && p.prec == P64)
        LAUNCH((k_axpy_norm<SpF64, SpF64>), n, st, make_sp<SpF64>(x), make_sp<SpF64>(p), make_sp<SpF64>(r), make_sp<SpF64>(ap), n, s, partial, skip);
    else if (x.prec == P32) {
        DISPATCH_SP(p.prec, F, LAUNCH((k_axpy_norm<SpF32, F>), n, st, make_sp<SpF32>(x), make_sp<F>(p), make_sp<F>(r), make_sp<F>(ap), n, s, partial, skip));
    } else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_xpay(const FieldDesc &r, const FieldDesc &p, const CgScalars *s, const int *skip, hipStream_t st)
{
    if (r.prec != p.prec) return hipErrorInvalidValue;
    DISPATCH_SP(p.prec, F, LAUNCH(k_xpay<F>, p.n, st, make_sp<F>(r), make_sp<F>(p), p.n, s, skip));
    return hipGetLastError();
}

hipError_t launch_residual(const FieldDesc &b, const FieldDesc &ax, const FieldDesc &r, double *partial,
                           hipStream_t st)
{
    if (b.prec != P64 || ax.prec != P64 || r.prec != P64) return hipErrorInvalidValue;
    LAUNCH(k_residual, b.n, st, make_sp<SpF64>(b), make_sp<SpF64>(ax), make_sp<SpF64>(r), b.n, partial);
    return hipGetLastError();
}

hipError_t launch_accumulate(const FieldDesc &x64, const FieldDesc &xs, hipStream_t st)
{
    if (x64.prec != P64) return hipErrorInvalidValue;
    DISPATCH_SP(xs.prec, F, LAUNCH(k_accumulate<F>, x64.n, st, make_sp<SpF64>(x64), make_sp<F>(xs), x64.n));
    return hipGetLastError();
}

hipError_t launch_axpy_host(double a, const FieldDesc &x, const FieldDesc &y, hipStream_t st)
{
    if (x.prec != P64 || y.prec != P64) return hipErrorInvalidValue;
    LAUNCH(k_axpy_host, x.n, st, a, make_sp<SpF64>(x), make_sp<SpF64>(y), x.n);
    return hipGetLastError();
}

hipError_t launch_scalar(int op, const double *partial, int n, CgScalars *s, double tol2, int relative,
                         const int *skip, hipStream_t st, CgScalars *publish)
{
    hipLaunchKernelGGL(k_scalar, dim3(1), dim3(SC_THREADS), 0, st, op, partial, n, s, tol2, relative, skip,
                       publish);
    return hipGetLastError();
}

// plain streaming copy, 16 bytes per lane, for bandwidth calibration
__global__ __launch_bounds__(256) void k_stream_copy(const float4 *__restrict__ a, float4 *__restrict__ b, long n)
{
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) b[i] = a[i];
}

hipError_t launch_stream_copy(const void *src, void *dst, size_t bytes, hipStream_t st)
{
    const long n = (long)(bytes / 16);
    hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, (const float4 *)src,
                       (float4 *)dst, n);
    return hipGetLastError();
}

hipError_t launch_sum(const double *partial, int n, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(SUM_THREADS), 0, st, partial, n, out);
    return hipGetLastError();
}

hipError_t launch_max(const double *partial, int n, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_max, dim3(1), dim3(SUM_THREADS), 0, st, partial, n, out);
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

size_t field_elem_bytes(int prec) { return 16; }  // double2, float4, uint4
int field_blocks(int prec) { return prec == P64 ? 12 : prec == P32 ? 6 : 3; }

}  // namespace tmq
