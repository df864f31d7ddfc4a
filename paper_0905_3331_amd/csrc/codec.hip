// codec.hip -- conversions between the canonical host layout and the device
// formats, and the gauge-field ingest.
//
// Canonical layout: complex128, site-major ([site][spin][colour] for spinors,
// [site][mu][row][col] for links), site = ((t*LZ + z)*LY + y)*LX + x.
// Device layout: per-parity arrays of 8-site chunks (fields.h).
//
// 16-bit spinor encoding of FP64 input (one rounding to FP32, then RNE to
// FP16/BF16): scale = fp32(max |part|) over the site's 24 reals, code =
// to16(fp32(value / scale)) with the division in FP64; an all-zero site has
// scale 0 and zero codes.  Inside the solver, FP32 values are encoded with
// value * (1 / scale) in FP32.
#include <type_traits>

#include "devutil.h"
#include "views.h"

namespace tmq {

// store FP64 values; 16-bit formats follow the FP64 encoding rule above
template <class SP>
__device__ __forceinline__ void store_f64(const SP &f, long h, const spinor<double> &s)
{
    f.store(h, s);
}

template <bool BF>
__device__ __forceinline__ void store_f64_16(const Sp16<BF> &f, long h, const spinor<double> &s)
{
    double m = 0.0;
#pragma unroll
    for (int k = 0; k < 12; k++) {
        m = fmax(m, fabs(s.c[k / 3][k % 3].re));
        m = fmax(m, fabs(s.c[k / 3][k % 3].im));
    }
    const float sc = (float)m;
    const double d = (double)sc;
    f.scale[h] = sc;
    uint4 *q = f.p + aidx(h, 0, 3);
#pragma unroll
    for (int k = 0; k < 3; k++) {
        uint32_t w[4];
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int comp = 4 * k + j;
            const cx<double> v = s.c[comp / 3][comp % 3];
            const float yr = sc > 0.f ? (float)(v.re / d) : 0.f;
            const float yi = sc > 0.f ? (float)(v.im / d) : 0.f;
            w[j] = pack16(f32_to_code<BF>(yr), f32_to_code<BF>(yi));
        }
        q[k * 8] = make_uint4(w[0], w[1], w[2], w[3]);
    }
}
template <>
__device__ __forceinline__ void store_f64<SpH16>(const SpH16 &f, long h, const spinor<double> &s)
{
    store_f64_16<false>(f, h, s);
}
template <>
__device__ __forceinline__ void store_f64<SpB16>(const SpB16 &f, long h, const spinor<double> &s)
{
    store_f64_16<true>(f, h, s);
}

__device__ __forceinline__ void load_canonical(const double2 *in, long site, spinor<double> &s)
{
    const double2 *q = in + site * 12;
#pragma unroll
    for (int k = 0; k < 12; k++) {
        double2 v = q[k];
        s.c[k / 3][k % 3] = cx<double>{v.x, v.y};
    }
}

__device__ __forceinline__ void store_canonical(double2 *out, long site, const spinor<double> &s)
{
    double2 *q = out + site * 12;
#pragma unroll
    for (int k = 0; k < 12; k++) q[k] = make_double2(s.c[k / 3][k % 3].re, s.c[k / 3][k % 3].im);
}

template <class SP>
__global__ __launch_bounds__(BLAS_BLOCK) void k_from_canonical(const double2 *in, SP out, long n)
{
    const long h = (long)blockIdx.x * BLAS_BLOCK + threadIdx.x;
    if (h < n) {
        spinor<double> s;
        load_canonical(in, h, s);
        store_f64(out, h, s);
    }
}

template <class SP>
__global__ __launch_bounds__(BLAS_BLOCK) void k_to_canonical(SP in, double2 *out, long n)
{
    const long h = (long)blockIdx.x * BLAS_BLOCK + threadIdx.x;
    if (h < n) {
        spinor<double> s;
        in.load(h, s);
        store_canonical(out, h, s);
    }
}

// parity of canonical site s
__device__ __forceinline__ int site_parity(const Geom &g, long s)
{
    const unsigned su = (unsigned)s;
    const unsigned x = su % (unsigned)g.LX;
    unsigned r = su / (unsigned)g.LX;
    const unsigned y = r % (unsigned)g.LY;
    r /= (unsigned)g.LY;
    const unsigned z = r % (unsigned)g.LZ;
    const unsigned t = r / (unsigned)g.LZ;
    return (int)((t + z + y + x) & 1u);
}

template <class SP, bool TO>
__global__ __launch_bounds__(BLAS_BLOCK) void k_full_canonical(Geom g, double2 *can, SP f)
{
    const long s = (long)blockIdx.x * BLAS_BLOCK + threadIdx.x;
    if (s < 2 * g.vh) {
        const long v = site_parity(g, s) * g.vh + (s >> 1);
        spinor<double> sp;
        if (TO) {
            f.load(v, sp);
            store_canonical(can, s, sp);
        } else {
            load_canonical(can, s, sp);
            store_f64(f, v, sp);
        }
    }
}

template <class SP>
__global__ __launch_bounds__(BLAS_BLOCK) void k_export_codes(SP in, uint16_t *codes, float *scale, long n)
{
    const long h = (long)blockIdx.x * BLAS_BLOCK + threadIdx.x;
    if (h < n) {
        scale[h] = in.scale[h];
#pragma unroll
        for (int k = 0; k < 3; k++) {
            const uint4 v = in.p[aidx(h, k, 3)];
            const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int j = 0; j < 4; j++) {
                codes[h * 24 + 2 * (4 * k + j)] = lo16(w[j]);
                codes[h * 24 + 2 * (4 * k + j) + 1] = hi16(w[j]);
            }
        }
    }
}

// ------------------------------------------------------- even/odd split

// Canonical full field <-> canonical even and odd fields, one thread per
// complex component (reads or writes of the full field coalesced).  A null
// parity pointer: split skips it, merge writes zeros there.
template <bool MERGE>
__global__ __launch_bounds__(BLAS_BLOCK) void k_split_eo(Geom g, double2 *full, double2 *even, double2 *odd)
{
    const long i = (long)blockIdx.x * BLAS_BLOCK + threadIdx.x;
    if (i >= 2 * g.vh * 12) return;
    const long s = i / 12;
    const int c = (int)(i - s * 12);
    double2 *part = site_parity(g, s) ? odd : even;
    const long j = (s >> 1) * 12 + c;
    if (MERGE)
        full[i] = part ? part[j] : make_double2(0.0, 0.0);
    else if (part)
        part[j] = full[i];
}

// ------------------------------------------------------------------ gauge

__global__ __launch_bounds__(BLAS_BLOCK) void k_gauge_ingest(Geom g, const double2 *U, GaugeOut o, double *partial)
{
    const long s = (long)blockIdx.x * BLAS_BLOCK + threadIdx.x;
    double dev = 0.0;
    if (s < 2 * g.vh) {
        const int par = site_parity(g, s);
        const long h = s >> 1, st = g.vh;
        for (int mu = 0; mu < 4; mu++) {
            su3<double> u;
            const double2 *q = U + (s * 4 + mu) * 9;
#pragma unroll
            for (int k = 0; k < 9; k++) u.e[k / 3][k % 3] = cx<double>{q[k].x, q[k].y};
            if (o.full64) {
                double2 *q = o.full64 + par * 36 * st + lidx(h, mu, 0, 9);
#pragma unroll
                for (int k = 0; k < 9; k++) q[k * 8] = make_double2(u.e[k / 3][k % 3].re, u.e[k / 3][k % 3].im);
            }
            if (o.row64) {
                double2 *q = o.row64 + par * 24 * st + lidx(h, mu, 0, 6);
#pragma unroll
                for (int k = 0; k < 6; k++) q[k * 8] = make_double2(u.e[k / 3][k % 3].re, u.e[k / 3][k % 3].im);
            }
            if (o.row32) {
                float4 *q = o.row32 + par * 12 * st + lidx(h, mu, 0, 3);
#pragma unroll
                for (int k = 0; k < 3; k++) {
                    const cx<double> a = u.e[(2 * k) / 3][(2 * k) % 3], b = u.e[(2 * k + 1) / 3][(2 * k + 1) % 3];
                    q[k * 8] = make_float4((float)a.re, (float)a.im, (float)b.re, (float)b.im);
                }
            }
            if (o.full32) {
                float2 *q = o.full32 + par * 36 * st + lidx(h, mu, 0, 9);
#pragma unroll
                for (int k = 0; k < 9; k++)
                    q[k * 8] = make_float2((float)u.e[k / 3][k % 3].re, (float)u.e[k / 3][k % 3].im);
            }
            if (o.row16a) {
                uint32_t w[6];
#pragma unroll
                for (int k = 0; k < 6; k++)
                    w[k] = pack16(f32_to_h16((float)u.e[k / 3][k % 3].re), f32_to_h16((float)u.e[k / 3][k % 3].im));
                o.row16a[par * 4 * st + lidx(h, mu, 0, 1)] = make_uint4(w[0], w[1], w[2], w[3]);
                o.row16b[par * 4 * vh16(st) + lidx16(h, mu)] = make_uint2(w[4], w[5]);
            }
            // distance from SU(3): max |(U U^+ - 1)_ab| and |det U - 1|
#pragma unroll
            for (int a = 0; a < 3; a++)
#pragma unroll
                for (int b = 0; b < 3; b++) {
                    cx<double> e = {a == b ? -1.0 : 0.0, 0.0};
#pragma unroll
                    for (int c = 0; c < 3; c++) e = cfma(u.e[b][c], u.e[a][c], e);
                    dev = fmax(dev, sqrt(norm2(e)));
                }
            su3<double> w = u;
            su3_third_row(w);
            cx<double> det = {-1.0, 0.0};
#pragma unroll
            for (int c = 0; c < 3; c++) det = fma(u.e[2][c], conj(w.e[2][c]), det);
            dev = fmax(dev, sqrt(norm2(det)));
        }
    }
    __shared__ double sh[BLAS_BLOCK / 64];
    const double m = block_max(dev, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = m;
}

// -------------------------------------------------------------- dispatch

#define DISPATCH_SPC TMQ_DISPATCH_SP

hipError_t launch_from_canonical(const double2 *in, const FieldDesc &out, hipStream_t st)
{
    DISPATCH_SPC(out.prec, F,
                 hipLaunchKernelGGL(k_from_canonical<F>, dim3(blas_grid(out.n)), dim3(BLAS_BLOCK), 0, st, in,
                                    make_sp<F>(out), out.n));
    return hipGetLastError();
}

hipError_t launch_to_canonical(const FieldDesc &in, double2 *out, hipStream_t st)
{
    DISPATCH_SPC(in.prec, F,
                 hipLaunchKernelGGL(k_to_canonical<F>, dim3(blas_grid(in.n)), dim3(BLAS_BLOCK), 0, st,
                                    make_sp<F>(in), out, in.n));
    return hipGetLastError();
}

hipError_t launch_full_from_canonical(const Geom &g, const double2 *in, const FieldDesc &out, hipStream_t st)
{
    if (out.n != 2 * g.vh) return hipErrorInvalidValue;
    DISPATCH_SPC(out.prec, F,
                 hipLaunchKernelGGL((k_full_canonical<F, false>), dim3(blas_grid(out.n)), dim3(BLAS_BLOCK), 0, st,
                                    g, (double2 *)in, make_sp<F>(out)));
    return hipGetLastError();
}

hipError_t launch_full_to_canonical(const Geom &g, const FieldDesc &in, double2 *out, hipStream_t st)
{
    if (in.n != 2 * g.vh) return hipErrorInvalidValue;
    DISPATCH_SPC(in.prec, F,
                 hipLaunchKernelGGL((k_full_canonical<F, true>), dim3(blas_grid(in.n)), dim3(BLAS_BLOCK), 0, st,
                                    g, out, make_sp<F>(in)));
    return hipGetLastError();
}

hipError_t launch_split_eo(const Geom &g, const double2 *full, double2 *even, double2 *odd, hipStream_t st)
{
    hipLaunchKernelGGL(k_split_eo<false>, dim3(blas_grid(2 * g.vh * 12)), dim3(BLAS_BLOCK), 0, st, g, (double2 *)full,
                       even, odd);
    return hipGetLastError();
}

hipError_t launch_merge_eo(const Geom &g, const double2 *even, const double2 *odd, double2 *full, hipStream_t st)
{
    hipLaunchKernelGGL(k_split_eo<true>, dim3(blas_grid(2 * g.vh * 12)), dim3(BLAS_BLOCK), 0, st, g, full,
                       (double2 *)even, (double2 *)odd);
    return hipGetLastError();
}

hipError_t launch_export_codes(const FieldDesc &in, uint16_t *codes, float *scale, hipStream_t st)
{
    if (in.prec == P16)
        hipLaunchKernelGGL(k_export_codes<SpH16>, dim3(blas_grid(in.n)), dim3(BLAS_BLOCK), 0, st, make_sp<SpH16>(in),
                           codes, scale, in.n);
    else if (in.prec == PB16)
        hipLaunchKernelGGL(k_export_codes<SpB16>, dim3(blas_grid(in.n)), dim3(BLAS_BLOCK), 0, st, make_sp<SpB16>(in),
                           codes, scale, in.n);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_gauge_ingest(const Geom &g, const double2 *U, const GaugeOut &o, double *partial_max,
                               hipStream_t st)
{
    hipLaunchKernelGGL(k_gauge_ingest, dim3(blas_grid(2 * g.vh)), dim3(BLAS_BLOCK), 0, st, g, U, o, partial_max);
    return hipGetLastError();
}

}  // namespace tmq
