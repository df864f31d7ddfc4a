// fields.h -- device storage formats of spinor fields and gauge links.
//
// Every field lives on one parity (V/2 sites, eo index h = site >> 1) as an
// array of structures of arrays with 8-site chunks: the 16-byte component
// block c of site h sits at element ((h >> 3) * NB + c) * 8 + (h & 7), NB
// being the blocks per site.  A wavefront reading one block of 64
// consecutive sites touches 8 whole 128-byte lines, and the blocks of a site
// are 128 bytes apart, so a site's data lies in one NB * 128-byte stretch
// instead of NB distant streams (measured on MI355X: a 12-block streaming
// kernel moves 4.3 TB/s with one array per block, 5.2 TB/s with 8-site chunks).
//
//   spinors (12 complex per site, k = 3 * spin + colour)
//     F64  : 12 blocks of double2 (one complex each)                 192 B/site
//     F32  :  6 blocks of float4 (complex 2c, 2c+1)                   96 B/site
//     H16  :  3 blocks of 8 x fp16 (complex 4c..4c+3) + fp32 scale    52 B/site
//     B16  :  as H16 with bf16 codes                                  52 B/site
//     value of a 16-bit code = code * scale (FP32), scale = largest |real or
//     imaginary part| of the site; scales are a plain array [h].
//   links, per parity: the blocks of the 4 directions of a site chunk are
//   stored together, element ((h >> 3) * 4 * NB + mu * NB + b) * 8 + (h & 7)
//     L64F : 9 blocks of double2 (full 3x3)                          144 B/link
//     L64R : 6 blocks of double2 (rows 0, 1; row 2 = conj(r0 x r1))   96 B/link
//     L32R : 3 blocks of float4 (rows 0, 1)                            48 B/link
//     L16R : one block of 8 x fp16 (in array a) and one of 4 x fp16
//            (array b, 8-byte elements in 16-site chunks, lidx16)      24 B/link
//     L32F : 9 blocks of float2 (full 3x3; links that are not SU(3))   72 B/link
//   A field of n sites (n a multiple of 8) stacked from two parities is one
//   such array of 2 * V/2 sites: the odd sites start at site V/2.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include "spin.h"

namespace tmq {

// element of block c (of nb per site) of site h
__device__ __forceinline__ long aidx(long h, int c, int nb) { return ((h >> 3) * nb + c) * 8 + (h & 7); }
// element of block b of direction mu of the links of site h (nb blocks per link)
__device__ __forceinline__ long lidx(long h, int mu, int b, int nb)
{
    return ((h >> 3) * 4 * nb + mu * nb + b) * 8 + (h & 7);
}
// 8-byte link blocks use 16-site chunks, so that one direction of a chunk is
// one whole 128-byte line: element ((h >> 4) * 4 + mu) * 16 + (h & 15) of an
// array of 4 * vh16 elements per parity, vh16 = V/2 rounded up to 16
__device__ __forceinline__ long lidx16(long h, int mu) { return ((h >> 4) * 4 + mu) * 16 + (h & 15); }
__host__ __device__ __forceinline__ long vh16(long vh) { return (vh + 15) & ~15L; }

// ------------------------------------------------------- streaming loads
// Loads of data that is used once per kernel (the links) can bypass the
// caches' retention (non-temporal), leaving L2 and the Infinity Cache to the
// spinors, which every site reads 8 times through its neighbours.
typedef double nv_d2 __attribute__((ext_vector_type(2)));
typedef float nv_f4 __attribute__((ext_vector_type(4)));
typedef unsigned int nv_u4 __attribute__((ext_vector_type(4)));
typedef unsigned int nv_u2 __attribute__((ext_vector_type(2)));
typedef float nv_f2 __attribute__((ext_vector_type(2)));

template <bool NT>
__device__ __forceinline__ double2 ld(const double2 *p)
{
    if (NT) {
        nv_d2 v = __builtin_nontemporal_load((const nv_d2 *)p);
        return make_double2(v.x, v.y);
    }
    return *p;
}
template <bool NT>
__device__ __forceinline__ float4 ld(const float4 *p)
{
    if (NT) {
        nv_f4 v = __builtin_nontemporal_load((const nv_f4 *)p);
        return make_float4(v.x, v.y, v.z, v.w);
    }
    return *p;
}
template <bool NT>
__device__ __forceinline__ float2 ld(const float2 *p)
{
    if (NT) {
        nv_f2 v = __builtin_nontemporal_load((const nv_f2 *)p);
        return make_float2(v.x, v.y);
    }
    return *p;
}
template <bool NT>
__device__ __forceinline__ uint4 ld(const uint4 *p)
{
    if (NT) {
        nv_u4 v = __builtin_nontemporal_load((const nv_u4 *)p);
        return make_uint4(v.x, v.y, v.z, v.w);
    }
    return *p;
}
template <bool NT>
__device__ __forceinline__ uint2 ld(const uint2 *p)
{
    if (NT) {
        nv_u2 v = __builtin_nontemporal_load((const nv_u2 *)p);
        return make_uint2(v.x, v.y);
    }
    return *p;
}

// Stores of data that this kernel does not read again (a hop's output) can
// be non-temporal too, so that they do not displace the spinors in L2.
template <bool NT>
__device__ __forceinline__ void st(double2 *p, double2 v)
{
    if (NT)
        __builtin_nontemporal_store(nv_d2{v.x, v.y}, (nv_d2 *)p);
    else
        *p = v;
}
template <bool NT>
__device__ __forceinline__ void st(float4 *p, float4 v)
{
    if (NT)
        __builtin_nontemporal_store(nv_f4{v.x, v.y, v.z, v.w}, (nv_f4 *)p);
    else
        *p = v;
}
template <bool NT>
__device__ __forceinline__ void st(uint4 *p, uint4 v)
{
    if (NT)
        __builtin_nontemporal_store(nv_u4{v.x, v.y, v.z, v.w}, (nv_u4 *)p);
    else
        *p = v;
}
template <bool NT>
__device__ __forceinline__ void st(float *p, float v)
{
    if (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

// ------------------------------------------------------------ 16-bit codes

__device__ __forceinline__ float h16_to_f32(uint16_t c) { return __half2float(__ushort_as_half(c)); }
__device__ __forceinline__ uint16_t f32_to_h16(float f) { return __half_as_ushort(__float2half_rn(f)); }
__device__ __forceinline__ float b16_to_f32(uint16_t c) { return __uint_as_float(((uint32_t)c) << 16); }
// round to nearest even on the dropped 16 bits (finite inputs)
__device__ __forceinline__ uint16_t f32_to_b16(float f)
{
    uint32_t u = __float_as_uint(f);
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

template <bool BF>
__device__ __forceinline__ float code_to_f32(uint16_t c) { return BF ? b16_to_f32(c) : h16_to_f32(c); }
template <bool BF>
__device__ __forceinline__ uint16_t f32_to_code(float f) { return BF ? f32_to_b16(f) : f32_to_h16(f); }

__device__ __forceinline__ uint16_t lo16(uint32_t w) { return (uint16_t)(w & 0xFFFFu); }
__device__ __forceinline__ uint16_t hi16(uint32_t w) { return (uint16_t)(w >> 16); }
__device__ __forceinline__ uint32_t pack16(uint16_t lo, uint16_t hi) { return (uint32_t)lo | ((uint32_t)hi << 16); }

// Value of the low / high 16-bit code of a word as FP32.  For FP16 the result
// is a plain widening conversion, which the compiler folds into the operand
// of a following FMA (v_fma_mix_f32 reads FP16 halves directly); the kernels
// therefore combine codes with FMAs, an opaque 1.0 standing in for a plain add.
template <bool BF>
__device__ __forceinline__ float code_lo(uint32_t w)
{
    if (BF) return __uint_as_float(w << 16);
    return (float)__builtin_bit_cast(_Float16, (uint16_t)(w & 0xFFFFu));
}
template <bool BF>
__device__ __forceinline__ float code_hi(uint32_t w)
{
    if (BF) return __uint_as_float(w & 0xFFFF0000u);
    return (float)__builtin_bit_cast(_Float16, (uint16_t)(w >> 16));
}

// --------------------------------------------------------------- spinors

struct SpF64 {
    using real = double;
    static constexpr bool coded = false;
    double2 *p;
    template <typename R>
    __device__ __forceinline__ void load(long h, spinor<R> &s) const
    {
        const double2 *q = p + aidx(h, 0, 12);
#pragma unroll
        for (int k = 0; k < 12; k++) {
            double2 v = q[k * 8];
            s.c[k / 3][k % 3] = cx<R>{(R)v.x, (R)v.y};
        }
    }
    template <bool NT = false, typename R>
    __device__ __forceinline__ void store(long h, const spinor<R> &s) const
    {
        double2 *q = p + aidx(h, 0, 12);
#pragma unroll
        for (int k = 0; k < 12; k++) {
            cx<R> v = s.c[k / 3][k % 3];
            st<NT>(q + k * 8, make_double2((double)v.re, (double)v.im));
        }
    }
};

struct SpF32 {
    using real = float;
    static constexpr bool coded = false;
    float4 *p;
    template <typename R>
    __device__ __forceinline__ void load(long h, spinor<R> &s) const
    {
        const float4 *q = p + aidx(h, 0, 6);
#pragma unroll
        for (int k = 0; k < 6; k++) {
            float4 v = q[k * 8];
            s.c[(2 * k) / 3][(2 * k) % 3] = cx<R>{(R)v.x, (R)v.y};
            s.c[(2 * k + 1) / 3][(2 * k + 1) % 3] = cx<R>{(R)v.z, (R)v.w};
        }
    }
    template <bool NT = false, typename R>
    __device__ __forceinline__ void store(long h, const spinor<R> &s) const
    {
        float4 *q = p + aidx(h, 0, 6);
#pragma unroll
        for (int k = 0; k < 6; k++) {
            cx<R> a = s.c[(2 * k) / 3][(2 * k) % 3];
            cx<R> b = s.c[(2 * k + 1) / 3][(2 * k + 1) % 3];
            st<NT>(q + k * 8, make_float4((float)a.re, (float)a.im, (float)b.re, (float)b.im));
        }
    }
};

template <bool BF>
struct Sp16 {
    using real = float;
    static constexpr bool coded = true;
    static constexpr bool bf = BF;
    uint4 *p;
    float *scale;
    // the 12 words of a site (word k: complex component k = 3 * spin + colour,
    // real part in the low half) and its scale, undecoded
    __device__ __forceinline__ void load_codes(long h, uint32_t w[12], float &sc) const
    {
        sc = scale[h];
        const uint4 *q = p + aidx(h, 0, 3);
#pragma unroll
        for (int k = 0; k < 3; k++) {
            uint4 v = q[k * 8];
            w[4 * k] = v.x;
            w[4 * k + 1] = v.y;
            w[4 * k + 2] = v.z;
            w[4 * k + 3] = v.w;
        }
    }
    template <typename R>
    __device__ __forceinline__ void load(long h, spinor<R> &s) const
    {
        const float sc = scale[h];
        const uint4 *q = p + aidx(h, 0, 3);
#pragma unroll
        for (int k = 0; k < 3; k++) {
            uint4 v = q[k * 8];
            uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int j = 0; j < 4; j++) {
                int comp = 4 * k + j;
                s.c[comp / 3][comp % 3] =
                    cx<R>{(R)(code_to_f32<BF>(lo16(w[j])) * sc), (R)(code_to_f32<BF>(hi16(w[j])) * sc)};
            }
        }
    }
    // store FP32 values: scale = largest |part|, codes = value * (1 / scale).
    // A site whose largest part is below the smallest normal FP32 number is
    // stored as zero (its reciprocal would overflow); a non-finite site keeps
    // a NaN scale so that the solver's checks see it.
    template <bool NT = false, typename R>
    __device__ __forceinline__ void store(long h, const spinor<R> &s) const
    {
        float m = 0.f;
        bool bad = false;
#pragma unroll
        for (int k = 0; k < 12; k++) {
            const float a = fabsf((float)s.c[k / 3][k % 3].re), b = fabsf((float)s.c[k / 3][k % 3].im);
            bad |= !(a <= 3.0e38f) || !(b <= 3.0e38f);
            m = fmaxf(m, fmaxf(a, b));
        }
        const bool tiny = m < 1.17549435e-38f;
        const float inv = tiny ? 0.f : 1.0f / m;
        st<NT>(scale + h, bad ? __int_as_float(0x7fc00000) : (tiny ? 0.f : m));
        uint4 *q = p + aidx(h, 0, 3);
#pragma unroll
        for (int k = 0; k < 3; k++) {
            uint32_t w[4];
#pragma unroll
            for (int j = 0; j < 4; j++) {
                int comp = 4 * k + j;
                cx<R> v = s.c[comp / 3][comp % 3];
                w[j] = pack16(f32_to_code<BF>((float)v.re * inv), f32_to_code<BF>((float)v.im * inv));
            }
            st<NT>(q + k * 8, make_uint4(w[0], w[1], w[2], w[3]));
        }
    }
};
using SpH16 = Sp16<false>;
using SpB16 = Sp16<true>;

// ----------------------------------------------------------------- links
// One array per parity half: parity par starts at element par * 4 * NB * V/2.

struct L64F {
    using real = double;
    const double2 *p;
    long vh;
    template <bool NT, typename R>
    __device__ __forceinline__ void load(int par, int mu, long h, su3<R> &u) const
    {
        const double2 *q = p + par * 36 * vh + lidx(h, mu, 0, 9);
#pragma unroll
        for (int k = 0; k < 9; k++) {
            double2 v = ld<NT>(q + k * 8);
            u.e[k / 3][k % 3] = cx<R>{(R)v.x, (R)v.y};
        }
    }
    // a link held in registers, and out = U p or U^+ p with it
    using Loaded = su3<real>;
    template <bool NT>
    __device__ __forceinline__ void load_link(int par, int mu, long h, Loaded &u) const
    {
        load<NT>(par, mu, h, u);
    }
    template <bool DAG>
    __device__ __forceinline__ void apply(const Loaded &u, const half<real> &p, half<real> &out) const
    {
        link_mul<DAG>(u, p, out);
    }
};

struct L64R {
    using real = double;
    const double2 *p;
    long vh;
    template <bool NT, typename R>
    __device__ __forceinline__ void load(int par, int mu, long h, su3<R> &u) const
    {
        const double2 *q = p + par * 24 * vh + lidx(h, mu, 0, 6);
#pragma unroll
        for (int k = 0; k < 6; k++) {
            double2 v = ld<NT>(q + k * 8);
            u.e[k / 3][k % 3] = cx<R>{(R)v.x, (R)v.y};
        }
        su3_third_row(u);
    }
    // a link held in registers, and out = U p or U^+ p with it
    using Loaded = su3<real>;
    template <bool NT>
    __device__ __forceinline__ void load_link(int par, int mu, long h, Loaded &u) const
    {
        load<NT>(par, mu, h, u);
    }
    template <bool DAG>
    __device__ __forceinline__ void apply(const Loaded &u, const half<real> &p, half<real> &out) const
    {
        link_mul<DAG>(u, p, out);
    }
};

struct L32R {
    using real = float;
    const float4 *p;
    long vh;
    template <bool NT, typename R>
    __device__ __forceinline__ void load(int par, int mu, long h, su3<R> &u) const
    {
        load_rows<NT>(par, mu, h, u);
        su3_third_row(u);
    }
    // rows 0 and 1 only (load = load_rows + su3_third_row)
    template <bool NT, typename R>
    __device__ __forceinline__ void load_rows(int par, int mu, long h, su3<R> &u) const
    {
        const float4 *q = p + par * 12 * vh + lidx(h, mu, 0, 3);
#pragma unroll
        for (int k = 0; k < 3; k++) {
            float4 v = ld<NT>(q + k * 8);
            u.e[(2 * k) / 3][(2 * k) % 3] = cx<R>{(R)v.x, (R)v.y};
            u.e[(2 * k + 1) / 3][(2 * k + 1) % 3] = cx<R>{(R)v.z, (R)v.w};
        }
    }
    // a link held in registers, and out = U p or U^+ p with it
    using Loaded = su3<real>;
    template <bool NT>
    __device__ __forceinline__ void load_link(int par, int mu, long h, Loaded &u) const
    {
        load<NT>(par, mu, h, u);
    }
    template <bool DAG>
    __device__ __forceinline__ void apply(const Loaded &u, const half<real> &p, half<real> &out) const
    {
        link_mul<DAG>(u, p, out);
    }
};

// FP32 copy of links that are not SU(3): all three rows stored (row 2 cannot
// be rebuilt from rows 0 and 1), the reduced-precision operator of any U
struct L32F {
    using real = float;
    const float2 *p;
    long vh;
    template <bool NT, typename R>
    __device__ __forceinline__ void load(int par, int mu, long h, su3<R> &u) const
    {
        const float2 *q = p + par * 36 * vh + lidx(h, mu, 0, 9);
#pragma unroll
        for (int k = 0; k < 9; k++) {
            float2 v = ld<NT>(q + k * 8);
            u.e[k / 3][k % 3] = cx<R>{(R)v.x, (R)v.y};
        }
    }
    using Loaded = su3<real>;
    template <bool NT>
    __device__ __forceinline__ void load_link(int par, int mu, long h, Loaded &u) const
    {
        load<NT>(par, mu, h, u);
    }
    template <bool DAG>
    __device__ __forceinline__ void apply(const Loaded &u, const half<real> &p, half<real> &out) const
    {
        link_mul<DAG>(u, p, out);
    }
};

struct L16R {
    using real = float;
    const uint4 *a;  // complex 0..3 of rows 0,1 (row-major)
    const uint2 *b;  // complex 4, 5
    long vh;
    // A link held in registers: the words of rows 0 and 1 (entry (i, j) is
    // word 3 i + j, real part in the low half) and row 2 = conj(row0 x row1)
    // formed in FP32 from them.  apply() computes U p or U^+ p in FP32 with
    // the FP16 entries read directly by the FMAs.
    struct Loaded {
        uint32_t w[6];
        cx<float> r2[3];
    };
    // the six words of rows 0 and 1 (load_link = load_raw + rebuild)
    template <bool NT>
    __device__ __forceinline__ void load_raw(int par, int mu, long h, uint32_t w[6]) const
    {
        const uint4 va = ld<NT>(a + par * 4 * vh + lidx(h, mu, 0, 1));
        const uint2 vb = ld<NT>(b + par * 4 * vh16(vh) + lidx16(h, mu));
        w[0] = va.x;
        w[1] = va.y;
        w[2] = va.z;
        w[3] = va.w;
        w[4] = vb.x;
        w[5] = vb.y;
    }
    template <bool NT>
    __device__ __forceinline__ void load_link(int par, int mu, long h, Loaded &u) const
    {
        load_raw<NT>(par, mu, h, u.w);
        rebuild(u);
    }
    // row 2 from the words of rows 0 and 1
    __device__ __forceinline__ void rebuild(Loaded &u) const
    {
        auto re = [&](int i, int j) { return code_lo<false>(u.w[3 * i + j]); };
        auto im = [&](int i, int j) { return code_hi<false>(u.w[3 * i + j]); };
        // row 2, column c: conj(u0a u1b - u0b u1a) with (a, b) the other two columns in cyclic order
#pragma unroll
        for (int c = 0; c < 3; c++) {
            const int ca = (c + 1) % 3, cb = (c + 2) % 3;
            u.r2[c].re = fmad(re(0, ca), re(1, cb),
                              fmad(-im(0, ca), im(1, cb), fmad(-re(0, cb), re(1, ca), fmad(im(0, cb), im(1, ca), 0.f))));
            u.r2[c].im = fmad(-re(0, ca), im(1, cb),
                              fmad(-im(0, ca), re(1, cb), fmad(re(0, cb), im(1, ca), fmad(im(0, cb), re(1, ca), 0.f))));
        }
    }
    template <bool DAG>
    __device__ __forceinline__ void apply(const Loaded &u, const half<float> &p, half<float> &out) const
    {
        auto re = [&](int i, int j) { return code_lo<false>(u.w[3 * i + j]); };
        auto im = [&](int i, int j) { return code_hi<false>(u.w[3 * i + j]); };
#pragma unroll
        for (int k = 0; k < 2; k++)
#pragma unroll
            for (int r = 0; r < 3; r++) {
                float sr = 0.f, si = 0.f;
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    const cx<float> x = p.c[k][c];
                    if (!DAG) {  // + U[r][c] x
                        if (r < 2) {
                            sr = fmad(re(r, c), x.re, fmad(-im(r, c), x.im, sr));
                            si = fmad(re(r, c), x.im, fmad(im(r, c), x.re, si));
                        } else {
                            sr = fmad(u.r2[c].re, x.re, fmad(-u.r2[c].im, x.im, sr));
                            si = fmad(u.r2[c].re, x.im, fmad(u.r2[c].im, x.re, si));
                        }
                    } else {  // + conj(U[c][r]) x
                        if (c < 2) {
                            sr = fmad(re(c, r), x.re, fmad(im(c, r), x.im, sr));
                            si = fmad(re(c, r), x.im, fmad(-im(c, r), x.re, si));
                        } else {
                            sr = fmad(u.r2[r].re, x.re, fmad(u.r2[r].im, x.im, sr));
                            si = fmad(u.r2[r].re, x.im, fmad(-u.r2[r].im, x.re, si));
                        }
                    }
                }
                out.c[k][r] = cx<float>{sr, si};
            }
    }
    template <bool NT, typename R>
    __device__ __forceinline__ void load(int par, int mu, long h, su3<R> &u) const
    {
        uint4 va = ld<NT>(a + par * 4 * vh + lidx(h, mu, 0, 1));
        uint2 vb = ld<NT>(b + par * 4 * vh16(vh) + lidx16(h, mu));
        uint32_t w[6] = {va.x, va.y, va.z, va.w, vb.x, vb.y};
#pragma unroll
        for (int k = 0; k < 6; k++)
            u.e[k / 3][k % 3] = cx<R>{(R)h16_to_f32(lo16(w[k])), (R)h16_to_f32(hi16(w[k]))};
        su3_third_row(u);
    }
};

}  // namespace tmq
