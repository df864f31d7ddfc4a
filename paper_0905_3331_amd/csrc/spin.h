// spin.h -- complex arithmetic and the spin projectors of the hopping term.
//
// Plain C++ usable on host and device (a CPU test compiles it with g++ to
// check the projector table against dense (1 +- gamma_mu)).
//
// For each direction mu and sign s, (1 + s gamma_mu) has rank 2 (Sec. 4.1): its
// first two rows h0, h1 determine the whole image.  With the gamma basis of
// Appendix A (spinor components s0..s3, each a colour vector):
//
//   mu s   h0          h1          rows 2, 3 of (1 + s gamma_mu) psi
//   t  +   s0 - s2     s1 - s3     -h0,   -h1
//   t  -   s0 + s2     s1 + s3      h0,    h1
//   x  +   s0 - i s3   s1 - i s2    i h1,  i h0
//   x  -   s0 + i s3   s1 + i s2   -i h1, -i h0
//   y  +   s0 - s3     s1 + s2      h1,   -h0
//   y  -   s0 + s3     s1 - s2     -h1,    h0
//   z  +   s0 - i s2   s1 + i s3    i h0, -i h1
//   z  -   s0 + i s2   s1 - i s3   -i h0,  i h1
//
// The link multiplies only h0 and h1 (2 colour vectors instead of 4), which is
// the projection / multiply / reconstruction split of eqs. (Dsplit), (Dunsplit).
#pragma once

#if defined(__HIPCC__)
#define TMQ_HD __host__ __device__ __forceinline__
#else
#define TMQ_HD inline
#endif

namespace tmq {

template <typename R>
struct cx {
    R re, im;
};

// Fused multiply-adds are written out (the device code is compiled without
// floating-point contraction), so that every kernel instantiation that runs
// the same operations rounds the same way.
TMQ_HD float fmad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
TMQ_HD double fmad(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename R>
TMQ_HD cx<R> mk(R a, R b) { return cx<R>{a, b}; }
template <typename R>
TMQ_HD cx<R> operator+(cx<R> a, cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R>
TMQ_HD cx<R> operator-(cx<R> a, cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R>
TMQ_HD cx<R> operator-(cx<R> a) { return {-a.re, -a.im}; }
template <typename R>
TMQ_HD cx<R> operator*(cx<R> a, cx<R> b)
{
    return {fmad(a.re, b.re, -(a.im * b.im)), fmad(a.re, b.im, a.im * b.re)};
}
template <typename R>
TMQ_HD cx<R> operator*(R a, cx<R> b) { return {a * b.re, a * b.im}; }
template <typename R>
TMQ_HD cx<R> conj(cx<R> a) { return {a.re, -a.im}; }
// i * a and -i * a
template <typename R>
TMQ_HD cx<R> ipl(cx<R> a) { return {-a.im, a.re}; }
template <typename R>
TMQ_HD cx<R> imi(cx<R> a) { return {a.im, -a.re}; }
// a + b * c and a + conj(b) * c
template <typename R>
TMQ_HD cx<R> fma(cx<R> b, cx<R> c, cx<R> a)
{
    return {fmad(b.re, c.re, fmad(-b.im, c.im, a.re)), fmad(b.re, c.im, fmad(b.im, c.re, a.im))};
}
template <typename R>
TMQ_HD cx<R> cfma(cx<R> b, cx<R> c, cx<R> a)
{
    return {fmad(b.re, c.re, fmad(b.im, c.im, a.re)), fmad(b.re, c.im, fmad(-b.im, c.re, a.im))};
}
template <typename R>
TMQ_HD R norm2(cx<R> a) { return fmad(a.re, a.re, a.im * a.im); }

// A spinor: 4 spins x 3 colours; a half spinor: 2 x 3.
template <typename R>
struct spinor {
    cx<R> c[4][3];
};
template <typename R>
struct half {
    cx<R> c[2][3];
};
// An SU(3) link, full 3x3.
template <typename R>
struct su3 {
    cx<R> e[3][3];
};

// third row of an SU(3) matrix from the first two: conj(row0 x row1)
template <typename R>
TMQ_HD void su3_third_row(su3<R> &u)
{
    u.e[2][0] = conj(u.e[0][1] * u.e[1][2] - u.e[0][2] * u.e[1][1]);
    u.e[2][1] = conj(u.e[0][2] * u.e[1][0] - u.e[0][0] * u.e[1][2]);
    u.e[2][2] = conj(u.e[0][0] * u.e[1][1] - u.e[0][1] * u.e[1][0]);
}

// h = first two rows of (1 + S gamma_MU) s
template <int MU, int S, typename R>
TMQ_HD void project(const spinor<R> &s, half<R> &h)
{
#pragma unroll
    for (int a = 0; a < 3; a++) {
        if (MU == 0) {
            h.c[0][a] = S > 0 ? s.c[0][a] - s.c[2][a] : s.c[0][a] + s.c[2][a];
            h.c[1][a] = S > 0 ? s.c[1][a] - s.c[3][a] : s.c[1][a] + s.c[3][a];
        } else if (MU == 1) {
            h.c[0][a] = S > 0 ? s.c[0][a] + imi(s.c[3][a]) : s.c[0][a] + ipl(s.c[3][a]);
            h.c[1][a] = S > 0 ? s.c[1][a] + imi(s.c[2][a]) : s.c[1][a] + ipl(s.c[2][a]);
        } else if (MU == 2) {
            h.c[0][a] = S > 0 ? s.c[0][a] - s.c[3][a] : s.c[0][a] + s.c[3][a];
            h.c[1][a] = S > 0 ? s.c[1][a] + s.c[2][a] : s.c[1][a] - s.c[2][a];
        } else {
            h.c[0][a] = S > 0 ? s.c[0][a] + imi(s.c[2][a]) : s.c[0][a] + ipl(s.c[2][a]);
            h.c[1][a] = S > 0 ? s.c[1][a] + ipl(s.c[3][a]) : s.c[1][a] + imi(s.c[3][a]);
        }
    }
}

// acc += (1 + S gamma_MU) image rebuilt from its first two rows h
template <int MU, int S, typename R>
TMQ_HD void reconstruct_add(spinor<R> &acc, const half<R> &h)
{
#pragma unroll
    for (int a = 0; a < 3; a++) {
        acc.c[0][a] = acc.c[0][a] + h.c[0][a];
        acc.c[1][a] = acc.c[1][a] + h.c[1][a];
        if (MU == 0) {
            if (S > 0) {
                acc.c[2][a] = acc.c[2][a] - h.c[0][a];
                acc.c[3][a] = acc.c[3][a] - h.c[1][a];
            } else {
                acc.c[2][a] = acc.c[2][a] + h.c[0][a];
                acc.c[3][a] = acc.c[3][a] + h.c[1][a];
            }
        } else if (MU == 1) {
            if (S > 0) {
                acc.c[2][a] = acc.c[2][a] + ipl(h.c[1][a]);
                acc.c[3][a] = acc.c[3][a] + ipl(h.c[0][a]);
            } else {
                acc.c[2][a] = acc.c[2][a] + imi(h.c[1][a]);
                acc.c[3][a] = acc.c[3][a] + imi(h.c[0][a]);
            }
        } else if (MU == 2) {
            if (S > 0) {
                acc.c[2][a] = acc.c[2][a] + h.c[1][a];
                acc.c[3][a] = acc.c[3][a] - h.c[0][a];
            } else {
                acc.c[2][a] = acc.c[2][a] - h.c[1][a];
                acc.c[3][a] = acc.c[3][a] + h.c[0][a];
            }
        } else {
            if (S > 0) {
                acc.c[2][a] = acc.c[2][a] + ipl(h.c[0][a]);
                acc.c[3][a] = acc.c[3][a] + imi(h.c[1][a]);
            } else {
                acc.c[2][a] = acc.c[2][a] + imi(h.c[0][a]);
                acc.c[3][a] = acc.c[3][a] + ipl(h.c[1][a]);
            }
        }
    }
}

// out = U h (DAG = false) or U^+ h (DAG = true), on both rows of h
template <bool DAG, typename R>
TMQ_HD void link_mul(const su3<R> &u, const half<R> &h, half<R> &out)
{
#pragma unroll
    for (int k = 0; k < 2; k++)
#pragma unroll
        for (int a = 0; a < 3; a++) {
            cx<R> s = {R(0), R(0)};
#pragma unroll
            for (int b = 0; b < 3; b++) s = DAG ? cfma(u.e[b][a], h.c[k][b], s) : fma(u.e[a][b], h.c[k][b], s);
            out.c[k][a] = s;
        }
}

// h *= ph (a complex phase)
template <typename R>
TMQ_HD void half_scale(half<R> &h, cx<R> ph)
{
#pragma unroll
    for (int k = 0; k < 2; k++)
#pragma unroll
        for (int a = 0; a < 3; a++) h.c[k][a] = ph * h.c[k][a];
}

}  // namespace tmq
