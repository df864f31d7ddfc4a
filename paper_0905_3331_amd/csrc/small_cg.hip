// small_cg.hip -- the whole full-lattice CG of a tiny lattice in one workgroup.
//
// On a lattice of a few hundred sites every kernel of a CG iteration is a
// handful of wavefronts, and the iteration costs what the GPU needs to start
// its nine dependent kernels (about 5 us each).  Here one workgroup of 256
// lanes (one wavefront per SIMD of a single CU) runs textbook CG on
// Q^+ Q^- (Sec. 4.4, eq. (eo1) on both parities) from start to finish: the
// vectors stay in global memory, which for such sizes lives in the CU's L1
// and the XCD's L2; block-wide barriers order the phases, and the inner
// products are fixed-order block reductions (so results are reproducible).
// After the iterated residual meets the target the kernel recomputes the
// true residual b - A x and leaves the decision to the host, which calls it
// again (CG restarted from the true residual) if the true residual has not
// met the target.
#include "devutil.h"
#include "views.h"

namespace tmq {

constexpr int SMALL_THREADS = 256;

template <class LK>
struct SmallCgArgs {
    Geom g;
    SpF64 b, x, r, p, t, ap;  // stacked (even, odd) full-lattice fields
    LK lk;
    double ph[4][2];
    double kappa, mut, tol2;
    int relative, max_iter;
    CgScalars *sc;  // in/out: counters and residuals across calls
};

namespace {

// H psi at output site h of parity out_par, from the other parity's field
template <int MU, class LK>
__device__ __forceinline__ void small_dir(const LK &lk, int out_par, const SpF64 &in, cx<double> ph, bool phase,
                                          long h, long hf, long hb, spinor<double> &acc)
{
    typename LK::Loaded u;
    spinor<double> sp;
    half<double> p, w;
    // forward: e^{i theta pi/L} U(x, mu) (1 + gamma_mu) psi(x + mu)
    lk.template load_link<false>(out_par, MU, h, u);
    in.load(hf, sp);
    project<MU, +1>(sp, p);
    lk.template apply<false>(u, p, w);
    if (phase) half_scale(w, ph);
    reconstruct_add<MU, +1>(acc, w);
    // backward: e^{-i theta pi/L} U(x - mu, mu)^+ (1 - gamma_mu) psi(x - mu)
    lk.template load_link<false>(out_par ^ 1, MU, hb, u);
    in.load(hb, sp);
    project<MU, -1>(sp, p);
    lk.template apply<true>(u, p, w);
    if (phase) half_scale(w, conj(ph));
    reconstruct_add<MU, -1>(acc, w);
}

// out(s) = g5 [(1 + sign i mut g5) in(s) - kappa (H in)(s)] for full-lattice site s
template <class LK>
__device__ __forceinline__ void small_q_site(const SmallCgArgs<LK> &a, const SpF64 &in, int sign, long s,
                                             spinor<double> &o)
{
    const Geom &g = a.g;
    const int par = s >= g.vh ? 1 : 0;
    const long h = s - par * g.vh;
    const SpF64 other{in.p + (long)(1 - par) * g.vh * 12};
    const unsigned hu = (unsigned)h;
    const unsigned xh = hu % (unsigned)g.XH;
    unsigned rr = hu / (unsigned)g.XH;
    const int y = (int)(rr % (unsigned)g.LY);
    rr /= (unsigned)g.LY;
    const int z = (int)(rr % (unsigned)g.LZ);
    const int t = (int)(rr / (unsigned)g.LZ);
    const int x = 2 * (int)xh + ((par + t + z + y) & 1);
    const long row = h - xh, sy = g.XH, sz = (long)g.LY * g.XH, stt = (long)g.LZ * sz;
    spinor<double> acc;
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int c = 0; c < 3; c++) acc.c[i][c] = cx<double>{0.0, 0.0};
    auto phase = [&](int mu) { return cx<double>{a.ph[mu][0], a.ph[mu][1]}; };
    auto trivial = [&](int mu) { return a.ph[mu][0] == 1.0 && a.ph[mu][1] == 0.0; };
    small_dir<0>(a.lk, par, other, phase(0), !trivial(0), h, t + 1 == g.T ? h - (g.T - 1) * stt : h + stt,
                 t == 0 ? h + (g.T - 1) * stt : h - stt, acc);
    small_dir<1>(a.lk, par, other, phase(1), !trivial(1), h, row + ((x + 1 == g.LX ? 0 : x + 1) >> 1),
                 row + ((x == 0 ? g.LX - 1 : x - 1) >> 1), acc);
    small_dir<2>(a.lk, par, other, phase(2), !trivial(2), h, y + 1 == g.LY ? h - (g.LY - 1) * sy : h + sy,
                 y == 0 ? h + (g.LY - 1) * sy : h - sy, acc);
    small_dir<3>(a.lk, par, other, phase(3), !trivial(3), h, z + 1 == g.LZ ? h - (g.LZ - 1) * sz : h + sz,
                 z == 0 ? h + (g.LZ - 1) * sz : h - sz, acc);
    spinor<double> v;
    in.load(s, v);
    const double m = sign * a.mut, k = a.kappa;
    const cx<double> Au = {1.0, m}, Ad = {-1.0, m}, Bu = {-k, 0.0}, Bd = {k, 0.0};
#pragma unroll
    for (int c = 0; c < 3; c++) {
        o.c[0][c] = fma(Au, v.c[0][c], Bu * acc.c[0][c]);
        o.c[1][c] = fma(Au, v.c[1][c], Bu * acc.c[1][c]);
        o.c[2][c] = fma(Ad, v.c[2][c], Bd * acc.c[2][c]);
        o.c[3][c] = fma(Ad, v.c[3][c], Bd * acc.c[3][c]);
    }
}

__device__ __forceinline__ double snorm(const spinor<double> &s)
{
    double n = 0.0;
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int c = 0; c < 3; c++) n = fmad(s.c[i][c].re, s.c[i][c].re, fmad(s.c[i][c].im, s.c[i][c].im, n));
    return n;
}

// block-wide sum, the same value in every lane (includes the barriers)
__device__ __forceinline__ double bsum(double v, double *red, double *bc)
{
    const double s = block_sum(v, red);
    if (threadIdx.x == 0) *bc = s;
    __syncthreads();
    const double r = *bc;
    __syncthreads();
    return r;
}

}  // namespace

template <class LK>
__global__ __launch_bounds__(SMALL_THREADS) void k_small_cg(SmallCgArgs<LK> a)
{
    __shared__ double red[SMALL_THREADS / 64];
    __shared__ double bc;
    const long n = 2 * a.g.vh;
    const long t0 = threadIdx.x, step = blockDim.x;
    CgScalars S = *a.sc;
    spinor<double> o, v, w;

    // r = b - A x (x as left by the previous call, zero at the start), p = r
    for (long s = t0; s < n; s += step) {
        small_q_site(a, a.x, -1, s, o);
        a.t.store(s, o);
    }
    __syncthreads();
    double part = 0.0, partb = 0.0;
    for (long s = t0; s < n; s += step) {
        small_q_site(a, a.t, +1, s, o);
        a.b.load(s, v);
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int c = 0; c < 3; c++) v.c[i][c] = v.c[i][c] - o.c[i][c];
        a.r.store(s, v);
        a.p.store(s, v);
        part += snorm(v);
        a.b.load(s, w);
        partb += snorm(w);
    }
    double rr = bsum(part, red, &bc);
    const double bb = bsum(partb, red, &bc);
    if (S.iter == 0 && S.reliable == 0) {
        S.bb = bb;
        S.target = a.tol2 * (a.relative ? bb : 1.0);
    }
    bool nan = !isfinite(rr);
    // CG from r (Sec. 4.4): alpha = rr / |Q^- p|^2, x += alpha p, r -= alpha A p, beta = rr' / rr
    while (!nan && rr >= S.target && rr > 0.0 && S.iter < a.max_iter) {
        part = 0.0;
        for (long s = t0; s < n; s += step) {
            small_q_site(a, a.p, -1, s, o);
            a.t.store(s, o);
            part += snorm(o);
        }
        const double pap = bsum(part, red, &bc);  // its barriers also publish t
        const double alpha = rr / pap;
        part = 0.0;
        for (long s = t0; s < n; s += step) {
            small_q_site(a, a.t, +1, s, o);
            a.x.load(s, v);
            a.p.load(s, w);
            spinor<double> r;
            a.r.load(s, r);
#pragma unroll
            for (int i = 0; i < 4; i++)
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    v.c[i][c].re = fmad(alpha, w.c[i][c].re, v.c[i][c].re);
                    v.c[i][c].im = fmad(alpha, w.c[i][c].im, v.c[i][c].im);
                    r.c[i][c].re = fmad(-alpha, o.c[i][c].re, r.c[i][c].re);
                    r.c[i][c].im = fmad(-alpha, o.c[i][c].im, r.c[i][c].im);
                }
            a.x.store(s, v);
            a.r.store(s, r);
            part += snorm(r);
        }
        const double rr_new = bsum(part, red, &bc);
        const double beta = rr_new / rr;
        rr = rr_new;
        S.iter += 1;
        nan = !isfinite(rr) || !isfinite(alpha) || !isfinite(beta);
        for (long s = t0; s < n; s += step) {
            a.r.load(s, v);
            a.p.load(s, w);
#pragma unroll
            for (int i = 0; i < 4; i++)
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    w.c[i][c].re = fmad(beta, w.c[i][c].re, v.c[i][c].re);
                    w.c[i][c].im = fmad(beta, w.c[i][c].im, v.c[i][c].im);
                }
            a.p.store(s, w);
        }
        __syncthreads();
    }
    // the true residual b - A x
    for (long s = t0; s < n; s += step) {
        small_q_site(a, a.x, -1, s, o);
        a.t.store(s, o);
    }
    __syncthreads();
    part = 0.0;
    for (long s = t0; s < n; s += step) {
        small_q_site(a, a.t, +1, s, o);
        a.b.load(s, v);
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int c = 0; c < 3; c++) v.c[i][c] = v.c[i][c] - o.c[i][c];
        part += snorm(v);
    }
    const double rt = bsum(part, red, &bc);
    if (threadIdx.x == 0) {
        S.rr = rt;
        S.reliable += 1;
        S.last_true = 1;
        S.nan = (nan || !isfinite(rt)) ? 1 : 0;
        S.done = (S.nan || rt < S.target || rt == 0.0) ? 1 : 0;
        *a.sc = S;
    }
}

template <class LK>
static hipError_t go_small(const Geom &g, const FieldDesc *f, const LinkDesc &lk, const OpParams &op, double tol2,
                           int relative, int max_iter, CgScalars *sc, hipStream_t st)
{
    SmallCgArgs<LK> a;
    a.g = g;
    a.b = make_sp<SpF64>(f[0]);
    a.x = make_sp<SpF64>(f[1]);
    a.r = make_sp<SpF64>(f[2]);
    a.p = make_sp<SpF64>(f[3]);
    a.t = make_sp<SpF64>(f[4]);
    a.ap = make_sp<SpF64>(f[5]);
    a.lk = make_lk<LK>(lk);
    for (int mu = 0; mu < 4; mu++) a.ph[mu][0] = op.ph[mu][0], a.ph[mu][1] = op.ph[mu][1];
    a.kappa = op.kappa[0];
    a.mut = op.mut[0];
    a.tol2 = tol2;
    a.relative = relative;
    a.max_iter = max_iter;
    a.sc = sc;
    hipLaunchKernelGGL(k_small_cg<LK>, dim3(1), dim3(SMALL_THREADS), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_small_cg(const Geom &g, const FieldDesc *f, const LinkDesc &lk, const OpParams &op, double tol2,
                           int relative, int max_iter, CgScalars *sc, hipStream_t st)
{
    for (int i = 0; i < 6; i++)
        if (f[i].prec != P64 || f[i].n != 2 * g.vh) return hipErrorInvalidValue;
    if (lk.fmt == LK64R) return go_small<L64R>(g, f, lk, op, tol2, relative, max_iter, sc, st);
    if (lk.fmt == LK64F) return go_small<L64F>(g, f, lk, op, tol2, relative, max_iter, sc, st);
    return hipErrorInvalidValue;
}

}  // namespace tmq
