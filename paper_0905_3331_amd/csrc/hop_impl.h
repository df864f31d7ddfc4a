// hop_impl.h -- the hopping half-sweep H_eo / H_oe with fused site-term epilogues.
//
// Included by one translation unit per spinor format (hop_f64.hip, ...), so
// that the many template instantiations compile in parallel; hop.hip holds
// the dispatch.
//
// One output site per lane.  For each of the 8 neighbours the lane loads the
// neighbour spinor, projects it to two spin components with (1 +- gamma_mu)
// (Sec. 4.1), multiplies both by the link U(x,mu) or U(x-mu,mu)^+ (each link
// is read exactly once per half-sweep: the forward links of the output
// parity, the backward links of the input parity), multiplies by the boundary
// phase e^{+-i theta_mu pi/L_mu} (Sec. 4.1.2; skipped where the phase is 1)
// and accumulates the rebuilt four-spinor.  The epilogue forms
// out = A * self + B * acc per spin half, which covers both factors of the
// even/odd operator (eqs. (eo3), (eo4)) and the full-lattice operator, and
// optionally reduces |out|^2 per block.
//
// Work distribution: blocks of 256 lanes over consecutive eo indices (x
// fastest, then y, z, t).  Hardware hands consecutive workgroups to the 8 XCDs
// in turn; the block index is remapped so that each XCD walks a contiguous
// slab of the lattice and its private L2 sees the y/z/t neighbours of its
// own sites.
#pragma once
#include <algorithm>
#include <type_traits>

#include "devutil.h"
#include "views.h"

namespace tmq {

__device__ __forceinline__ int xcd_remap(int bid, int nblk)
{
    // nblk is a multiple of 8: XCD k = bid % 8 gets logical blocks [k*nblk/8, (k+1)*nblk/8)
    return (bid & 7) * (nblk >> 3) + (bid >> 3);
}

// format of the solution correction updated by the fused CG epilogue
template <class SP>
struct XsOf {
    using type = SpF32;
};
template <>
struct XsOf<SpF64> {
    using type = SpF64;
};

enum HopEp { EP_STORE = 0, EP_CG = 1, EP_RES = 2 };

// Divisors of a batched 16-bit launch's block and site decode (FastDiv): the
// blocks of an RHS group per XCD (grp), the group size (gsz) and the size of
// the last group (glast); the x-row and (t, z) plane lengths, LY and LZ, and
// the sites of one time-slice of an XCD's z-slab (or of one z-plane of its
// t-slab), which come in two sizes: slab[1] for the XCDs that take one plane
// (or slice) more.
struct SiteDiv {
    FastDiv grp, gsz, glast;
    FastDiv xh, ly, lz, plane, slab[2];
};
inline SiteDiv make_site_div(const Geom &g, int ord, int nblk, int group, int ntup)
{
    SiteDiv d;
    d.grp = make_fastdiv((uint32_t)(nblk >> 3) * (uint32_t)group);
    d.gsz = make_fastdiv((uint32_t)group);
    d.glast = make_fastdiv((uint32_t)(ntup - (ntup - 1) / group * group));
    const uint32_t plane = (uint32_t)g.LY * (uint32_t)g.XH;
    d.xh = make_fastdiv((uint32_t)g.XH);
    d.ly = make_fastdiv((uint32_t)g.LY);
    d.lz = make_fastdiv((uint32_t)g.LZ);
    d.plane = make_fastdiv(plane);
    const uint32_t ext = ord == ORD_TSLAB ? (uint32_t)g.T : (uint32_t)g.LZ;
    d.slab[0] = make_fastdiv(std::max(1u, ext >> 3) * plane);
    d.slab[1] = make_fastdiv(((ext >> 3) + 1) * plane);
    return d;
}
// n / d for the divisor of f (FastDiv; n < 2^31)
__device__ __forceinline__ uint32_t fdiv(uint32_t n, const FastDiv &f) { return (__umulhi(n, f.m) + n) >> f.s; }

// Site-term coefficients of a batched 16-bit launch, per right-hand side
// (doublets: per doublet), formed on the host in FP64 by the operations the
// single-field launches perform in each lane and rounded to FP32 once, so the
// two agree bit for bit: m = sigma mut, e = eps, c = kappa^2 / (1 + m^2)
// (doublets: kappa^2 / (1 + m^2 - e^2)), cm = c m, ce = c e
struct EpiCoef {
    float c, cm, ce, m, e;
};

template <class SP, class LK>
struct HopArgs {
    Geom g;
    int out_par;
    int epi, sign;
    int phase_mask;  // bit mu set when the boundary phase of direction mu is not 1
    int nblk;        // blocks per RHS
    int group;       // RHS processed together per site block (see the kernel)
    BatchView<SP> in, self, out;
    LK lk;
    OpParams op;
    RhsList rl;
    double *partial;
    long pstride;
    const CgScalars *scal;
    float one;  // 1.0, opaque to the compiler (see code_lo in fields.h)
    // fused epilogues (EPI_K2_CG, EPI_K2_RES)
    BatchView<SP> cg_r, cg_p;
    BatchView<typename XsOf<SP>::type> cg_x;
    // batched 16-bit launches
    SiteDiv dv;
    EpiCoef ec[MAX_RHS];
};

// x + C y for C = 1, -1, i, -i (selector 0..3), x and y complex 16-bit codes
template <int C, bool BF>
__device__ __forceinline__ cx<float> addc(uint32_t x, uint32_t y, float one)
{
    const float xr = code_lo<BF>(x), xi = code_hi<BF>(x), yr = code_lo<BF>(y), yi = code_hi<BF>(y);
    if (C == 0) return {fmad(xr, one, yr), fmad(xi, one, yi)};
    if (C == 1) return {fmad(xr, one, -yr), fmad(xi, one, -yi)};
    if (C == 2) return {fmad(xr, one, -yi), fmad(xi, one, yr)};
    return {fmad(xr, one, yi), fmad(xi, one, -yr)};
}

// first two rows of (1 + S gamma_MU) s from the codes of s (same table as
// project() in spin.h), unscaled
template <int MU, int S, bool BF>
__device__ __forceinline__ void project_codes(const uint32_t w[12], float one, half<float> &h)
{
#pragma unroll
    for (int a = 0; a < 3; a++) {
        const uint32_t s0 = w[a], s1 = w[3 + a], s2 = w[6 + a], s3 = w[9 + a];
        if (MU == 0) {
            h.c[0][a] = S > 0 ? addc<1, BF>(s0, s2, one) : addc<0, BF>(s0, s2, one);
            h.c[1][a] = S > 0 ? addc<1, BF>(s1, s3, one) : addc<0, BF>(s1, s3, one);
        } else if (MU == 1) {
            h.c[0][a] = S > 0 ? addc<3, BF>(s0, s3, one) : addc<2, BF>(s0, s3, one);
            h.c[1][a] = S > 0 ? addc<3, BF>(s1, s2, one) : addc<2, BF>(s1, s2, one);
        } else if (MU == 2) {
            h.c[0][a] = S > 0 ? addc<1, BF>(s0, s3, one) : addc<0, BF>(s0, s3, one);
            h.c[1][a] = S > 0 ? addc<0, BF>(s1, s2, one) : addc<1, BF>(s1, s2, one);
        } else {
            h.c[0][a] = S > 0 ? addc<3, BF>(s0, s2, one) : addc<2, BF>(s0, s2, one);
            h.c[1][a] = S > 0 ? addc<2, BF>(s1, s3, one) : addc<3, BF>(s1, s3, one);
        }
    }
}

// acc += sc * T(h) for T = identity, negation, i, -i (selector 0..3)
template <int T>
__device__ __forceinline__ void acc_fma(cx<float> &acc, cx<float> h, float sc)
{
    if (T == 0) acc = {fmad(sc, h.re, acc.re), fmad(sc, h.im, acc.im)};
    if (T == 1) acc = {fmad(-sc, h.re, acc.re), fmad(-sc, h.im, acc.im)};
    if (T == 2) acc = {fmad(-sc, h.im, acc.re), fmad(sc, h.re, acc.im)};
    if (T == 3) acc = {fmad(sc, h.im, acc.re), fmad(-sc, h.re, acc.im)};
}

// acc += sc * (1 + S gamma_MU) image rebuilt from h (reconstruct_add of spin.h, scaled)
template <int MU, int S>
__device__ __forceinline__ void reconstruct_fma(spinor<float> &acc, const half<float> &h, float sc)
{
#pragma unroll
    for (int a = 0; a < 3; a++) {
        acc_fma<0>(acc.c[0][a], h.c[0][a], sc);
        acc_fma<0>(acc.c[1][a], h.c[1][a], sc);
        if (MU == 0) {
            acc_fma<(S > 0 ? 1 : 0)>(acc.c[2][a], h.c[0][a], sc);
            acc_fma<(S > 0 ? 1 : 0)>(acc.c[3][a], h.c[1][a], sc);
        } else if (MU == 1) {
            acc_fma<(S > 0 ? 2 : 3)>(acc.c[2][a], h.c[1][a], sc);
            acc_fma<(S > 0 ? 2 : 3)>(acc.c[3][a], h.c[0][a], sc);
        } else if (MU == 2) {
            acc_fma<(S > 0 ? 0 : 1)>(acc.c[2][a], h.c[1][a], sc);
            acc_fma<(S > 0 ? 1 : 0)>(acc.c[3][a], h.c[0][a], sc);
        } else {
            acc_fma<(S > 0 ? 2 : 3)>(acc.c[2][a], h.c[0][a], sc);
            acc_fma<(S > 0 ? 3 : 2)>(acc.c[3][a], h.c[1][a], sc);
        }
    }
}

// One hop of a 16-bit spinor (DIR 0 forward, 1 backward) from its codes and
// scale and the loaded link: project the codes, multiply by the link, and
// apply the site's scale (times the phase when PH) when accumulating
template <int MU, int DIR, bool PH, class SP, class LK, typename R>
__device__ __forceinline__ void coded_hop_ph(const HopArgs<SP, LK> &a, const typename LK::Loaded &u,
                                             const uint32_t (&c)[12], float sc, spinor<R> &acc)
{
    constexpr bool phase = PH;
    half<R> p, w;
    project_codes<MU, DIR == 0 ? +1 : -1, SP::bf>(c, a.one, p);
    a.lk.template apply<DIR == 1>(u, p, w);
    if (phase) {
        const cx<R> ph = {(R)a.op.ph[MU][0], (R)a.op.ph[MU][1]};
        const cx<R> phd = DIR == 0 ? ph : conj(ph);
        half_scale(w, cx<R>{sc * phd.re, sc * phd.im});
        reconstruct_add<MU, DIR == 0 ? +1 : -1>(acc, w);
    } else {
        reconstruct_fma<MU, DIR == 0 ? +1 : -1>(acc, w, sc);
    }
}
// the same with the phase flag of direction MU read from the launch (uniform)
template <int MU, int DIR, class SP, class LK, typename R>
__device__ __forceinline__ void coded_hop(const HopArgs<SP, LK> &a, const typename LK::Loaded &u,
                                          const uint32_t (&c)[12], float sc, spinor<R> &acc)
{
    if ((a.phase_mask >> MU) & 1)
        coded_hop_ph<MU, DIR, true>(a, u, c, sc, acc);
    else
        coded_hop_ph<MU, DIR, false>(a, u, c, sc, acc);
}

// One hop of an FP64 or FP32 spinor (DIR 0 forward, 1 backward) with the
// loaded link: project, multiply by the link, apply the phase, accumulate
template <int MU, int DIR, class SP, class LK, typename R>
__device__ __forceinline__ void plain_hop(const HopArgs<SP, LK> &a, const typename LK::Loaded &u,
                                          const spinor<R> &sp, spinor<R> &acc)
{
    const bool phase = (a.phase_mask >> MU) & 1;  // uniform over the launch
    half<R> p, w;
    project<MU, DIR == 0 ? +1 : -1>(sp, p);
    a.lk.template apply<DIR == 1>(u, p, w);
    if (phase) {
        const cx<R> ph = {(R)a.op.ph[MU][0], (R)a.op.ph[MU][1]};
        half_scale(w, DIR == 0 ? ph : conj(ph));
    }
    reconstruct_add<MU, DIR == 0 ? +1 : -1>(acc, w);
}

// The contribution of direction MU (forward and backward hop) for the G
// right-hand sides of a lane: each link is loaded once and applied to the
// projected neighbour spinor of every RHS in turn; per RHS the operations are
// those of a lane with one RHS.
template <int MU, bool NT, int G, class SP, class LK, typename R>
__device__ __forceinline__ void hop_dir(const HopArgs<SP, LK> &a, const SP (&in)[G], const bool (&live)[G],
                                        spinor<R> (&acc)[G], long h, long hf, long hb)
{
    typename LK::Loaded u;
#pragma unroll
    for (int dir = 0; dir < 2; dir++) {
        // forward: e^{i theta pi/L} U(x,mu) (1 + gamma_mu) psi(x+mu), U at the output site;
        // backward: e^{-i theta pi/L} U(x-mu,mu)^+ (1 - gamma_mu) psi(x-mu), U at the neighbour
        const long hn = dir == 0 ? hf : hb;
        a.lk.template load_link<NT>(dir == 0 ? a.out_par : a.out_par ^ 1, MU, dir == 0 ? h : hb, u);
#pragma unroll
        for (int gi = 0; gi < G; gi++) {
            if (!live[gi]) continue;
            if constexpr (SP::coded) {
                uint32_t c[12];
                float sc;
                in[gi].load_codes(hn, c, sc);
                if (dir == 0)
                    coded_hop<MU, 0>(a, u, c, sc, acc[gi]);
                else
                    coded_hop<MU, 1>(a, u, c, sc, acc[gi]);
            } else {
                spinor<R> sp;
                in[gi].load(hn, sp);
                if (dir == 0)
                    plain_hop<MU, 0>(a, u, sp, acc[gi]);
                else
                    plain_hop<MU, 1>(a, u, sp, acc[gi]);
            }
        }
    }
}

// The loads of one direction of a 16-bit spinor with FP16 two-row links
// (forward and backward hop), taken before any arithmetic on them
struct Raw16 {
    uint32_t lw[2][6];  // link rows 0 and 1
    uint32_t c[2][12];  // neighbour codes
    float sc[2];        // neighbour scales
};
template <int MU, bool NT, class SP, class LK>
__device__ __forceinline__ void load16(const HopArgs<SP, LK> &a, const SP &in, long h, long hf, long hb, Raw16 &d)
{
    a.lk.template load_raw<NT>(a.out_par, MU, h, d.lw[0]);
    in.load_codes(hf, d.c[0], d.sc[0]);
    a.lk.template load_raw<NT>(a.out_par ^ 1, MU, hb, d.lw[1]);
    in.load_codes(hb, d.c[1], d.sc[1]);
}
// the arithmetic of hop_dir for one RHS on loaded data
template <int MU, class SP, class LK, typename R>
__device__ __forceinline__ void math16(const HopArgs<SP, LK> &a, const Raw16 &d, spinor<R> &acc)
{
#pragma unroll
    for (int dir = 0; dir < 2; dir++) {
        typename LK::Loaded u;
#pragma unroll
        for (int k = 0; k < 6; k++) u.w[k] = d.lw[dir][k];
        a.lk.rebuild(u);
        if (dir == 0)
            coded_hop<MU, 0>(a, u, d.c[0], d.sc[0], acc);
        else
            coded_hop<MU, 1>(a, u, d.c[1], d.sc[1], acc);
    }
}

// The same for FP32 spinors with FP32 two-row links, one direction at a time
// (two directions at once need about 210 VGPRs and were slower)
struct Raw32 {
    su3<float> u[2];        // rows 0 and 1 of the forward and backward link
    spinor<float> sp[2];    // forward and backward neighbour
};
template <int MU, bool NT, class SP, class LK>
__device__ __forceinline__ void load32(const HopArgs<SP, LK> &a, const SP &in, long h, long hf, long hb, Raw32 &d)
{
    a.lk.template load_rows<NT>(a.out_par, MU, h, d.u[0]);
    in.load(hf, d.sp[0]);
    a.lk.template load_rows<NT>(a.out_par ^ 1, MU, hb, d.u[1]);
    in.load(hb, d.sp[1]);
}
// the arithmetic of hop_dir for one RHS on loaded data
template <int MU, class SP, class LK>
__device__ __forceinline__ void math32(const HopArgs<SP, LK> &a, Raw32 &d, spinor<float> &acc)
{
#pragma unroll
    for (int dir = 0; dir < 2; dir++) {
        su3_third_row(d.u[dir]);
        if (dir == 0)
            plain_hop<MU, 0>(a, d.u[0], d.sp[0], acc);
        else
            plain_hop<MU, 1>(a, d.u[1], d.sp[1], acc);
    }
}

// The partner lane's value (lanes 2i and 2i+1 swap: DPP quad permutation
// [1, 0, 3, 2]).  Both lanes of a pair are active or inactive together.
__device__ __forceinline__ float pair_swap(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));
}
__device__ __forceinline__ double pair_swap(double v)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, 0xB1, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), 0xB1, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// The site terms of the flavour doublet (eq. (Dh)).  A doublet's two
// flavours at one site sit in a lane pair (flavour f = lane & 1, f = 0 the
// upper); acc is this lane's hop sum, the partner's comes by pair_swap.
// K1 multiplies by kappa^2 A^-1, A^-1 = (1 - i m g5 tau^3 - e tau^1) / d with
// m = sigma mubar, e = epsbar, d = 1 + m^2 - e^2; K2 forms g5 (A self - acc).
// Upper spins have g5 = +1, lower g5 = -1; tau^3 is +1 on the upper flavour.
template <class SP, class LK, typename R>
__device__ __forceinline__ void nd_mix(const HopArgs<SP, LK> &a, spinor<R> &acc, int rhs, long h)
{
    const int d = rhs >> 1;
    const bool up = (rhs & 1) == 0;
    const double kap = a.op.kappa[d], m = a.sign * a.op.mut[d], e = a.op.eps[d];
    if (a.epi == EPI_K1) {
        const double c = kap * kap / (1.0 + m * m - e * e);
        const cx<R> pm = {(R)c, (R)(-c * m)}, pp = {(R)c, (R)(c * m)};  // c (1 - i m), c (1 + i m)
        const R ce = (R)(-c * e);
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int c3 = 0; c3 < 3; c3++) {
                const cx<R> own = acc.c[i][c3];
                const cx<R> other = {pair_swap(own.re), pair_swap(own.im)};
                // c (1 -+ i m g5) own - c e other (upper / lower flavour)
                acc.c[i][c3] = fma((i < 2) == up ? pm : pp, own, ce * other);
            }
    } else {
        spinor<R> so, sx;
        a.self.at(rhs).load(h, so);
        a.self.at(rhs ^ 1).load(h, sx);
        const cx<R> one_pm = {R(1), (R)m}, one_mm = {R(1), (R)(-m)};  // 1 + i m, 1 - i m
        const R ee = (R)e;
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int c3 = 0; c3 < 3; c3++) {
                // A self = (1 +- i m g5) own + e other
                const cx<R> as = fma((i < 2) == up ? one_pm : one_mm, so.c[i][c3], ee * sx.c[i][c3]);
                const cx<R> o = as - acc.c[i][c3];
                acc.c[i][c3] = i < 2 ? o : -o;
            }
    }
}

// K2 of eq. (eo4) with the own-site term first: out = g5[(1 + s i mut g5) self - H]
// is Au self - H on the upper spins and Ad self + H on the lower (Au = 1 + s i mut,
// Ad = -1 + s i mut, H the hop sum), so the accumulator starts from -Au self
// (upper) and Ad self (lower), the hops are added to it, and the epilogue only
// flips the sign of the upper spins.  The own-site spinor is then dead before the hops, which keeps the
// half-sweep within fewer registers; every K2 store launch, single-field or
// batched, sums in this order, so their results agree bit for bit.
template <typename R, class SP, class LK>
__device__ __forceinline__ spinor<R> k2_self_first(const HopArgs<SP, LK> &a, int rhs, long h)
{
    spinor<R> sf, acc;
    a.self.at(rhs).load(h, sf);
    const double m = a.sign * a.op.mut[rhs];
    const cx<R> Au = cx<R>{R(1), (R)m}, Ad = cx<R>{R(-1), (R)m};
#pragma unroll
    for (int c = 0; c < 3; c++) {
        acc.c[0][c] = -(Au * sf.c[0][c]);
        acc.c[1][c] = -(Au * sf.c[1][c]);
        acc.c[2][c] = Ad * sf.c[2][c];
        acc.c[3][c] = Ad * sf.c[3][c];
    }
    return acc;
}

// The epilogue of a half-sweep at output site h for right-hand side rhs (batch
// index) from the hop sum acc_in: the site terms of the launch's epilogue
// (HopEpi), then the store (non-temporal when NTOUT) or the fused CG /
// residual update; returns |out|^2 when NORM (else 0).  PRESELF: the launch is
// EPI_K2 and acc_in already holds the own-site term (k2_self_first), so out =
// B acc with B = -1 on the upper spins and +1 on the lower.  TAB: the
// coefficients come from the launch's table (EpiCoef; batched 16-bit launches).
template <class SP, class LK, bool SELF, bool NORM, int EP, bool ND, bool NTOUT = true, bool PRESELF = false,
          bool TAB = false, typename R>
__device__ __forceinline__ double hop_epilogue(const HopArgs<SP, LK> &a, const spinor<R> &acc_in, int rhs, long h)
{
    double nrm = 0.0;
    const int si = ND ? rhs >> 1 : rhs;  // index of the scalars
    // epilogue coefficients of this RHS (upper spins: gamma_5 = +1, lower: -1)
    const double kap = a.op.kappa[rhs], m = a.sign * a.op.mut[rhs];
    cx<R> Au, Ad, Bu, Bd;
    if (a.epi == EPI_K1) {
        Au = Ad = cx<R>{R(0), R(0)};
        if constexpr (TAB && !ND) {
            const EpiCoef &k = a.ec[rhs];
            Bu = cx<R>{k.c, -k.cm};
            Bd = cx<R>{k.c, k.cm};
        } else {
            const double c = kap * kap / (1.0 + m * m);
            Bu = cx<R>{(R)c, (R)(-c * m)};
            Bd = cx<R>{(R)c, (R)(c * m)};
        }
    } else if (a.epi == EPI_SRC) {
        Au = Ad = cx<R>{R(1), R(0)};
        Bu = Bd = cx<R>{(R)kap, R(0)};
    } else if (a.epi == EPI_REC) {
        const double c = 1.0 / (1.0 + m * m);
        Au = cx<R>{(R)c, (R)(-c * m)};
        Ad = cx<R>{(R)c, (R)(c * m)};
        Bu = cx<R>{(R)(kap * c), (R)(-kap * c * m)};
        Bd = cx<R>{(R)(kap * c), (R)(kap * c * m)};
    } else {
        const double b = a.epi == EPI_FULL ? kap : 1.0;
        R mr;
        if constexpr (TAB && !ND)
            mr = a.ec[rhs].m;
        else
            mr = (R)m;
        Au = cx<R>{R(1), mr};
        Ad = cx<R>{R(-1), mr};
        Bu = cx<R>{(R)(-b), R(0)};
        Bd = cx<R>{(R)b, R(0)};
    }
    const spinor<R> &ac = acc_in;
    spinor<R> o;
    if (ND) {
        o = ac;  // the doublet's site terms are applied already
    } else if (PRESELF) {
#pragma unroll
        for (int c = 0; c < 3; c++) {
            o.c[0][c] = -ac.c[0][c];
            o.c[1][c] = -ac.c[1][c];
            o.c[2][c] = ac.c[2][c];
            o.c[3][c] = ac.c[3][c];
        }
    } else if (SELF) {
        spinor<R> sf;
        a.self.at(rhs).load(h, sf);
#pragma unroll
        for (int c = 0; c < 3; c++) {
            o.c[0][c] = fma(Au, sf.c[0][c], Bu * ac.c[0][c]);
            o.c[1][c] = fma(Au, sf.c[1][c], Bu * ac.c[1][c]);
            o.c[2][c] = fma(Ad, sf.c[2][c], Bd * ac.c[2][c]);
            o.c[3][c] = fma(Ad, sf.c[3][c], Bd * ac.c[3][c]);
        }
    } else {
#pragma unroll
        for (int c = 0; c < 3; c++) {
            o.c[0][c] = Bu * ac.c[0][c];
            o.c[1][c] = Bu * ac.c[1][c];
            o.c[2][c] = Bd * ac.c[2][c];
            o.c[3][c] = Bd * ac.c[3][c];
        }
    }
    if (EP == EP_CG) {
        // CG update: x += alpha p ; r -= alpha (A p) ; |r|^2
        using XS = typename XsOf<SP>::type;
        using RX = typename XS::real;
        const double al = a.scal[si].alpha;
        const R ar = (R)al;
        const RX ax = (RX)al;
        spinor<R> rr, pp;
        spinor<RX> xx;
        a.cg_r.at(rhs).load(h, rr);
        a.cg_p.at(rhs).load(h, pp);
        a.cg_x.at(rhs).load(h, xx);
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int c = 0; c < 3; c++) {
                xx.c[i][c].re = fmad(ax, (RX)pp.c[i][c].re, xx.c[i][c].re);
                xx.c[i][c].im = fmad(ax, (RX)pp.c[i][c].im, xx.c[i][c].im);
                rr.c[i][c].re = fmad(-ar, o.c[i][c].re, rr.c[i][c].re);
                rr.c[i][c].im = fmad(-ar, o.c[i][c].im, rr.c[i][c].im);
            }
        a.cg_x.at(rhs).store(h, xx);
        a.cg_r.at(rhs).store(h, rr);
        o = rr;
    } else if (EP == EP_RES) {
        // true residual r = b - A x
        spinor<R> bb;
        a.cg_p.at(rhs).load(h, bb);
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int c = 0; c < 3; c++) o.c[i][c] = bb.c[i][c] - o.c[i][c];
        a.cg_r.at(rhs).store(h, o);
    } else {
        a.out.at(rhs).template store<NTOUT>(h, o);
    }
    if (NORM) {
        R n2 = R(0);
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int c = 0; c < 3; c++) n2 += norm2(o.c[i][c]);
        nrm = (double)n2;
    }
    return nrm;
}

// The order in which a half-sweep sums its directions (t, x, y, z = 0..3):
// t, x, y, z, except for K1 (no own-site term) of 16-bit and FP64 spinors,
// which takes x, y, t, z.  The 16-bit kernel loads two directions at a time in
// this order, and its K1 measured 2.5 % faster at 32^3x64 with the x and y
// neighbours (the nearest in memory) in the first group, FP64 K1 1.6 %
// faster; 16-bit K2 was 1 % slower that way, FP32 K1 1.4 % slower.  Every
// kernel sums in this order, so a batch equals its solves alone bit for bit
// whichever kernel runs each.
template <bool XY_FIRST>
__host__ __device__ constexpr int k1_order(int i)
{
    return XY_FIRST ? (i == 0 ? 1 : i == 1 ? 2 : i == 2 ? 0 : 3) : i;
}

// Variant bits: ORD is the order in which an XCD's blocks walk the lattice
// (physical block b runs on XCD j = b % 8): ORD_PLAIN gives XCD j the j-th
// eighth of the eo index range (a range of time-slices, lexicographic);
// ORD_ZSLAB gives it its own range of z-planes, walked with t outermost, so
// that the sites of time-slices t-1, t, t+1 that the XCD needs at a time fit
// its L2; ORD_TSLAB gives it a range of time-slices walked with z outermost
// (half the boundary planes of ORD_ZSLAB when T >= LZ).  NT makes the link
// loads non-temporal (single RHS); SB puts a scheduling barrier between
// directions.  The autotuner picks the fastest variant per format and lattice.
//
// Batches: the RHS are taken in groups of `group`; an XCD sweeps its whole
// share of sites for one group before the next, and within a group its
// consecutive blocks apply the same links to every RHS of the group in turn.
// The links are then fetched from HBM once per group, while the neighbour
// spinors of a group (three time-slices of the XCD's share per RHS) still fit
// its L2; the host sizes the group for that.  With one RHS this is the
// single-field order, and each RHS's arithmetic and partial sums do not depend
// on the batch around it.
//
// Doublets (ND): a block covers HOP_BLOCK / 2 sites, each in a lane pair
// holding the doublet's two flavours (tuple = doublet = RHS pair 2d, 2d + 1
// of the list); both lanes load the same link at once, so it is fetched once.
template <class SP, class LK, bool SELF, bool NORM, bool NT, int ORD, bool SB, int G, int EP, bool ND = false>
__global__ __launch_bounds__(HOP_BLOCK) void hop_kernel(HopArgs<SP, LK> a)
{
    static_assert(!ND || G == 1, "a doublet lane holds one flavour, its partner lane the other");
    constexpr int SPB = ND ? HOP_BLOCK / 2 : HOP_BLOCK;   // sites per block
    const int ls = ND ? (int)(threadIdx.x >> 1) : (int)threadIdx.x;  // site of the lane within the block
    using R = typename LK::real;
    const Geom &g = a.g;
    const int j = blockIdx.x & 7;
    const int k = blockIdx.x >> 3;
    const int nb = a.nblk >> 3;                        // site blocks of this XCD's share
    const int ntup = ND ? a.rl.n / 2 : (a.rl.n + G - 1) / G;  // tuples of G RHS (one per lane), or doublets
    const int GR = a.group, gr = k / (nb * GR);        // group of tuples of this block
    const int gsize = min(GR, ntup - gr * GR);         // the last group may be smaller
    const int within = k - gr * nb * GR;
    const int sb = within / gsize;                     // site block within the XCD's share
    const int tup = gr * GR + (within - sb * gsize);
    int rhs[G];
    bool live[G];
    bool any = false;
#pragma unroll
    for (int gi = 0; gi < G; gi++) {
        const int ri = ND ? 2 * tup + (int)(threadIdx.x & 1) : tup * G + gi;
        live[gi] = ri < a.rl.n;
        rhs[gi] = live[gi] ? a.rl.idx[ri] : 0;
        if (live[gi] && a.scal && a.scal[ND ? rhs[gi] >> 1 : rhs[gi]].done) live[gi] = false;
        any |= live[gi];
    }
    if (!any) return;
    const long plane = (long)g.LY * g.XH;  // sites of one (t, z) plane
    long h;
    int t, z, y, pidx;
    unsigned xh;
    bool active;
    if (ORD == ORD_ZSLAB) {
        const int zb = g.LZ >> 3, zr = g.LZ & 7;
        const int zc = zb + (j < zr ? 1 : 0), z0 = j * zb + (j < zr ? j : zr);
        const long S = (long)zc * plane;  // sites of one time-slice of this slab
        const long l = (long)sb * SPB + ls;
        active = l < (long)g.T * S;
        const unsigned lu = active ? (unsigned)l : 0u;
        t = (int)(lu / (unsigned)S);
        const unsigned rem = lu - (unsigned)t * (unsigned)S;
        z = z0 + (int)(rem / (unsigned)plane);
        const unsigned r2 = rem - (unsigned)(z - z0) * (unsigned)plane;
        y = (int)(r2 / (unsigned)g.XH);
        xh = r2 - (unsigned)y * (unsigned)g.XH;
        h = ((long)t * g.LZ + z) * plane + (long)y * g.XH + xh;
        pidx = 8 * sb + j;
    } else if (ORD == ORD_TSLAB) {
        const int tb = g.T >> 3, tr = g.T & 7;
        const int tc = tb + (j < tr ? 1 : 0), t0 = j * tb + (j < tr ? j : tr);
        const long P = (long)tc * plane;  // sites of one z-plane of this block of time-slices
        const long l = (long)sb * SPB + ls;
        active = l < (long)g.LZ * P;
        const unsigned lu = active ? (unsigned)l : 0u;
        z = (int)(lu / (unsigned)P);
        const unsigned rem = lu - (unsigned)z * (unsigned)P;
        t = t0 + (int)(rem / (unsigned)plane);
        const unsigned r2 = rem - (unsigned)(t - t0) * (unsigned)plane;
        y = (int)(r2 / (unsigned)g.XH);
        xh = r2 - (unsigned)y * (unsigned)g.XH;
        h = ((long)t * g.LZ + z) * plane + (long)y * g.XH + xh;
        pidx = 8 * sb + j;
    } else {
        const int lb = j * (a.nblk >> 3) + sb;
        h = (long)lb * SPB + ls;
        active = h < g.vh;
        const unsigned hu = active ? (unsigned)h : 0u;
        xh = hu % (unsigned)g.XH;
        unsigned r = hu / (unsigned)g.XH;
        y = (int)(r % (unsigned)g.LY);
        r /= (unsigned)g.LY;
        z = (int)(r % (unsigned)g.LZ);
        t = (int)(r / (unsigned)g.LZ);
        pidx = lb;
    }
    double nrm[G];
#pragma unroll
    for (int gi = 0; gi < G; gi++) nrm[gi] = 0.0;
    if (active) {
        SP in[G];
#pragma unroll
        for (int gi = 0; gi < G; gi++) in[gi] = a.in.at(rhs[gi]);
        // x parity makes (t+z+y+x) = out_par mod 2
        const int x = 2 * (int)xh + ((a.out_par + t + z + y) & 1);
        const long row = h - xh;  // eo index of (t, z, y, 0)
        const long sy = g.XH, sz = plane, stt = (long)g.LZ * plane;

        // K2 store launches start from the own-site term (k2_self_first)
        const bool pre = SELF && !ND && EP == EP_STORE && a.epi == EPI_K2;
        spinor<R> acc[G];
#pragma unroll
        for (int gi = 0; gi < G; gi++) {
            if (pre && live[gi]) {
                acc[gi] = k2_self_first<R>(a, rhs[gi], h);
                continue;
            }
#pragma unroll
            for (int i = 0; i < 4; i++)
#pragma unroll
                for (int c = 0; c < 3; c++) acc[gi].c[i][c] = cx<R>{R(0), R(0)};
        }

        // forward and backward neighbours in t, x, y, z (periodic), formed where used
        auto f0 = [&] { return t + 1 == g.T ? h - (g.T - 1) * stt : h + stt; };
        auto b0 = [&] { return t == 0 ? h + (g.T - 1) * stt : h - stt; };
        auto f1 = [&] { return row + ((x + 1 == g.LX ? 0 : x + 1) >> 1); };
        auto b1 = [&] { return row + ((x == 0 ? g.LX - 1 : x - 1) >> 1); };
        auto f2 = [&] { return y + 1 == g.LY ? h - (g.LY - 1) * sy : h + sy; };
        auto b2 = [&] { return y == 0 ? h + (g.LY - 1) * sy : h - sy; };
        auto f3 = [&] { return z + 1 == g.LZ ? h - (g.LZ - 1) * sz : h + sz; };
        auto b3 = [&] { return z == 0 ? h + (g.LZ - 1) * sz : h - sz; };
        // the directions in the order of the sum (K1_ORDER), neighbours by index
        constexpr bool XY1 = (SP::coded || __is_same(SP, SpF64)) && !SELF;
        constexpr int D0 = k1_order<XY1>(0), D1 = k1_order<XY1>(1), D2 = k1_order<XY1>(2), D3 = k1_order<XY1>(3);
        auto fn = [&](auto m) -> long {
            constexpr int M = decltype(m)::value;
            if constexpr (M == 0) return f0();
            else if constexpr (M == 1) return f1();
            else if constexpr (M == 2) return f2();
            else return f3();
        };
        auto bn = [&](auto m) -> long {
            constexpr int M = decltype(m)::value;
            if constexpr (M == 0) return b0();
            else if constexpr (M == 1) return b1();
            else if constexpr (M == 2) return b2();
            else return b3();
        };
        using I0 = std::integral_constant<int, D0>;
        using I1 = std::integral_constant<int, D1>;
        using I2 = std::integral_constant<int, D2>;
        using I3 = std::integral_constant<int, D3>;
        if constexpr (SP::coded && __is_same(LK, L16R) && NT && G == 1) {
            // 16-bit spinors, single-RHS (or single-doublet) launch: the loads of
            // two directions (four hops) are issued before their arithmetic,
            // which shortens the chain of dependent memory waits of a lane; same
            // arithmetic, same order (batched launches keep more waves resident
            // instead)
            if (live[0]) {
                Raw16 d0, d1;
                load16<D0, NT>(a, in[0], h, fn(I0{}), bn(I0{}), d0);
                load16<D1, NT>(a, in[0], h, fn(I1{}), bn(I1{}), d1);
                math16<D0>(a, d0, acc[0]);
                math16<D1>(a, d1, acc[0]);
                if (SB) __builtin_amdgcn_sched_barrier(0);
                load16<D2, NT>(a, in[0], h, fn(I2{}), bn(I2{}), d0);
                load16<D3, NT>(a, in[0], h, fn(I3{}), bn(I3{}), d1);
                math16<D2>(a, d0, acc[0]);
                math16<D3>(a, d1, acc[0]);
            }
        } else if constexpr (__is_same(SP, SpF32) && __is_same(LK, L32R) && NT && G == 1) {
            // FP32, single-RHS (or single-doublet) launch: the four loads of a
            // direction before its arithmetic
            if (live[0]) {
                Raw32 d;
                load32<0, NT>(a, in[0], h, f0(), b0(), d);
                math32<0>(a, d, acc[0]);
                if (SB) __builtin_amdgcn_sched_barrier(0);
                load32<1, NT>(a, in[0], h, f1(), b1(), d);
                math32<1>(a, d, acc[0]);
                if (SB) __builtin_amdgcn_sched_barrier(0);
                load32<2, NT>(a, in[0], h, f2(), b2(), d);
                math32<2>(a, d, acc[0]);
                if (SB) __builtin_amdgcn_sched_barrier(0);
                load32<3, NT>(a, in[0], h, f3(), b3(), d);
                math32<3>(a, d, acc[0]);
            }
        } else {
            hop_dir<D0, NT>(a, in, live, acc, h, fn(I0{}), bn(I0{}));
            if (SB) __builtin_amdgcn_sched_barrier(0);
            hop_dir<D1, NT>(a, in, live, acc, h, fn(I1{}), bn(I1{}));
            if (SB) __builtin_amdgcn_sched_barrier(0);
            hop_dir<D2, NT>(a, in, live, acc, h, fn(I2{}), bn(I2{}));
            if (SB) __builtin_amdgcn_sched_barrier(0);
            hop_dir<D3, NT>(a, in, live, acc, h, fn(I3{}), bn(I3{}));
        }

        if constexpr (ND) {
            if (live[0]) nd_mix(a, acc[0], rhs[0], h);
        }
#pragma unroll
        for (int gi = 0; gi < G; gi++) {
            if (!live[gi]) continue;
            nrm[gi] = pre ? hop_epilogue<SP, LK, SELF, NORM, EP, ND, true, true>(a, acc[gi], rhs[gi], h)
                          : hop_epilogue<SP, LK, SELF, NORM, EP, ND, true, false>(a, acc[gi], rhs[gi], h);
        }
    }
    if (NORM) {
        // (doublets: the block's lanes hold both flavours, so the sum is over the doublet)
        __shared__ double sh[G][HOP_BLOCK / 64];
#pragma unroll
        for (int gi = 0; gi < G; gi++) {
            if (!live[gi]) continue;
            const double s = block_sum(nrm[gi], sh[gi]);
            if (threadIdx.x == 0) a.partial[(ND ? rhs[gi] >> 1 : rhs[gi]) * a.pstride + pidx] = s;
        }
    }
}

// ---------------------------------------------------------- 16-bit kernel
//
// 16-bit spinors with FP16 two-row links, one right-hand side (or one
// doublet) per lane, for single fields and batches (BATCH): the arithmetic of
// hop_kernel's 16-bit paths (the same functions, the directions in the order
// of k1_order, so the results are identical bit for bit), with
//   * every offset 32-bit from a base that is uniform over the launch (the
//     field of the right-hand side, the link arrays of a parity), so that a
//     load is one instruction with a scalar base and the component blocks of
//     a site are immediate offsets: no 64-bit address arithmetic per hop;
//   * the boundary phases known at compile time (PM: bit mu set when direction
//     mu carries a phase; the launch's phase mask must equal it), so the
//     accumulation has no branches.
// Used when every byte offset fits 32 bits (V/2 < 2^26) and PM is 0 or 1 (no
// phase, or a phase in time only, as for antiperiodic fermions).

// byte offsets: 16-bit codes (3 blocks of 16 B per site, 8-site chunks), the
// 16-byte link block of direction 0 (4 per site), the 8-byte link block of
// direction 0 (16-site chunks); direction mu adds mu * 128 to both link offsets
__device__ __forceinline__ uint32_t off_codes(uint32_t h) { return ((h >> 3) * 384u) | ((h & 7u) << 4); }
__device__ __forceinline__ uint32_t off_link16a(uint32_t h) { return ((h >> 3) << 9) | ((h & 7u) << 4); }
__device__ __forceinline__ uint32_t off_link16b(uint32_t h) { return ((h >> 4) << 9) | ((h & 15u) << 3); }

// an ordering point: the values of s are final here, and no memory access
// moves across it (emits no instruction)
__device__ __forceinline__ void pin_order(spinor<float> &s)
{
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int c = 0; c < 3; c++) asm volatile("" : "+v"(s.c[i][c].re), "+v"(s.c[i][c].im)::"memory");
}

template <bool NT>
__device__ __forceinline__ uint4 ld_u4(const char *p)
{
    return ld<NT>((const uint4 *)p);
}
template <bool NT>
__device__ __forceinline__ uint2 ld_u2(const char *p)
{
    return ld<NT>((const uint2 *)p);
}

// uniform bases of a launch
struct Bases16 {
    const char *codes, *scale;   // input field (parity out_par ^ 1)
    const char *fa, *fb;         // links of the output parity (forward hops)
    const char *ba, *bb;         // links of the input parity (backward hops)
};

// the loads of direction MU (both hops) into d: the link of site h (its
// offsets oa, ob precomputed), the neighbour hf, the link of hb and the
// neighbour hb
template <int MU, bool NT>
__device__ __forceinline__ void load16o(const Bases16 &B, uint32_t oa, uint32_t ob, uint32_t hf, uint32_t hb, Raw16 &d)
{
    {
        const uint4 va = ld_u4<NT>(B.fa + oa + MU * 128);
        const uint2 vb = ld_u2<NT>(B.fb + ob + MU * 128);
        d.lw[0][0] = va.x, d.lw[0][1] = va.y, d.lw[0][2] = va.z, d.lw[0][3] = va.w, d.lw[0][4] = vb.x, d.lw[0][5] = vb.y;
    }
    {
        const char *q = B.codes + off_codes(hf);
        d.sc[0] = *(const float *)(B.scale + (hf << 2));
#pragma unroll
        for (int k = 0; k < 3; k++) {
            const uint4 v = *(const uint4 *)(q + k * 128);
            d.c[0][4 * k] = v.x, d.c[0][4 * k + 1] = v.y, d.c[0][4 * k + 2] = v.z, d.c[0][4 * k + 3] = v.w;
        }
    }
    {
        const uint4 va = ld_u4<NT>(B.ba + off_link16a(hb) + MU * 128);
        const uint2 vb = ld_u2<NT>(B.bb + off_link16b(hb) + MU * 128);
        d.lw[1][0] = va.x, d.lw[1][1] = va.y, d.lw[1][2] = va.z, d.lw[1][3] = va.w, d.lw[1][4] = vb.x, d.lw[1][5] = vb.y;
    }
    {
        const char *q = B.codes + off_codes(hb);
        d.sc[1] = *(const float *)(B.scale + (hb << 2));
#pragma unroll
        for (int k = 0; k < 3; k++) {
            const uint4 v = *(const uint4 *)(q + k * 128);
            d.c[1][4 * k] = v.x, d.c[1][4 * k + 1] = v.y, d.c[1][4 * k + 2] = v.z, d.c[1][4 * k + 3] = v.w;
        }
    }
}
// math16 with the phase of direction MU fixed at compile time
template <int MU, bool PH, class SP, class LK, typename R>
__device__ __forceinline__ void math16p(const HopArgs<SP, LK> &a, const Raw16 &d, spinor<R> &acc)
{
#pragma unroll
    for (int dir = 0; dir < 2; dir++) {
        typename LK::Loaded u;
#pragma unroll
        for (int k = 0; k < 6; k++) u.w[k] = d.lw[dir][k];
        a.lk.rebuild(u);
        if (dir == 0)
            coded_hop_ph<MU, 0, PH>(a, u, d.c[0], d.sc[0], acc);
        else
            coded_hop_ph<MU, 1, PH>(a, u, d.c[1], d.sc[1], acc);
    }
}

// the loads of one hop (DIR 0 forward: the link of the output site; DIR 1
// backward: the link of the neighbour) and of its neighbour spinor
struct Hop16 {
    uint32_t lw[6];
    uint32_t c[12];
    float sc;
};
template <int MU, int DIR, bool NT>
__device__ __forceinline__ void load16h(const Bases16 &B, uint32_t oa, uint32_t ob, uint32_t hn, Hop16 &d)
{
    const uint4 va = DIR == 0 ? ld_u4<NT>(B.fa + oa + MU * 128) : ld_u4<NT>(B.ba + off_link16a(hn) + MU * 128);
    const uint2 vb = DIR == 0 ? ld_u2<NT>(B.fb + ob + MU * 128) : ld_u2<NT>(B.bb + off_link16b(hn) + MU * 128);
    d.lw[0] = va.x, d.lw[1] = va.y, d.lw[2] = va.z, d.lw[3] = va.w, d.lw[4] = vb.x, d.lw[5] = vb.y;
    const char *q = B.codes + off_codes(hn);
    d.sc = *(const float *)(B.scale + (hn << 2));
#pragma unroll
    for (int k = 0; k < 3; k++) {
        const uint4 v = *(const uint4 *)(q + k * 128);
        d.c[4 * k] = v.x, d.c[4 * k + 1] = v.y, d.c[4 * k + 2] = v.z, d.c[4 * k + 3] = v.w;
    }
}
template <int MU, int DIR, bool PH, class SP, class LK, typename R>
__device__ __forceinline__ void math16h(const HopArgs<SP, LK> &a, const Hop16 &d, spinor<R> &acc)
{
    typename LK::Loaded u;
#pragma unroll
    for (int k = 0; k < 6; k++) u.w[k] = d.lw[k];
    a.lk.rebuild(u);
    coded_hop_ph<MU, DIR, PH>(a, u, d.c, d.sc, acc);
}

// The loads of one hop of a doublet site for both flavours: the link once and
// the neighbour codes and scales of each flavour (codes and scales of the
// lower flavour from its own bases)
struct Hop16N {
    uint32_t lw[6];
    uint32_t c[2][12];
    float sc[2];
};
template <int MU, int DIR, bool NT>
__device__ __forceinline__ void load16n(const Bases16 &B, const char *codes_d, const char *scale_d, uint32_t oa,
                                        uint32_t ob, uint32_t hn, Hop16N &d)
{
    const uint4 va = DIR == 0 ? ld_u4<NT>(B.fa + oa + MU * 128) : ld_u4<NT>(B.ba + off_link16a(hn) + MU * 128);
    const uint2 vb = DIR == 0 ? ld_u2<NT>(B.fb + ob + MU * 128) : ld_u2<NT>(B.bb + off_link16b(hn) + MU * 128);
    d.lw[0] = va.x, d.lw[1] = va.y, d.lw[2] = va.z, d.lw[3] = va.w, d.lw[4] = vb.x, d.lw[5] = vb.y;
#pragma unroll
    for (int f = 0; f < 2; f++) {
        const char *q = (f == 0 ? B.codes : codes_d) + off_codes(hn);
        d.sc[f] = *(const float *)((f == 0 ? B.scale : scale_d) + (hn << 2));
#pragma unroll
        for (int k = 0; k < 3; k++) {
            const uint4 v = *(const uint4 *)(q + k * 128);
            d.c[f][4 * k] = v.x, d.c[f][4 * k + 1] = v.y, d.c[f][4 * k + 2] = v.z, d.c[f][4 * k + 3] = v.w;
        }
    }
}
// the hop for both flavours: row 2 of the link formed once, then each
// flavour's projection, product and accumulation as for one flavour
template <int MU, int DIR, bool PH, class SP, class LK, typename R>
__device__ __forceinline__ void math16n(const HopArgs<SP, LK> &a, const Hop16N &d, spinor<R> &au, spinor<R> &ad)
{
    typename LK::Loaded u;
#pragma unroll
    for (int k = 0; k < 6; k++) u.w[k] = d.lw[k];
    a.lk.rebuild(u);
    coded_hop_ph<MU, DIR, PH>(a, u, d.c[0], d.sc[0], au);
    coded_hop_ph<MU, DIR, PH>(a, u, d.c[1], d.sc[1], ad);
}

// nd_mix for both flavours of a site held by one lane (au upper, ad lower
// flavour of doublet rhs_u >> 1): the same operations, the partner's values
// taken from the other accumulator instead of the other lane (TAB: the
// coefficients from the launch's table, as in hop_epilogue)
template <bool TAB, class SP, class LK, typename R>
__device__ __forceinline__ void nd_mix2(const HopArgs<SP, LK> &a, spinor<R> &au, spinor<R> &ad, int rhs_u, int rhs_d,
                                        long h)
{
    const int d = rhs_u >> 1;
    const double kap = a.op.kappa[d], md = a.sign * a.op.mut[d], ed = a.op.eps[d];
    R m, e;
    if constexpr (TAB) {
        m = a.ec[d].m;
        e = a.ec[d].e;
    } else {
        m = (R)md;
        e = (R)ed;
    }
    if (a.epi == EPI_K1) {
        cx<R> pm, pp;  // c (1 - i m), c (1 + i m)
        R ce;
        if constexpr (TAB) {
            const EpiCoef &k = a.ec[d];
            pm = {k.c, -k.cm};
            pp = {k.c, k.cm};
            ce = -k.ce;
        } else {
            const double c = kap * kap / (1.0 + md * md - ed * ed);
            pm = {(R)c, (R)(-c * md)};
            pp = {(R)c, (R)(c * md)};
            ce = (R)(-c * ed);
        }
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int c3 = 0; c3 < 3; c3++) {
                const cx<R> ou = au.c[i][c3], od = ad.c[i][c3];
                // c (1 -+ i m g5) own - c e other (upper / lower flavour)
                au.c[i][c3] = fma(i < 2 ? pm : pp, ou, ce * od);
                ad.c[i][c3] = fma(i < 2 ? pp : pm, od, ce * ou);
            }
    } else {
        spinor<R> su, sd;
        a.self.at(rhs_u).load(h, su);
        a.self.at(rhs_d).load(h, sd);
        const cx<R> one_pm = {R(1), (R)m}, one_mm = {R(1), (R)(-m)};  // 1 + i m, 1 - i m
        const R ee = (R)e;
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int c3 = 0; c3 < 3; c3++) {
                // A self = (1 +- i m g5) own + e other
                const cx<R> asu = fma(i < 2 ? one_pm : one_mm, su.c[i][c3], ee * sd.c[i][c3]);
                const cx<R> asd = fma(i < 2 ? one_mm : one_pm, sd.c[i][c3], ee * su.c[i][c3]);
                const cx<R> ou = asu - au.c[i][c3], od = asd - ad.c[i][c3];
                au.c[i][c3] = i < 2 ? ou : -ou;
                ad.c[i][c3] = i < 2 ? od : -od;
            }
    }
}

// K2F: a K2 store launch (a.epi == EPI_K2), which starts from the own-site term.
// BATCH: the launch covers several tuples (right-hand sides, or doublets), one
// per block, in the RHS groups of hop_kernel, with the link loads cached (the
// blocks of a group read the same links); otherwise one tuple, links streamed.
// ND: doublets, both flavours of a site in one lane (tuple = RHS pair 2d, 2d + 1).
// TWO (batches): two right-hand sides per lane (tuple = RHS 2i, 2i + 1 of the
// list), sharing the link loads and row 2 as the flavours of a doublet do.
template <class SP, bool SELF, bool NORM, int ORD, bool SB, int EP, bool ND, int PM, bool K2F = false,
          bool BATCH = false, bool TWO = false>
__global__ __launch_bounds__(HOP_BLOCK) void hop16_kernel(HopArgs<SP, L16R> a)
{
    static_assert(!TWO || (BATCH && !ND), "two right-hand sides per lane are a batched single-flavour launch");
    constexpr bool DUAL = ND || TWO;  // two accumulators per lane
    using LK = L16R;
    using R = float;
    constexpr bool LNT = !BATCH;                                           // links non-temporal
    constexpr int SPB = HOP_BLOCK;    // sites per block
    const uint32_t ls = threadIdx.x;  // site of the lane in the block
    const Geom &g = a.g;
    const int j = blockIdx.x & 7;
    uint32_t sb;  // site block within the XCD's share
    int tup;      // tuple of the block
    if constexpr (BATCH) {
        // (the divisions by launch constants through the host's multipliers, a.dv)
        const uint32_t k = blockIdx.x >> 3;
        const int nb = a.nblk >> 3;
        const int ntup = ND ? a.rl.n / 2 : TWO ? (a.rl.n + 1) / 2 : a.rl.n;
        const int GR = a.group;
        const int gr = (int)fdiv(k, a.dv.grp);      // k / (nb GR)
        const int gsize = min(GR, ntup - gr * GR);  // the last group may be smaller
        const uint32_t within = k - (uint32_t)(gr * nb * GR);
        sb = fdiv(within, gsize == GR ? a.dv.gsz : a.dv.glast);  // within / gsize
        tup = gr * GR + (int)(within - sb * (uint32_t)gsize);
    } else {
        sb = blockIdx.x >> 3;
        tup = 0;
    }
    int rhs, rhs_d;    // the tuple's right-hand sides (doublets: upper, lower flavour)
    bool two = DUAL;  // (TWO: whether the second one is live)
    if constexpr (TWO) {
        // a finished or missing second RHS leaves the lane with the first; a
        // finished first one hands its place to the second
        int r0 = a.rl.idx[2 * tup];
        const int r1 = 2 * tup + 1 < a.rl.n ? a.rl.idx[2 * tup + 1] : -1;
        bool l0 = !(a.scal && a.scal[r0].done), l1 = r1 >= 0 && !(a.scal && a.scal[r1].done);
        if (!l0 && !l1) return;
        if (!l0) {
            r0 = r1;
            l1 = false;
        }
        rhs = r0;
        rhs_d = l1 ? r1 : r0;
        two = l1;
    } else {
        rhs = a.rl.idx[ND ? 2 * tup : tup];
        rhs_d = ND ? a.rl.idx[2 * tup + 1] : rhs;
        if (a.scal && a.scal[ND ? rhs >> 1 : rhs].done) return;
    }
    const uint32_t XH = (uint32_t)g.XH, LY = (uint32_t)g.LY, LZ = (uint32_t)g.LZ, T = (uint32_t)g.T;
    const uint32_t plane = LY * XH;  // sites of one (t, z) plane
    uint32_t h, t, z, y, xh, pidx;
    bool active;
    if (ORD == ORD_ZSLAB) {
        const uint32_t zb = LZ >> 3, zr = LZ & 7;
        const uint32_t zc = zb + ((uint32_t)j < zr ? 1 : 0), z0 = j * zb + ((uint32_t)j < zr ? j : zr);
        const uint32_t S = zc * plane;  // sites of one time-slice of this slab
        const uint32_t l = sb * SPB + ls;
        active = l < T * S;
        const uint32_t lu = active ? l : 0u;
        t = BATCH ? fdiv(lu, a.dv.slab[(uint32_t)j < zr ? 1 : 0]) : lu / S;
        const uint32_t rem = lu - t * S;
        z = z0 + (BATCH ? fdiv(rem, a.dv.plane) : rem / plane);
        const uint32_t r2 = rem - (z - z0) * plane;
        y = BATCH ? fdiv(r2, a.dv.xh) : r2 / XH;
        xh = r2 - y * XH;
        h = ((t * LZ + z) * LY + y) * XH + xh;
        pidx = 8 * sb + j;
    } else if (ORD == ORD_TSLAB) {
        const uint32_t tb = T >> 3, tr = T & 7;
        const uint32_t tc = tb + ((uint32_t)j < tr ? 1 : 0), t0 = j * tb + ((uint32_t)j < tr ? j : tr);
        const uint32_t P = tc * plane;  // sites of one z-plane of this block of time-slices
        const uint32_t l = sb * SPB + ls;
        active = l < LZ * P;
        const uint32_t lu = active ? l : 0u;
        z = BATCH ? fdiv(lu, a.dv.slab[(uint32_t)j < tr ? 1 : 0]) : lu / P;
        const uint32_t rem = lu - z * P;
        t = t0 + (BATCH ? fdiv(rem, a.dv.plane) : rem / plane);
        const uint32_t r2 = rem - (t - t0) * plane;
        y = BATCH ? fdiv(r2, a.dv.xh) : r2 / XH;
        xh = r2 - y * XH;
        h = ((t * LZ + z) * LY + y) * XH + xh;
        pidx = 8 * sb + j;
    } else {
        const uint32_t lb = j * ((uint32_t)a.nblk >> 3) + sb;
        h = lb * SPB + ls;
        active = h < (uint32_t)g.vh;
        const uint32_t hu = active ? h : 0u;
        if constexpr (BATCH) {
            const uint32_t r = fdiv(hu, a.dv.xh), r1 = fdiv(r, a.dv.ly);
            xh = hu - r * XH;
            y = r - r1 * LY;
            t = fdiv(r1, a.dv.lz);
            z = r1 - t * LZ;
        } else {
            xh = hu % XH;
            uint32_t r = hu / XH;
            y = r % LY;
            r /= LY;
            z = r % LZ;
            t = r / LZ;
        }
        pidx = lb;
    }
    double nrm = 0.0, nrm2 = 0.0;
    if (active) {
        const int ip = a.out_par ^ 1;
        const SP in = a.in.at(rhs);
        const uint32_t vh = (uint32_t)g.vh, vh16q = (uint32_t)vh16(g.vh);
        Bases16 B;
        B.codes = (const char *)in.p;
        B.scale = (const char *)in.scale;
        B.fa = (const char *)(a.lk.a + (uint32_t)a.out_par * 4u * vh);
        B.fb = (const char *)(a.lk.b + (uint32_t)a.out_par * 4u * vh16q);
        B.ba = (const char *)(a.lk.a + (uint32_t)ip * 4u * vh);
        B.bb = (const char *)(a.lk.b + (uint32_t)ip * 4u * vh16q);
        const uint32_t x = 2 * xh + ((a.out_par + t + z + y) & 1);
        const uint32_t row = h - xh;
        const uint32_t sy = XH, sz = plane, stt = LZ * plane;
        const uint32_t LX = (uint32_t)g.LX;
        spinor<R> acc, acd;  // (acd: a doublet's lower flavour, or the second right-hand side)
        if constexpr (K2F) {
            // the operations of k2_self_first, written out: through the
            // helper the compiler keeps about 30 more registers live here
#pragma unroll
            for (int q = 0; q < (TWO ? 2 : 1); q++) {
                const int r = q == 0 ? rhs : rhs_d;
                spinor<R> sf;
                a.self.at(r).load((long)h, sf);
                R m;
                if constexpr (BATCH)
                    m = a.ec[r].m;
                else
                    m = (R)(a.sign * a.op.mut[r]);
                const cx<R> Au = cx<R>{R(1), m}, Ad = cx<R>{R(-1), m};
                spinor<R> &dst = q == 0 ? acc : acd;
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    dst.c[0][c] = -(Au * sf.c[0][c]);
                    dst.c[1][c] = -(Au * sf.c[1][c]);
                    dst.c[2][c] = Ad * sf.c[2][c];
                    dst.c[3][c] = Ad * sf.c[3][c];
                }
            }
        } else {
#pragma unroll
            for (int i = 0; i < 4; i++)
#pragma unroll
                for (int c = 0; c < 3; c++) acc.c[i][c] = acd.c[i][c] = cx<R>{R(0), R(0)};
        }
        const uint32_t oa = off_link16a(h), ob = off_link16b(h);
        // neighbours (periodic), with the wrap as a select of uniform values
        // (no branches): h +- stride -+ (extent * stride at the boundary)
        const uint32_t tf = h + stt - (t + 1 == T ? T * stt : 0u), tb = h - stt + (t == 0 ? T * stt : 0u);
        const uint32_t xf = row + ((x + 1 == LX ? 0u : x + 1) >> 1), xb = row + ((x == 0 ? LX - 1 : x - 1) >> 1);
        const uint32_t yf = h + sy - (y + 1 == LY ? LY * sy : 0u), yb = h - sy + (y == 0 ? LY * sy : 0u);
        const uint32_t zf = h + sz - (z + 1 == LZ ? LZ * sz : 0u), zb = h - sz + (z == 0 ? LZ * sz : 0u);
        // the directions in the order of the sum (k1_order), neighbours by index
        constexpr int D0 = k1_order<!SELF>(0), D1 = k1_order<!SELF>(1), D2 = k1_order<!SELF>(2),
                      D3 = k1_order<!SELF>(3);
        const uint32_t nf[4] = {tf, xf, yf, zf}, nbk[4] = {tb, xb, yb, zb};
        if constexpr (DUAL) {
            // doublets (VALU-bound), or two right-hand sides: both fields of the
            // site in this lane, so the link is loaded and its row 2 formed once
            // for the two; one hop at a time with the next one in flight (about
            // 155 registers, 3 waves per SIMD).  A doublet K1 executes 2557 VALU
            // instructions per site this way, 3098 with a lane per flavour.
            // (TWO with one live RHS repeats it in the second accumulator, which
            // is not stored.)
            const SP ind = a.in.at(rhs_d);
            const char *cd = (const char *)ind.p, *sd = (const char *)ind.scale;
            Hop16N b0, b1;
            load16n<D0, 0, LNT>(B, cd, sd, oa, ob, nf[D0], b0);
            load16n<D0, 1, LNT>(B, cd, sd, oa, ob, nbk[D0], b1);
            __builtin_amdgcn_sched_barrier(0);
            math16n<D0, 0, ((PM >> D0) & 1) != 0>(a, b0, acc, acd);
            pin_order(acc);
            pin_order(acd);
            load16n<D1, 0, LNT>(B, cd, sd, oa, ob, nf[D1], b0);
            __builtin_amdgcn_sched_barrier(0);
            math16n<D0, 1, ((PM >> D0) & 1) != 0>(a, b1, acc, acd);
            pin_order(acc);
            pin_order(acd);
            load16n<D1, 1, LNT>(B, cd, sd, oa, ob, nbk[D1], b1);
            __builtin_amdgcn_sched_barrier(0);
            math16n<D1, 0, ((PM >> D1) & 1) != 0>(a, b0, acc, acd);
            pin_order(acc);
            pin_order(acd);
            load16n<D2, 0, LNT>(B, cd, sd, oa, ob, nf[D2], b0);
            __builtin_amdgcn_sched_barrier(0);
            math16n<D1, 1, ((PM >> D1) & 1) != 0>(a, b1, acc, acd);
            pin_order(acc);
            pin_order(acd);
            load16n<D2, 1, LNT>(B, cd, sd, oa, ob, nbk[D2], b1);
            __builtin_amdgcn_sched_barrier(0);
            math16n<D2, 0, ((PM >> D2) & 1) != 0>(a, b0, acc, acd);
            pin_order(acc);
            pin_order(acd);
            load16n<D3, 0, LNT>(B, cd, sd, oa, ob, nf[D3], b0);
            __builtin_amdgcn_sched_barrier(0);
            math16n<D2, 1, ((PM >> D2) & 1) != 0>(a, b1, acc, acd);
            pin_order(acc);
            pin_order(acd);
            load16n<D3, 1, LNT>(B, cd, sd, oa, ob, nbk[D3], b1);
            __builtin_amdgcn_sched_barrier(0);
            math16n<D3, 0, ((PM >> D3) & 1) != 0>(a, b0, acc, acd);
            math16n<D3, 1, ((PM >> D3) & 1) != 0>(a, b1, acc, acd);
        } else {
            // one flavour: two directions (four hops) loaded at a time, in the
            // order of the sum
            Raw16 d0, d1;
            load16o<D0, LNT>(B, oa, ob, nf[D0], nbk[D0], d0);
            load16o<D1, LNT>(B, oa, ob, nf[D1], nbk[D1], d1);
            __builtin_amdgcn_sched_barrier(0);  // every load of the group issued before its arithmetic
            math16p<D0, ((PM >> D0) & 1) != 0>(a, d0, acc);
            math16p<D1, ((PM >> D1) & 1) != 0>(a, d1, acc);
            // the loads of the other two directions after this arithmetic: two
            // directions in flight keep the lane within 128 registers (all four at
            // once need about 200, half the waves per SIMD).  The empty asm takes
            // the accumulators as operands, so the arithmetic above completes
            // before it, and clobbers memory, so the loads below stay after it.
            pin_order(acc);
            if (SB) __builtin_amdgcn_sched_barrier(0);
            load16o<D2, LNT>(B, oa, ob, nf[D2], nbk[D2], d0);
            load16o<D3, LNT>(B, oa, ob, nf[D3], nbk[D3], d1);
            __builtin_amdgcn_sched_barrier(0);
            math16p<D2, ((PM >> D2) & 1) != 0>(a, d0, acc);
            math16p<D3, ((PM >> D3) & 1) != 0>(a, d1, acc);
        }
        // one tuple: the output is stored through the caches, since the next
        // half-sweep reads it (measured 2 % faster than non-temporal stores for
        // both K1 and K2); a batch's outputs are read again only after the
        // whole batch, so they are stored non-temporally
        if constexpr (ND) {
            nd_mix2<BATCH>(a, acc, acd, rhs, rhs_d, (long)h);
            nrm = hop_epilogue<SP, LK, SELF, NORM, EP, ND, BATCH, false, BATCH>(a, acc, rhs, (long)h);
            nrm += hop_epilogue<SP, LK, SELF, NORM, EP, ND, BATCH, false, BATCH>(a, acd, rhs_d, (long)h);
        } else if constexpr (TWO) {
            nrm = hop_epilogue<SP, LK, SELF, NORM, EP, ND, BATCH, K2F, BATCH>(a, acc, rhs, (long)h);
            if (two) nrm2 = hop_epilogue<SP, LK, SELF, NORM, EP, ND, BATCH, K2F, BATCH>(a, acd, rhs_d, (long)h);
        } else {
            nrm = hop_epilogue<SP, LK, SELF, NORM, EP, ND, BATCH, K2F, BATCH>(a, acc, rhs, (long)h);
        }
    }
    if (NORM) {
        // (doublets: each lane's value covers both flavours, so the sum is over the doublet)
        __shared__ double sh[HOP_BLOCK / 64];
        const double s = block_sum(nrm, sh);
        if (threadIdx.x == 0) a.partial[(ND ? rhs >> 1 : rhs) * a.pstride + pidx] = s;
        if (TWO && two) {  // (uniform over the block)
            __shared__ double sh2[HOP_BLOCK / 64];
            const double s2 = block_sum(nrm2, sh2);
            if (threadIdx.x == 0) a.partial[rhs_d * a.pstride + pidx] = s2;
        }
    }
}

// launches of hop16_kernel: the block order of the variant, the epilogue
// flavours of go_w / go_nd, the compile-time phase mask, and single-tuple or
// batched (BATCH) launches
template <class SP, int ORD, bool SB, bool ND, int PM, bool BATCH, bool TWO = false>
void go16_e(const HopArgs<SP, L16R> &a, bool s, bool n, int ep, dim3 grid, dim3 block, unsigned lds, hipStream_t st)
{
    if (ep == EP_CG)
        hipLaunchKernelGGL((hop16_kernel<SP, true, true, ORD, SB, EP_CG, ND, PM, false, BATCH, TWO>), grid, block, lds, st,
                           a);
    else if (ep == EP_RES)
        hipLaunchKernelGGL((hop16_kernel<SP, true, true, ORD, SB, EP_RES, ND, PM, false, BATCH, TWO>), grid, block, lds,
                           st, a);
    else if (s && !ND && a.epi == EPI_K2) {
        if (n)
            hipLaunchKernelGGL((hop16_kernel<SP, true, true, ORD, SB, EP_STORE, ND, PM, true, BATCH, TWO>), grid, block,
                               lds, st, a);
        else
            hipLaunchKernelGGL((hop16_kernel<SP, true, false, ORD, SB, EP_STORE, ND, PM, true, BATCH, TWO>), grid, block,
                               lds, st, a);
    } else if (s && n)
        hipLaunchKernelGGL((hop16_kernel<SP, true, true, ORD, SB, EP_STORE, ND, PM, false, BATCH, TWO>), grid, block, lds,
                           st, a);
    else if (s)
        hipLaunchKernelGGL((hop16_kernel<SP, true, false, ORD, SB, EP_STORE, ND, PM, false, BATCH, TWO>), grid, block, lds,
                           st, a);
    else if (n && !ND)
        hipLaunchKernelGGL((hop16_kernel<SP, false, true, ORD, SB, EP_STORE, ND, PM, false, BATCH, TWO>), grid, block, lds,
                           st, a);
    else
        hipLaunchKernelGGL((hop16_kernel<SP, false, false, ORD, SB, EP_STORE, ND, PM, false, BATCH, TWO>), grid, block,
                           lds, st, a);
}
template <class SP, bool ND, int PM, bool BATCH, bool TWO = false>
void go16_v(const HopArgs<SP, L16R> &a, int variant, bool s, bool n, int ep, dim3 grid, dim3 block, unsigned lds,
            hipStream_t st)
{
    switch (variant) {
    case 1: go16_e<SP, ORD_ZSLAB, false, ND, PM, BATCH, TWO>(a, s, n, ep, grid, block, lds, st); break;
    case 2: go16_e<SP, ORD_ZSLAB, true, ND, PM, BATCH, TWO>(a, s, n, ep, grid, block, lds, st); break;
    case 3: go16_e<SP, ORD_TSLAB, false, ND, PM, BATCH, TWO>(a, s, n, ep, grid, block, lds, st); break;
    case 4: go16_e<SP, ORD_TSLAB, true, ND, PM, BATCH, TWO>(a, s, n, ep, grid, block, lds, st); break;
    default: go16_e<SP, ORD_PLAIN, false, ND, PM, BATCH, TWO>(a, s, n, ep, grid, block, lds, st); break;
    }
}

// the launches of hop16_kernel, instantiated in hop16_f16.hip / hop16_b16.hip
// (own translation units, compiled in parallel with the others); batch: more
// than one tuple (right-hand side or doublet) in the launch; two: batched, two
// right-hand sides per lane
void launch_hop16(const HopArgs<SpH16, L16R> &a, bool nd, bool batch, bool two, int variant, bool s, bool n, int ep,
                  dim3 grid, dim3 block, unsigned lds, hipStream_t st);
void launch_hop16(const HopArgs<SpB16, L16R> &a, bool nd, bool batch, bool two, int variant, bool s, bool n, int ep,
                  dim3 grid, dim3 block, unsigned lds, hipStream_t st);
template <class SP>
void launch_hop16_impl(const HopArgs<SP, L16R> &a, bool nd, bool batch, bool two, int variant, bool s, bool n,
                       int ep, dim3 grid, dim3 block, unsigned lds, hipStream_t st)
{
    if (two) {
        if (a.phase_mask)
            go16_v<SP, false, 1, true, true>(a, variant, s, n, ep, grid, block, lds, st);
        else
            go16_v<SP, false, 0, true, true>(a, variant, s, n, ep, grid, block, lds, st);
    } else if (nd && batch) {
        if (a.phase_mask)
            go16_v<SP, true, 1, true>(a, variant, s, n, ep, grid, block, lds, st);
        else
            go16_v<SP, true, 0, true>(a, variant, s, n, ep, grid, block, lds, st);
    } else if (nd) {
        if (a.phase_mask)
            go16_v<SP, true, 1, false>(a, variant, s, n, ep, grid, block, lds, st);
        else
            go16_v<SP, true, 0, false>(a, variant, s, n, ep, grid, block, lds, st);
    } else if (batch) {
        if (a.phase_mask)
            go16_v<SP, false, 1, true>(a, variant, s, n, ep, grid, block, lds, st);
        else
            go16_v<SP, false, 0, true>(a, variant, s, n, ep, grid, block, lds, st);
    } else {
        if (a.phase_mask)
            go16_v<SP, false, 1, false>(a, variant, s, n, ep, grid, block, lds, st);
        else
            go16_v<SP, false, 0, false>(a, variant, s, n, ep, grid, block, lds, st);
    }
}

// ------------------------------------------------------------- dispatch

// doublet launches: a lane pair per site, K1 (no self, no norm), K2 with
// or without the norm, and the fused CG and residual epilogues
template <class SP, class LK, bool NT, int ORD>
void go_nd(const HopArgs<SP, LK> &a, bool s, bool n, int ep, dim3 grid, dim3 block, unsigned lds, hipStream_t st)
{
    if (ep == EP_CG)
        hipLaunchKernelGGL((hop_kernel<SP, LK, true, true, NT, ORD, false, 1, EP_CG, true>), grid, block, lds, st, a);
    else if (ep == EP_RES)
        hipLaunchKernelGGL((hop_kernel<SP, LK, true, true, NT, ORD, false, 1, EP_RES, true>), grid, block, lds, st, a);
    else if (s && n)
        hipLaunchKernelGGL((hop_kernel<SP, LK, true, true, NT, ORD, false, 1, EP_STORE, true>), grid, block, lds, st,
                           a);
    else if (s)
        hipLaunchKernelGGL((hop_kernel<SP, LK, true, false, NT, ORD, false, 1, EP_STORE, true>), grid, block, lds, st,
                           a);
    else
        hipLaunchKernelGGL((hop_kernel<SP, LK, false, false, NT, ORD, false, 1, EP_STORE, true>), grid, block, lds,
                           st, a);
}

template <class SP, class LK, bool NT, int ORD, bool SB, int G>
void go_w(const HopArgs<SP, LK> &a, bool s, bool n, int ep, dim3 grid, dim3 block, unsigned lds, hipStream_t st)
{
    if (ep == EP_CG)
        hipLaunchKernelGGL((hop_kernel<SP, LK, true, true, NT, ORD, SB, G, EP_CG>), grid, block, lds, st, a);
    else if (ep == EP_RES)
        hipLaunchKernelGGL((hop_kernel<SP, LK, true, true, NT, ORD, SB, G, EP_RES>), grid, block, lds, st, a);
    else if (s && n)
        hipLaunchKernelGGL((hop_kernel<SP, LK, true, true, NT, ORD, SB, G, EP_STORE>), grid, block, lds, st, a);
    else if (s)
        hipLaunchKernelGGL((hop_kernel<SP, LK, true, false, NT, ORD, SB, G, EP_STORE>), grid, block, lds, st, a);
    else if (n)
        hipLaunchKernelGGL((hop_kernel<SP, LK, false, true, NT, ORD, SB, G, EP_STORE>), grid, block, lds, st, a);
    else
        hipLaunchKernelGGL((hop_kernel<SP, LK, false, false, NT, ORD, SB, G, EP_STORE>), grid, block, lds, st, a);
}

// ALL = false: only variant 0 is instantiated (rarely used format pairs)
// RHS per group: three time-slices of an XCD's share of the sites (its slab,
// or 1/8 of a time-slice) for every RHS of the group within about 2 MB of L2
inline int rhs_group(const Geom &g, int prec, int n)
{
    const double sp = prec == P64 ? 192.0 : prec == P32 ? 96.0 : 52.0;
    const double slice = (double)((g.LZ + 7) / 8) * g.LY * g.XH * sp;
    int G = (int)(2.0e6 / (3.0 * slice));
    return G < 1 ? 1 : (G > n ? n : G);
}

// ALL = false: only variant 0 with one RHS per lane is instantiated (rarely
// used format pairs); MULTI = true adds 2 RHS per lane for batches (the
// FP32-arithmetic formats; FP64 lanes already use all 256 registers; 4 per
// lane measured slower than 1 and 2).
template <class SP, class LK, bool ALL, bool MULTI>
hipError_t go(const Geom &g, int out_par, const FieldDesc &in, const FieldDesc &self, const FieldDesc &out,
              const LinkDesc &lk, const OpParams &op, int epi, int sign, const RhsList &rl, double *partial,
              long pstride, const CgScalars *scal, const HopTune &tu, hipStream_t st, const CgFields *cg)
{
    if (rl.n <= 0) return hipSuccess;
    const int ep = epi == EPI_K2_CG ? EP_CG : epi == EPI_K2_RES ? EP_RES : EP_STORE;
    if (ep != EP_STORE) {
        // fused epilogues: the vectors must be given, in the right formats, the
        // norm asked for, and (for CG) the device scalars holding alpha
        if (!cg || !partial || (ep == EP_CG && !scal)) return hipErrorInvalidValue;
        if (cg->r.prec != in.prec || cg->p.prec != in.prec) return hipErrorInvalidValue;
        if (ep == EP_CG && cg->x.prec != (in.prec == P64 ? P64 : P32)) return hipErrorInvalidValue;
    }
    static_assert(sizeof(HopArgs<SP, LK>) <= 4096, "kernel arguments are limited to 4 KB");
    HopArgs<SP, LK> a;
    a.g = g;
    a.out_par = out_par;
    a.epi = epi;
    a.sign = sign;
    a.phase_mask = hop_phase_mask(op);
    a.in = make_bv<SP>(in);
    a.self = self.data ? make_bv<SP>(self) : a.in;
    a.out = make_bv<SP>(out);
    a.lk = make_lk<LK>(lk);
    a.op = op;
    a.rl = rl;
    a.partial = partial;
    a.pstride = pstride;
    a.scal = scal;
    a.one = 1.0f;
    if (ep != EP_STORE) {
        a.cg_r = make_bv<SP>(cg->r);
        a.cg_p = make_bv<SP>(cg->p);
        if (ep == EP_CG) a.cg_x = make_bv<typename XsOf<SP>::type>(cg->x);
    }
    if (ALL != hop_all_variants(in.prec, lk.fmt)) return hipErrorInvalidValue;  // tables out of step
    int variant = tu.variant;
    if (!ALL || !hop_variant_valid(g, variant)) variant = 0;
    // the divisors and site-term table of a batched 16-bit launch of ntup tuples
    auto batch16 = [&](int ntup) {
        if constexpr (SP::coded && __is_same(LK, L16R)) {
            a.dv = make_site_div(g, variant == 0 ? ORD_PLAIN : variant <= 2 ? ORD_ZSLAB : ORD_TSLAB, a.nblk, a.group,
                                 ntup);
            for (int i = 0; i < rl.n; i++) {
                const int r = op.nd ? rl.idx[i] >> 1 : rl.idx[i];
                if (r >= MAX_RHS) return false;
                const double kap = op.kappa[r], m = sign * op.mut[r], e = op.nd ? op.eps[r] : 0.0;
                const double c = op.nd ? kap * kap / (1.0 + m * m - e * e) : kap * kap / (1.0 + m * m);
                a.ec[r] = EpiCoef{(float)c, (float)(c * m), (float)(c * e), (float)m, (float)e};
            }
        }
        return true;
    };
    if (op.nd) {
        // doublets: the two flavours of a site in a lane pair (RHS pairs 2d, 2d + 1 of rl)
        if (rl.n % 2) return hipErrorInvalidValue;
        for (int i = 0; i < rl.n; i += 2)
            if (rl.idx[i] % 2 || rl.idx[i + 1] != rl.idx[i] + 1) return hipErrorInvalidValue;
        if (epi != EPI_K1 && epi != EPI_K2 && ep == EP_STORE) return hipErrorInvalidValue;
        const bool s = epi != EPI_K1, n = partial != nullptr;
        if (s && !self.data) return hipErrorInvalidValue;
        if (!s && n) return hipErrorInvalidValue;
        const int lanes = hop_nd_lanes(g, in.prec, lk.fmt, op);  // per doublet site
        a.nblk = hop_grid_variant(g, variant, lanes);
        const int ntup = rl.n / 2;
        const int grp = tu.group > 0 ? tu.group : rhs_group(g, in.prec, rl.n);
        a.group = (grp + 1) / 2;
        if (a.group > ntup) a.group = ntup;
        if (ntup > 1 && !batch16(ntup)) return hipErrorInvalidValue;
        a.epi = ep == EP_STORE ? epi : EPI_K2;
        const dim3 grid(a.nblk * ntup), block(HOP_BLOCK);
        const int ord = variant == 0 ? ORD_PLAIN : variant <= 2 ? ORD_ZSLAB : ORD_TSLAB;
        const bool nt = ntup == 1;
        if constexpr (ALL && SP::coded && __is_same(LK, L16R)) {
            if (lanes == 1) {
                // the 16-bit kernel: both flavours of a site in one lane
                launch_hop16(a, true, !nt, false, variant, s, n, ep, grid, block, tu.lds, st);
                return hipGetLastError();
            }
        }
#define GON(ORD)                                                                \
    do {                                                                        \
        if (nt)                                                                 \
            go_nd<SP, LK, true, ORD>(a, s, n, ep, grid, block, tu.lds, st);     \
        else                                                                    \
            go_nd<SP, LK, false, ORD>(a, s, n, ep, grid, block, tu.lds, st);    \
    } while (0)
        if constexpr (ALL) {
            if (ord == ORD_ZSLAB)
                GON(ORD_ZSLAB);
            else if (ord == ORD_TSLAB)
                GON(ORD_TSLAB);
            else
                GON(ORD_PLAIN);
        } else {
            GON(ORD_PLAIN);
        }
#undef GON
        return hipGetLastError();
    }
    int G = MULTI && ALL && rl.n > 1 ? tu.rpl : 1;
    if (G != 2) G = 1;
    const int ntup = (rl.n + G - 1) / G;
    a.nblk = hop_grid_variant(g, variant);
    const int grp = tu.group > 0 ? tu.group : rhs_group(g, in.prec, rl.n);  // in RHS
    a.group = (grp + G - 1) / G;
    if (a.group > ntup) a.group = ntup;
    if (rl.n > 1 && !batch16(ntup)) return hipErrorInvalidValue;
    dim3 grid(a.nblk * ntup), block(HOP_BLOCK);
    const bool s = epi != EPI_K1, n = partial != nullptr;
    if (s && !self.data) return hipErrorInvalidValue;
    a.epi = ep == EP_STORE ? epi : EPI_K2;
    const bool nt = rl.n == 1;
    const unsigned lds = tu.lds;
    if (!ALL) {
        if (nt)
            go_w<SP, LK, true, ORD_PLAIN, false, 1>(a, s, n, ep, grid, block, lds, st);
        else
            go_w<SP, LK, false, ORD_PLAIN, false, 1>(a, s, n, ep, grid, block, lds, st);
        return hipGetLastError();
    }
    if (MULTI && G > 1) {
        if constexpr (SP::coded && __is_same(LK, L16R)) {
            // two RHS per lane of 16-bit spinors: the 16-bit kernel
            if (hop16_ok(g, a.phase_mask)) {
                launch_hop16(a, false, true, true, variant, s, n, ep, grid, block, lds, st);
                return hipGetLastError();
            }
        }
        // several RHS per lane: no scheduling-barrier flavours (same block order)
        const int ord = variant == 0 ? ORD_PLAIN : variant <= 2 ? ORD_ZSLAB : ORD_TSLAB;
#define GOM(GG)                                                                                \
    do {                                                                                       \
        if (ord == ORD_ZSLAB)                                                                  \
            go_w<SP, LK, false, ORD_ZSLAB, false, GG>(a, s, n, ep, grid, block, lds, st);          \
        else if (ord == ORD_TSLAB)                                                             \
            go_w<SP, LK, false, ORD_TSLAB, false, GG>(a, s, n, ep, grid, block, lds, st);          \
        else                                                                                   \
            go_w<SP, LK, false, ORD_PLAIN, false, GG>(a, s, n, ep, grid, block, lds, st);          \
    } while (0)
        if constexpr (MULTI) GOM(2);
#undef GOM
        return hipGetLastError();
    }
    if constexpr (SP::coded && __is_same(LK, L16R)) {
        // one RHS per lane: the 16-bit kernel, for one RHS or a batch
        if (hop16_ok(g, a.phase_mask)) {
            launch_hop16(a, false, !nt, false, variant, s, n, ep, grid, block, lds, st);
            return hipGetLastError();
        }
    }
#define GOV(ORD, SB)                                                          \
    do {                                                                      \
        if (nt)                                                               \
            go_w<SP, LK, true, ORD, SB, 1>(a, s, n, ep, grid, block, lds, st);    \
        else                                                                  \
            go_w<SP, LK, false, ORD, SB, 1>(a, s, n, ep, grid, block, lds, st);   \
    } while (0)
    switch (variant) {
    case 1: GOV(ORD_ZSLAB, false); break;
    case 2: GOV(ORD_ZSLAB, true); break;
    case 3: GOV(ORD_TSLAB, false); break;
    case 4: GOV(ORD_TSLAB, true); break;
    default: GOV(ORD_PLAIN, false); break;
    }
#undef GOV
    return hipGetLastError();
}

}  // namespace tmq
