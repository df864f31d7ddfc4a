// hop.hip -- the hopping half-sweep H_eo / H_oe with fused site-term epilogues.
//
// One output site per lane.  For each of the 8 neighbours the lane loads the
// neighbour spinor, projects it to two spin components with (1 +- gamma_mu)
// (Sec. 4.1), multiplies both by the link U(x,mu) or U(x-mu,mu)^+ (each link
// is read exactly once per half-sweep: the forward links of the output
// parity, the backward links of the input parity), multiplies by the boundary
// phase e^{+-i theta_mu pi/L_mu} (Sec. 4.1.2) and accumulates the rebuilt
// four-spinor.  The epilogue forms  out = A * self + B * acc  per spin half,
// which covers both factors of the even/odd operator (eqs. (eo3), (eo4)) and
// the full-lattice operator, and optionally reduces |out|^2 per block.
//
// Work distribution: blocks of 256 lanes over consecutive eo indices (x
// fastest, then y, z, t).  Hardware hands consecutive workgroups to the 8 XCDs
// in turn; the block index is remapped so that each XCD walks a contiguous
// slab of the lattice and its private L2 sees the y/z/t neighbours of its
// own sites.
#include "devutil.h"
#include "views.h"

namespace tmq {

int hop_grid(long n)
{
    long g = (n + HOP_BLOCK - 1) / HOP_BLOCK;
    g = (g + 7) / 8 * 8;  // a multiple of the XCD count for the remap
    return (int)g;
}

// variant table: {W, NT, SLAB, SB}
struct HopVariant {
    int w;
    bool nt, slab, sb;
};
static const HopVariant kVariants[HOP_VARIANTS] = {
    {0, true, false, false}, {0, true, true, false}, {0, true, true, true},
    {2, true, true, true},   {3, true, true, true},  {2, true, false, true},
};

bool hop_variant_valid(const Geom &g, int v)
{
    if (v < 0 || v >= HOP_VARIANTS) return false;
    return !kVariants[v].slab || g.LZ >= 8;
}

int hop_grid_variant(const Geom &g, int v)
{
    if (!hop_variant_valid(g, v) || !kVariants[v].slab) return hop_grid(g.vh);
    const long zc = g.LZ / 8 + (g.LZ % 8 ? 1 : 0);
    const long per_xcd = ((long)g.T * zc * g.LY * g.XH + HOP_BLOCK - 1) / HOP_BLOCK;
    return (int)(8 * per_xcd);
}

__device__ __forceinline__ int xcd_remap(int bid, int nblk)
{
    // nblk is a multiple of 8: XCD k = bid % 8 gets logical blocks [k*nblk/8, (k+1)*nblk/8)
    return (bid & 7) * (nblk >> 3) + (bid >> 3);
}

template <class SP, class LK>
struct HopArgs {
    Geom g;
    int out_par;
    SP in, self, out;
    LK lk;
    HopCoef c;
    double *partial;
    const int *skip;
};

template <int MU, bool NT, class SP, class LK, typename R>
__device__ __forceinline__ void hop_dir(const HopArgs<SP, LK> &a, spinor<R> &acc, long h, long hf, long hb)
{
    const cx<R> ph = {(R)a.c.ph[MU][0], (R)a.c.ph[MU][1]};
    spinor<R> s;
    half<R> p, w;
    su3<R> u;
    // forward: e^{i theta pi/L} U(x,mu) (1 + gamma_mu) psi(x+mu); U at the output site
    a.in.load(hf, s);
    project<MU, +1>(s, p);
    a.lk.template load<NT>(a.out_par, MU, h, u);
    link_mul<false>(u, p, ph, w);
    reconstruct_add<MU, +1>(acc, w);
    // backward: e^{-i theta pi/L} U(x-mu,mu)^+ (1 - gamma_mu) psi(x-mu); U at the neighbour
    a.in.load(hb, s);
    project<MU, -1>(s, p);
    a.lk.template load<NT>(a.out_par ^ 1, MU, hb, u);
    link_mul<true>(u, p, conj(ph), w);
    reconstruct_add<MU, -1>(acc, w);
}

// Variant bits: W > 0 asks the compiler for at least W waves per SIMD (a
// register budget of 512 / W per lane), W = 0 leaves the choice to the
// compiler; NT makes the link loads non-temporal; SLAB gives XCD k = block % 8
// its own range of z-planes, walked with t outermost, so that the sites of
// time-slices t-1, t, t+1 that one XCD needs at a time fit its L2; SB puts a
// scheduling barrier between directions, which bounds how many loads the
// compiler hoists and therefore the register count.  The autotuner picks the
// fastest variant per format and lattice.
template <class SP, class LK, bool SELF, bool NORM, int W, bool NT, bool SLAB, bool SB>
__global__ __launch_bounds__(HOP_BLOCK) __attribute__((amdgpu_waves_per_eu(W > 0 ? W : 1, W > 0 ? 8 : 8)))
void hop_kernel(HopArgs<SP, LK> a)
{
    using R = typename LK::real;
    if (a.skip && *a.skip) return;
    const Geom &g = a.g;
    const long plane = (long)g.LY * g.XH;  // sites of one (t, z) plane
    long h;
    int t, z, y;
    unsigned xh;
    bool active;
    if (SLAB) {
        const int j = blockIdx.x & 7;
        const int zb = g.LZ >> 3, zr = g.LZ & 7;
        const int zc = zb + (j < zr ? 1 : 0), z0 = j * zb + (j < zr ? j : zr);
        const long S = (long)zc * plane;  // sites of one time-slice of this slab
        const long l = (long)(blockIdx.x >> 3) * HOP_BLOCK + threadIdx.x;
        active = l < (long)g.T * S;
        const unsigned lu = active ? (unsigned)l : 0u;
        t = (int)(lu / (unsigned)S);
        const unsigned rem = lu - (unsigned)t * (unsigned)S;
        z = z0 + (int)(rem / (unsigned)plane);
        const unsigned r2 = rem - (unsigned)(z - z0) * (unsigned)plane;
        y = (int)(r2 / (unsigned)g.XH);
        xh = r2 - (unsigned)y * (unsigned)g.XH;
        h = ((long)t * g.LZ + z) * plane + (long)y * g.XH + xh;
    } else {
        const int lb = xcd_remap(blockIdx.x, gridDim.x);
        h = (long)lb * HOP_BLOCK + threadIdx.x;
        active = h < g.vh;
        const unsigned hu = active ? (unsigned)h : 0u;
        xh = hu % (unsigned)g.XH;
        unsigned r = hu / (unsigned)g.XH;
        y = (int)(r % (unsigned)g.LY);
        r /= (unsigned)g.LY;
        z = (int)(r % (unsigned)g.LZ);
        t = (int)(r / (unsigned)g.LZ);
    }
    double nrm = 0.0;
    if (active) {
        // x parity makes (t+z+y+x) = out_par mod 2
        const int x = 2 * (int)xh + ((a.out_par + t + z + y) & 1);
        const long row = h - xh;  // eo index of (t, z, y, 0)
        const long sy = g.XH, sz = plane, stt = (long)g.LZ * plane;

        spinor<R> acc;
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int j = 0; j < 3; j++) acc.c[i][j] = cx<R>{R(0), R(0)};

        hop_dir<0, NT>(a, acc, h, t + 1 == g.T ? h - (g.T - 1) * stt : h + stt, t == 0 ? h + (g.T - 1) * stt : h - stt);
        if (SB) __builtin_amdgcn_sched_barrier(0);
        hop_dir<1, NT>(a, acc, h, row + ((x + 1 == g.LX ? 0 : x + 1) >> 1), row + ((x == 0 ? g.LX - 1 : x - 1) >> 1));
        if (SB) __builtin_amdgcn_sched_barrier(0);
        hop_dir<2, NT>(a, acc, h, y + 1 == g.LY ? h - (g.LY - 1) * sy : h + sy, y == 0 ? h + (g.LY - 1) * sy : h - sy);
        if (SB) __builtin_amdgcn_sched_barrier(0);
        hop_dir<3, NT>(a, acc, h, z + 1 == g.LZ ? h - (g.LZ - 1) * sz : h + sz, z == 0 ? h + (g.LZ - 1) * sz : h - sz);

        spinor<R> o;
        const cx<R> Bu = {(R)a.c.B[0][0], (R)a.c.B[0][1]}, Bd = {(R)a.c.B[1][0], (R)a.c.B[1][1]};
        if (SELF) {
            spinor<R> sf;
            a.self.load(h, sf);
            const cx<R> Au = {(R)a.c.A[0][0], (R)a.c.A[0][1]}, Ad = {(R)a.c.A[1][0], (R)a.c.A[1][1]};
#pragma unroll
            for (int j = 0; j < 3; j++) {
                o.c[0][j] = fma(Au, sf.c[0][j], Bu * acc.c[0][j]);
                o.c[1][j] = fma(Au, sf.c[1][j], Bu * acc.c[1][j]);
                o.c[2][j] = fma(Ad, sf.c[2][j], Bd * acc.c[2][j]);
                o.c[3][j] = fma(Ad, sf.c[3][j], Bd * acc.c[3][j]);
            }
        } else {
#pragma unroll
            for (int j = 0; j < 3; j++) {
                o.c[0][j] = Bu * acc.c[0][j];
                o.c[1][j] = Bu * acc.c[1][j];
                o.c[2][j] = Bd * acc.c[2][j];
                o.c[3][j] = Bd * acc.c[3][j];
            }
        }
        a.out.store(h, o);
        if (NORM) {
            R n2 = R(0);
#pragma unroll
            for (int i = 0; i < 4; i++)
#pragma unroll
                for (int j = 0; j < 3; j++) n2 += norm2(o.c[i][j]);
            nrm = (double)n2;
        }
    }
    if (NORM) {
        // one partial per block; the slab order indexes them by the physical block
        __shared__ double sh[HOP_BLOCK / 64];
        double s = block_sum(nrm, sh);
        if (threadIdx.x == 0) a.partial[SLAB ? (int)blockIdx.x : xcd_remap(blockIdx.x, gridDim.x)] = s;
    }
}

// ------------------------------------------------------------- dispatch

template <class SP, class LK, int W, bool NT, bool SLAB, bool SB>
static void go_w(const HopArgs<SP, LK> &a, bool s, bool n, dim3 grid, dim3 block, hipStream_t st)
{
    if (s && n)
        hipLaunchKernelGGL((hop_kernel<SP, LK, true, true, W, NT, SLAB, SB>), grid, block, 0, st, a);
    else if (s)
        hipLaunchKernelGGL((hop_kernel<SP, LK, true, false, W, NT, SLAB, SB>), grid, block, 0, st, a);
    else if (n)
        hipLaunchKernelGGL((hop_kernel<SP, LK, false, true, W, NT, SLAB, SB>), grid, block, 0, st, a);
    else
        hipLaunchKernelGGL((hop_kernel<SP, LK, false, false, W, NT, SLAB, SB>), grid, block, 0, st, a);
}

// ALL = false: only variant 0 is instantiated (rarely used format pairs)
template <class SP, class LK, bool ALL>
static hipError_t go(const Geom &g, int out_par, const FieldDesc &in, const FieldDesc &self,
                     const FieldDesc &out, const LinkDesc &lk, const HopCoef &c, double *partial,
                     const int *skip, int variant, hipStream_t st)
{
    HopArgs<SP, LK> a;
    a.g = g;
    a.out_par = out_par;
    a.in = make_sp<SP>(in);
    a.self = self.data ? make_sp<SP>(self) : a.in;
    a.out = make_sp<SP>(out);
    a.lk = make_lk<LK>(lk);
    a.c = c;
    a.partial = partial;
    a.skip = skip;
    if (!ALL || !hop_variant_valid(g, variant)) variant = 0;
    dim3 grid(hop_grid_variant(g, variant)), block(HOP_BLOCK);
    const bool s = self.data != nullptr, n = partial != nullptr;
    if (!ALL) {
        go_w<SP, LK, 0, true, false, false>(a, s, n, grid, block, st);
        return hipGetLastError();
    }
    switch (variant) {
    case 1: go_w<SP, LK, 0, true, true, false>(a, s, n, grid, block, st); break;
    case 2: go_w<SP, LK, 0, true, true, true>(a, s, n, grid, block, st); break;
    case 3: go_w<SP, LK, 2, true, true, true>(a, s, n, grid, block, st); break;
    case 4: go_w<SP, LK, 3, true, true, true>(a, s, n, grid, block, st); break;
    case 5: go_w<SP, LK, 2, true, false, true>(a, s, n, grid, block, st); break;
    default: go_w<SP, LK, 0, true, false, false>(a, s, n, grid, block, st); break;
    }
    return hipGetLastError();
}

hipError_t launch_hop(const Geom &g, int out_par, const FieldDesc &in, const FieldDesc &self,
                      const FieldDesc &out, const LinkDesc &lk, const HopCoef &c, double *partial,
                      const int *skip, int variant, hipStream_t st)
{
    if (in.prec != out.prec || (self.data && self.prec != in.prec)) return hipErrorInvalidValue;
#define GO(SPT, LKT, ALL) return go<SPT, LKT, ALL>(g, out_par, in, self, out, lk, c, partial, skip, variant, st)
    switch (in.prec) {
    case P64:
        if (lk.fmt == LK64F) GO(SpF64, L64F, true);
        if (lk.fmt == LK64R) GO(SpF64, L64R, true);
        break;
    case P32:
        if (lk.fmt == LK32R) GO(SpF32, L32R, true);
        if (lk.fmt == LK16R) GO(SpF32, L16R, false);
        break;
    case P16:
        if (lk.fmt == LK16R) GO(SpH16, L16R, true);
        if (lk.fmt == LK32R) GO(SpH16, L32R, false);
        break;
    case PB16:
        if (lk.fmt == LK16R) GO(SpB16, L16R, true);
        if (lk.fmt == LK32R) GO(SpB16, L32R, false);
        break;
    }
#undef GO
    return hipErrorInvalidValue;
}

}  // namespace tmq
