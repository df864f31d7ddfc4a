// hop.hip -- dispatch of the hopping half-sweep to the per-format translation
// units, the variant table and grid sizes.
#include "devutil.h"
#include "views.h"

namespace tmq {

int hop_grid(long n)
{
    long g = (n + HOP_BLOCK - 1) / HOP_BLOCK;
    g = (g + 7) / 8 * 8;  // a multiple of the XCD count for the remap
    return (int)g;
}

// variant table: {order, SB}; the link loads are non-temporal for a single
// RHS (each link is used once) and cached for a batch (each link is used once
// per RHS of a group, from L2)
struct HopVariant {
    int ord;
    bool sb;
};
static const HopVariant kVariants[HOP_VARIANTS] = {
    {ORD_PLAIN, false}, {ORD_ZSLAB, false}, {ORD_ZSLAB, true}, {ORD_TSLAB, false}, {ORD_TSLAB, true},
};

bool hop_variant_valid(const Geom &g, int v)
{
    if (v < 0 || v >= HOP_VARIANTS) return false;
    if (kVariants[v].ord == ORD_ZSLAB) return g.LZ >= 8;
    if (kVariants[v].ord == ORD_TSLAB) return g.T >= 8;
    return true;
}

int hop_grid_variant(const Geom &g, int v, int lanes_per_site)
{
    const long L = lanes_per_site;
    if (!hop_variant_valid(g, v) || kVariants[v].ord == ORD_PLAIN) return hop_grid(L * g.vh);
    const long plane = (long)g.LY * g.XH;
    long per_xcd;
    if (kVariants[v].ord == ORD_ZSLAB) {
        const long zc = g.LZ / 8 + (g.LZ % 8 ? 1 : 0);
        per_xcd = (L * g.T * zc * plane + HOP_BLOCK - 1) / HOP_BLOCK;
    } else {
        const long tc = g.T / 8 + (g.T % 8 ? 1 : 0);
        per_xcd = (L * g.LZ * tc * plane + HOP_BLOCK - 1) / HOP_BLOCK;
    }
    return (int)(8 * per_xcd);
}


bool hop_all_variants(int prec, int link_fmt)
{
    // the pairings of a solve's inner iteration and of FP64; the others
    // (FP32 spinors on FP16 links, 16-bit spinors on FP32 links) are
    // instantiated with the plain order only
    if (prec == P64) return true;
    if (prec == P32) return link_fmt == LK32R;
    return link_fmt == LK16R;
}

// per-format entry points (hop_f64.hip, hop_f32.hip, hop_f16.hip)
#define TMQ_HOP_ARGS                                                                                       \
    const Geom &g, int out_par, const FieldDesc &in, const FieldDesc &self, const FieldDesc &out,           \
        const LinkDesc &lk, const OpParams &op, int epi, int sign, const RhsList &rl, double *partial,      \
        long pstride, const CgScalars *scal, const HopTune &tu, hipStream_t st, const CgFields *cg
hipError_t launch_hop_f64(TMQ_HOP_ARGS);
hipError_t launch_hop_f32(TMQ_HOP_ARGS);
hipError_t launch_hop_f16(TMQ_HOP_ARGS);
hipError_t launch_hop_b16(TMQ_HOP_ARGS);

hipError_t launch_hop(TMQ_HOP_ARGS)
{
    const bool fused = epi == EPI_K2_CG || epi == EPI_K2_RES;  // no output field
    if ((!fused && in.prec != out.prec) || (self.data && self.prec != in.prec)) return hipErrorInvalidValue;
    switch (in.prec) {
    case P64: return launch_hop_f64(g, out_par, in, self, out, lk, op, epi, sign, rl, partial, pstride, scal, tu, st, cg);
    case P32: return launch_hop_f32(g, out_par, in, self, out, lk, op, epi, sign, rl, partial, pstride, scal, tu, st, cg);
    case P16: return launch_hop_f16(g, out_par, in, self, out, lk, op, epi, sign, rl, partial, pstride, scal, tu, st, cg);
    case PB16: return launch_hop_b16(g, out_par, in, self, out, lk, op, epi, sign, rl, partial, pstride, scal, tu, st, cg);
    }
    return hipErrorInvalidValue;
}

}  // namespace tmq
