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

// variant table: {W, SLAB, SB}; the link loads are non-temporal for a single
// RHS (each link is used once) and cached for a batch (each link is used once
// per RHS of a group, from L2)
struct HopVariant {
    int w;
    bool slab, sb;
};
static const HopVariant kVariants[HOP_VARIANTS] = {
    {0, false, false}, {0, true, false}, {0, true, true}, {2, true, true}, {2, false, true},
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


// per-format entry points (hop_f64.hip, hop_f32.hip, hop_f16.hip)
#define TMQ_HOP_ARGS                                                                                       \
    const Geom &g, int out_par, const FieldDesc &in, const FieldDesc &self, const FieldDesc &out,           \
        const LinkDesc &lk, const OpParams &op, int epi, int sign, const RhsList &rl, double *partial,      \
        long pstride, const CgScalars *scal, int variant, int group, hipStream_t st
hipError_t launch_hop_f64(TMQ_HOP_ARGS);
hipError_t launch_hop_f32(TMQ_HOP_ARGS);
hipError_t launch_hop_f16(TMQ_HOP_ARGS);
hipError_t launch_hop_b16(TMQ_HOP_ARGS);

hipError_t launch_hop(TMQ_HOP_ARGS)
{
    if (in.prec != out.prec || (self.data && self.prec != in.prec)) return hipErrorInvalidValue;
    switch (in.prec) {
    case P64: return launch_hop_f64(g, out_par, in, self, out, lk, op, epi, sign, rl, partial, pstride, scal, variant, group, st);
    case P32: return launch_hop_f32(g, out_par, in, self, out, lk, op, epi, sign, rl, partial, pstride, scal, variant, group, st);
    case P16: return launch_hop_f16(g, out_par, in, self, out, lk, op, epi, sign, rl, partial, pstride, scal, variant, group, st);
    case PB16: return launch_hop_b16(g, out_par, in, self, out, lk, op, epi, sign, rl, partial, pstride, scal, variant, group, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace tmq
