// hop_f32.hip -- hop half-sweep instantiations for one spinor format.
#include "hop_impl.h"

namespace tmq {

hipError_t launch_hop_f32(const Geom &g, int out_par, const FieldDesc &in, const FieldDesc &self, const FieldDesc &out,
                   const LinkDesc &lk, const OpParams &op, int epi, int sign, const RhsList &rl, double *partial,
                   long pstride, const CgScalars *scal, const HopTune &tu, hipStream_t st, const CgFields *cg)
{
#define GO(SPT, LKT, ALL, MULTI) return go<SPT, LKT, ALL, MULTI>(g, out_par, in, self, out, lk, op, epi, sign, rl, partial, pstride, scal, tu, st, cg)
    if (lk.fmt == LK32R) GO(SpF32, L32R, true, true);
    if (lk.fmt == LK16R) GO(SpF32, L16R, false, false);
    if (lk.fmt == LK32F) GO(SpF32, L32F, false, false);
#undef GO
    return hipErrorInvalidValue;
}

}  // namespace tmq
