// hop16_f16.hip -- instantiations of the 16-bit hop kernel
// (hop16_kernel in hop_impl.h) for FP16 spinor codes.
#include "hop_impl.h"

namespace tmq {

void launch_hop16(const HopArgs<SpH16, L16R> &a, bool nd, bool batch, bool two, int variant, bool s, bool n, int ep,
                  dim3 grid, dim3 block, unsigned lds, hipStream_t st)
{
    launch_hop16_impl<SpH16>(a, nd, batch, two, variant, s, n, ep, grid, block, lds, st);
}

}  // namespace tmq
