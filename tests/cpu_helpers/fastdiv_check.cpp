// Host build of the hop kernels' division by launch constants (fastdiv.h), so
// that the multipliers can be checked on the CPU against plain division.
#include "../../paper_0905_3331_amd/csrc/fastdiv.h"

using namespace tmq;

// quotients of n[i] by d through the multiplier of d
extern "C" void fastdiv_quotients(uint32_t d, const uint32_t *n, uint32_t *q, int count)
{
    const FastDiv f = make_fastdiv(d);
    for (int i = 0; i < count; i++) q[i] = fastdiv_q(n[i], f);
}
