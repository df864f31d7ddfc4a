// fastdiv.h -- division by a launch constant as a multiply-high (host side:
// the multipliers and the reference formula; the kernels apply the same
// formula with __umulhi).
#pragma once
#include <stdint.h>

namespace tmq {

// Division by a divisor 1 <= d <= 2^31 that is uniform over a launch, for
// numerators n < 2^31, as a multiply-high, an add and a shift: with s = ceil(log2 d) and
// M = ceil(2^(32+s) / d) (2^32 <= M < 2^33), floor(n / d) = floor(n M / 2^(32+s))
// because the rounding excess e = M d - 2^(32+s) < d <= 2^s keeps n e / 2^(32+s)
// below 1/d; m holds M - 2^32, so q = (umulhi(n, m) + n) >> s (the sum stays
// below 2^32 since n < 2^31).  Granlund and Montgomery's round-up multiplier.
struct FastDiv {
    uint32_t m = 0, s = 0;
};
inline FastDiv make_fastdiv(uint32_t d)
{
    FastDiv f;
    uint32_t s = 0;
    while (s < 31 && (1ull << s) < d) s++;
    const uint64_t num = 1ull << (32 + s);  // at most 2^63, so num + d - 1 fits
    const uint64_t M = (num + d - 1) / d;
    f.m = (uint32_t)(M - (1ull << 32));
    f.s = s;
    return f;
}
// the quotient by the same formula (host side)
inline uint32_t fastdiv_q(uint32_t n, FastDiv f)
{
    return (uint32_t)((((uint64_t)n * f.m) >> 32) + n) >> f.s;
}

}  // namespace tmq
