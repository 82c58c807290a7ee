// Unsigned 32-bit division by a divisor fixed at launch; no HIP dependency
// (the host builds the constants, the kernels divide, a CPU test checks it).
#pragma once

#include <stdint.h>

namespace lbm {

// n / d as a multiply-high and two shifts (Granlund and Montgomery, "Division
// by invariant integers using multiplication", 1994, Fig. 4.1): for d >= 1,
// l = ceil(log2 d), m = floor(2^32 (2^l - d) / d) + 1, and every n < 2^32
// gives n / d = (t + ((n - t) >> min(l, 1))) >> max(l - 1, 0) with
// t = mulhi(n, m).  On a uniform n all of it runs on the scalar unit (an
// integer division would expand into vector-unit reciprocal code).
struct DivU32 {
    uint32_t m, s1, s2;
};

// d >= 1 (grid extents are validated before; 0 is taken as 1)
inline DivU32 make_divu32(uint32_t d)
{
    if (d == 0) d = 1;
    uint32_t l = 0;
    while ((uint64_t(1) << l) < d) ++l;
    const uint64_t m = ((uint64_t(1) << 32) * ((uint64_t(1) << l) - d)) / d + 1;
    return DivU32{uint32_t(m), l < 1 ? l : 1u, l > 1 ? l - 1 : 0u};
}

__host__ __device__ inline uint32_t divu(const DivU32 &q, uint32_t n)
{
    const uint32_t t = uint32_t((uint64_t(n) * q.m) >> 32);  // mulhi(n, m)
    return (t + ((n - t) >> q.s1)) >> q.s2;
}

}  // namespace lbm
