// Division of 32-bit unsigned integers by an invariant divisor d >= 1 with a
// multiply-high, a subtract, an add and two shifts (Granlund and Montgomery,
// "Division by invariant integers using multiplication", PLDI 1994, Sec. 4):
// with l = ceil(log2 d) and m = floor(2^32 (2^l - d) / d) + 1,
//   x / d = (t + ((x - t) >> min(l, 1))) >> max(l - 1, 0),  t = mulhi(m, x),
// exact for every 32-bit x.  The host prepares (m, shifts); kernels divide.
#pragma once

#include <cstdint>

namespace rac {

struct FastDiv {
    uint32_t m, s1, s2;
};

__host__ __device__ inline FastDiv make_fastdiv(uint32_t d) {
    uint32_t l = 0;
    while (l < 32 && (1ull << l) < d) ++l;
    FastDiv f;
    f.m = (uint32_t)((((1ull << 32) * ((1ull << l) - d)) / d) + 1);
    f.s1 = l < 1 ? l : 1;
    f.s2 = l > 1 ? l - 1 : 0;
    return f;
}

__host__ __device__ inline uint32_t fastdiv(uint32_t x, const FastDiv& f) {
    const uint32_t t = (uint32_t)(((uint64_t)f.m * x) >> 32);
    return (t + ((x - t) >> f.s1)) >> f.s2;
}

}  // namespace rac
