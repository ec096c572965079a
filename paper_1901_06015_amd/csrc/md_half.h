// md_half.h -- binary16 rounding used by the epilogues of half-precision C.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace md {

// A double rounded to float with round-to-odd (truncate, then set the last
// bit when inexact).  With the 13 bits float has beyond binary16, rounding
// this value to binary16 gives the nearest-even binary16 value of x itself:
// one rounding, not two.
__device__ __forceinline__ float float_rto(double x) {
    // branch-free (selects): inside the k loop a branch here would split the
    // loop and make the staging wait for its loads at once
    const float f = (float)x;
    const bool inexact = (double)f != x;
    const bool away = fabs((double)f) > fabs(x);  // rounded away from zero: step back
    const uint32_t u = __float_as_uint(f) - (uint32_t)(inexact & away);
    return __uint_as_float(u | (uint32_t)inexact);
}

// Nearest-even binary16 value of a double, with a single rounding.
__device__ __forceinline__ _Float16 half_rn(double x) { return (_Float16)float_rto(x); }

__device__ __forceinline__ _Float16 half_rn(float x) { return (_Float16)x; }

// Error-free sum of two floats (Knuth's TwoSum): s + e == a + b exactly.
// Contraction is off so that no addition here fuses with a product of the
// caller (the error term must describe the rounded operands).
__device__ __forceinline__ float two_sum(float a, float b, float &e) {
#pragma clang fp contract(off)
    const float s = a + b;
    const float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
    return s;
}

// Round-to-odd float of the exact value s + r, where s = RN(s + r) (|r| at
// most half an ulp of s): keep s if exact, else truncate toward zero and set
// the last bit.
__device__ __forceinline__ float jam_odd(float s, float r) {
    if (r == 0.0f) return s;
    if (s == 0.0f) return r;
    uint32_t u = __float_as_uint(s);
    if ((r < 0.0f) != (s < 0.0f)) u -= 1;  // s lies beyond the exact value: step toward zero
    return __uint_as_float(u | 1u);
}

// Round-to-odd float of a + b (two floats).
__device__ __forceinline__ float add_rto(float a, float b) {
    float e;
    const float s = two_sum(a, b, e);
    return jam_odd(s, e);
}

// Round-to-odd float of a + b + c (three floats): the two error-free sums and
// the round-to-odd addition of their low parts of Boldo and Melquiond
// ("Emulation of FMA and correctly rounded sums: proved algorithms using
// rounding to odd", IEEE Trans. Computers 57(4), 2008); the sticky last bit
// of the low part carries what the high part drops, so rounding the result
// once more (to binary16) rounds the exact sum once.
__device__ __forceinline__ float add3_rto(float a, float b, float c) {
    float ul, tl;
    const float uh = two_sum(b, c, ul);
    const float th = two_sum(a, uh, tl);
    return add_rto(th, add_rto(tl, ul));
}

}  // namespace md
