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
    float f = (float)x;
    if ((double)f != x) {
        uint32_t u = __float_as_uint(f);
        if (fabs((double)f) > fabs(x)) u -= 1;  // rounded away from zero: step back
        u |= 1u;
        f = __uint_as_float(u);
    }
    return f;
}

// Nearest-even binary16 value of a double, with a single rounding.
__device__ __forceinline__ _Float16 half_rn(double x) { return (_Float16)float_rto(x); }

__device__ __forceinline__ _Float16 half_rn(float x) { return (_Float16)x; }

}  // namespace md
