// Correctly rounded FP64 division with a short dependency chain, for the
// substitution steps of the leaf and batched solvers (one division per row
// of the triangle, each on the critical path of the row recurrence).
//
// With r = RN(1/d) computed beforehand (off the critical path):
//   q0 = RN(a r)                  lies within two ulps of a/d,
//   q1 = RN(q0 + r (a - d q0))    lies within one ulp of a/d,
//   q  = RN(q1 + r (a - d q1))    equals RN(a/d) exactly,
// the last step by Markstein's theorem (r within half an ulp of 1/d and q1
// within one ulp of a/d); the remainders a - d q are exact under FMA.  So the
// result is bit for bit the IEEE quotient.  The theorem assumes no underflow
// or overflow: the guard below keeps every intermediate normal
// (|a| in [2^-400, 2^400] or a = 0, |d| in [2^-500, 2^500]); for any other
// operand (subnormal, infinite, NaN or extreme) the caller falls back to the
// IEEE division.
#pragma once

namespace redsea {

__device__ __forceinline__ bool div_fast_divisor(double d) {
    const double ad = __builtin_fabs(d);
    return ad >= 0x1p-500 && ad <= 0x1p500;
}

// a / d, given r = 1.0 / d and dok = div_fast_divisor(d), without branches.
// The result is the IEEE quotient whenever ok comes back true; callers redo
// the division in IEEE arithmetic otherwise.  A zero numerator is exact as
// a * r, which carries the sign of the IEEE quotient.
__device__ __forceinline__ double div_rn_fast(double a, double d, double r, bool dok, bool& ok) {
    const double q0 = a * r;
    const double e0 = __builtin_fma(-d, q0, a);
    const double q1 = __builtin_fma(e0, r, q0);
    const double e1 = __builtin_fma(-d, q1, a);
    const double q = __builtin_fma(e1, r, q1);
    const double aa = __builtin_fabs(a);
    ok = dok && ((aa >= 0x1p-400 && aa <= 0x1p400) || a == 0.0);
    return a == 0.0 ? q0 : q;
}

}  // namespace redsea
