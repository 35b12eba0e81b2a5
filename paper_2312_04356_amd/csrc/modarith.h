// Exact modular arithmetic for primes t < 2^50 on gfx950, done in FP64 with FMA.
//
// Residues live in HBM as uint64 and are moved into doubles in registers (every
// integer below 2^53 is exact in a double).  A product a*b (|a|,|b| < 2^50) is
// split exactly as h + l with h = fl(a*b) and l = fma(a, b, -h) (Dekker/Kahan
// two-product); a quotient estimate c = rint(h * (1/t)) is off by at most a
// few units, so h - c*t is an integer below 2^52 that one fma computes exactly,
// and adding l gives the exact a*b - c*t.  On gfx950 this costs ~8 full-rate
// FP64 operations, about 1.8x the throughput of a 64-bit Shoup product built from
// 32-bit integer multiplies (measured: 3.2 vs 1.8 T products/s).
//
// Bounds used below (u = 2^-53, every modulus t in [2^40, 2^50)):
//   mul_canon:  a, b in [0, t)              -> |ab/t - c| < 7/8, result in [0, t)
//   mul_lazy:   |a| <= 2^50, b in [0, t)    -> exact representative in (-t, t)
//   corr:       integer s in (-t, 2t)       -> [0, t)
//   reduce:     integer |x| < 2^53          -> [0, t)
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define NJ_HD __host__ __device__ __forceinline__

namespace nj {

constexpr double kTwo52 = 4503599627370496.0;  // 2^52

// uint64 x < 2^52  <->  double, by placing x in the mantissa of 2^52 + x
NJ_HD double u2d(uint64_t x)
{
    union { uint64_t u; double d; } v;
    v.u = x | 0x4330000000000000ull;
    return v.d - kTwo52;
}
NJ_HD uint64_t d2u(double x)  // x an integer in [0, 2^52)
{
    union { uint64_t u; double d; } v;
    v.d = x + kTwo52;
    return v.u & 0x000FFFFFFFFFFFFFull;
}

struct Mod {
    double t;   // the prime
    double ti;  // fl(1 / t)
};

// An integer s in (-t, 2t)  ->  s mod t in [0, t), with no compare or select:
// floor(s/t) = rint((s + 1/2)/t - 1/2), evaluated as rint(fma(s, ti, ti/2 - 1/2)).  The
// exact value lies at least 0.5/t >= 2^-51 from a half-integer; the computed one is
// within 2^-52 (ti's relative error 2^-53 on |s/t| < 2) + 2^-53 (the fma's rounding) +
// 2^-55 (the offset's rounding) of it, so rint returns floor(s/t) exactly.
NJ_HD double corr(double s, Mod m)
{
    const double c = rint(fma(s, m.ti, fma(0.5, m.ti, -0.5)));
    return fma(-c, m.t, s);
}

// a, b in [0, t)  ->  a*b mod t in [0, t)
NJ_HD double mul_canon(double a, double b, Mod m)
{
    double h = a * b;
    double l = fma(a, b, -h);
    double c = rint(h * m.ti);
    return corr(fma(-c, m.t, h) + l, m);
}

// Shoup-style product with a fixed canonical factor w and its companion wq = fl(w/t):
// b in [0, t) -> b*w mod t in [0, t).  |b wq - b w/t| <= 2u b w/t < 1/4.
NJ_HD double mul_shoup(double b, double w, double wq, Mod m)
{
    double h = b * w;
    double l = fma(b, w, -h);
    double c = rint(b * wq);
    return corr(fma(-c, m.t, h) + l, m);
}

// Lazy product for signed operands |a| < 2^50, |b| < t: returns an exact
// representative of a*b mod t in (-2t, 2t).  |ab/t| < 2^50, quotient error
// < 3u 2^50 < 1/2, so |ab - ct| < t; h - ct and the sum stay below 2^52.
NJ_HD double mul_lazy(double a, double b, Mod m)
{
    double h = a * b;
    double l = fma(a, b, -h);
    double c = rint(h * m.ti);
    return fma(-c, m.t, h) + l;
}

// any exact integer |x| < 2^52  ->  x mod t in [0, t)
NJ_HD double reduce(double x, Mod m)
{
    double c = rint(x * m.ti);
    return corr(fma(-c, m.t, x), m);
}

NJ_HD double add_mod(double a, double b, Mod m) { return corr(a + b, m); }
NJ_HD double sub_mod(double a, double b, Mod m) { return corr(a - b, m); }

}  // namespace nj
