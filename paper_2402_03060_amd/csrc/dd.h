// Double-double arithmetic (an unevaluated sum hi + lo of two doubles,
// about 106 significant bits), after Dekker and Knuth's error-free
// transformations.  Used by the encoder so that the rounding to integers of
// scale * m_j is decided on a value accurate far below one unit.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

struct dd {
    double hi, lo;
};

__host__ __device__ __forceinline__ dd dd_make(double h, double l) { dd r; r.hi = h; r.lo = l; return r; }

// s + e = a + b exactly
__host__ __device__ __forceinline__ dd two_sum(double a, double b)
{
    double s = a + b;
    double bb = s - a;
    double e = (a - (s - bb)) + (b - bb);
    return dd_make(s, e);
}
// |a| >= |b|
__host__ __device__ __forceinline__ dd quick_two_sum(double a, double b)
{
    double s = a + b;
    return dd_make(s, b - (s - a));
}
// p + e = a * b exactly
__host__ __device__ __forceinline__ dd two_prod(double a, double b)
{
    double p = a * b;
    return dd_make(p, fma(a, b, -p));
}
__host__ __device__ __forceinline__ dd dd_add(dd a, dd b)
{
    dd s = two_sum(a.hi, b.hi);
    dd t = two_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = quick_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return quick_two_sum(s.hi, s.lo);
}
__host__ __device__ __forceinline__ dd dd_mul_d(dd a, double b)
{
    dd p = two_prod(a.hi, b);
    p.lo += a.lo * b;
    return quick_two_sum(p.hi, p.lo);
}
__host__ __device__ __forceinline__ dd dd_mul(dd a, dd b)
{
    dd p = two_prod(a.hi, b.hi);
    p.lo += a.hi * b.lo + a.lo * b.hi;
    return quick_two_sum(p.hi, p.lo);
}
__host__ __device__ __forceinline__ dd dd_div_d(dd a, double b)
{
    double q1 = a.hi / b;
    dd p = two_prod(q1, b);
    dd r = two_sum(a.hi, -p.hi);
    r.lo += a.lo - p.lo;
    double q2 = (r.hi + r.lo) / b;
    return quick_two_sum(q1, q2);
}
__host__ __device__ __forceinline__ dd dd_neg(dd a) { return dd_make(-a.hi, -a.lo); }
