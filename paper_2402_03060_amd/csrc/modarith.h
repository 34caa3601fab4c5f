// Modular arithmetic on 64-bit residues for primes q < 2^61, built from the
// 32-bit integer ALUs of CDNA4 (the compiler lowers each 64x64 product to
// v_mad_u64_u32 / v_mul_hi_u32 sequences).
//
//   mul_shoup   x * w mod q for a fixed w with w' = floor(w 2^64 / q)
//               (Shoup's method): result in [0, 2q) for any 64-bit x.
//   mont_mul    a * b * 2^-64 mod q (Montgomery, R = 2^64): used where one
//               operand is stored pre-multiplied by R (keys, plaintexts).
//   reduce64    x mod q for any 64-bit x, with r = floor(2^64 / q).
//   WideAcc     a lazily reduced sum of Montgomery products (one reduction
//               per output instead of one per term).
//   fp_mulmod   x * w mod q in binary64 arithmetic for primes below 2^41
//               (FpModulus): the product is split exactly by an FMA and the
//               remainder formed by a second FMA; on gfx950 this runs about
//               three times the rate of the 32-bit-multiply Shoup product.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef uint64_t u64;
typedef uint32_t u32;
typedef int64_t i64;

// Per-prime constants, resident in device memory.
struct Modulus {
    u64 q;
    u64 ratio;     // floor(2^64 / q)
    u64 qinv_neg;  // -q^-1 mod 2^64
    u64 r2;        // 2^128 mod q  (mont_mul(x, r2) = x * 2^64 mod q)
    u64 half;      // (q - 1) / 2
    u64 n_inv;     // N^-1 mod q
    u64 n_inv_sh;  // Shoup companion of n_inv
    u64 pad;
};

// high 64 bits of a 64 x 64 product: four 32 x 32 + 64 multiply-adds
// (v_mad_u64_u32) whose addends absorb the carries, plus one 64-bit add
__host__ __device__ __forceinline__ u64 umulhi64(u64 a, u64 b)
{
#ifdef __HIP_DEVICE_COMPILE__
    const u32 a0 = (u32)a, a1 = (u32)(a >> 32), b0 = (u32)b, b1 = (u32)(b >> 32);
    const u64 p00 = (u64)a0 * b0;
    const u64 t = (u64)a0 * b1 + (p00 >> 32);
    const u64 v = (u64)a1 * b0 + (u32)t;
    return (u64)a1 * b1 + ((t >> 32) + (v >> 32));
#else
    return (u64)(((unsigned __int128)a * b) >> 64);
#endif
}

__host__ __device__ __forceinline__ u64 add_mod(u64 a, u64 b, u64 q)
{
    u64 s = a + b;
    return s >= q ? s - q : s;
}

__host__ __device__ __forceinline__ u64 sub_mod(u64 a, u64 b, u64 q)
{
    return a >= b ? a - b : a + q - b;
}

__host__ __device__ __forceinline__ u64 csub(u64 a, u64 q) { return a >= q ? a - q : a; }

// [0, 2q) result
__host__ __device__ __forceinline__ u64 mul_shoup_lazy(u64 x, u64 w, u64 w_sh, u64 q)
{
    u64 qh = umulhi64(x, w_sh);
    return x * w - qh * q;
}

__host__ __device__ __forceinline__ u64 mul_shoup(u64 x, u64 w, u64 w_sh, u64 q)
{
    return csub(mul_shoup_lazy(x, w, w_sh, q), q);
}

// a, b < q: returns a b 2^-64 mod q in [0, q)
__host__ __device__ __forceinline__ u64 mont_mul(u64 a, u64 b, u64 q, u64 qinv_neg)
{
    u64 lo = a * b;
    u64 hi = umulhi64(a, b);
    u64 m = lo * qinv_neg;
    u64 u = hi + umulhi64(m, q) + (lo != 0);
    return csub(u, q);
}

// any 64-bit x -> x mod q
__host__ __device__ __forceinline__ u64 reduce64(u64 x, u64 q, u64 ratio)
{
    u64 qh = umulhi64(x, ratio);
    return csub(x - qh * q, q);
}

// x is a residue mod p (odd); lift it to the centered range (-p/2, p/2) and
// reduce that integer mod q.  p_mod_q = p mod q.
__host__ __device__ __forceinline__ u64 centered_lift(u64 x, u64 p_half, u64 p_mod_q, u64 q, u64 ratio)
{
    u64 r = reduce64(x, q, ratio);
    return x > p_half ? sub_mod(r, p_mod_q, q) : r;
}

// Sum of Montgomery products with one reduction at the end.  The 128-bit
// value T = hi 2^64 + lo stands for T 2^-64 mod q.  wide_init(v) sets T = v
// 2^64 (standing for v); wide_mac adds a full product x y (x, y < 2^61), which
// contributes x y 2^-64 mod q like mont_mul.  T < 2 q 2^64 holds while at most
// floor(2^64 / q) products (each below q^2) are added after an init or fold,
// and wide_redc of such a T is (T + m q) / 2^64 < 3q, brought into [0, q).
struct WideAcc {
    u64 lo, hi;
};

__host__ __device__ __forceinline__ void wide_init(WideAcc& a, u64 v)
{
    a.lo = 0;
    a.hi = v;
}

__host__ __device__ __forceinline__ void wide_mac(WideAcc& a, u64 x, u64 y)
{
#ifdef __HIP_DEVICE_COMPILE__
    const u32 x0 = (u32)x, x1 = (u32)(x >> 32), y0 = (u32)y, y1 = (u32)(y >> 32);
    const u64 p00 = (u64)x0 * y0;
    const u64 mid = (u64)x0 * y1 + (u64)x1 * y0 + (p00 >> 32);   // < 2^62 + 2^32 for x, y < 2^61
    const u64 plo = (mid << 32) | (u32)p00;
    const u64 phi = (u64)x1 * y1 + (mid >> 32);
#else
    const unsigned __int128 p = (unsigned __int128)x * y;
    const u64 plo = (u64)p, phi = (u64)(p >> 64);
#endif
    a.lo += plo;
    a.hi += phi + (a.lo < plo);
}

__host__ __device__ __forceinline__ u64 wide_redc(const WideAcc& a, u64 q, u64 qinv_neg)
{
    const u64 m = a.lo * qinv_neg;
    const u64 u = a.hi + umulhi64(m, q) + (a.lo != 0);
    return csub(csub(u, q), q);
}

__host__ __device__ __forceinline__ void wide_fold(WideAcc& a, u64 q, u64 qinv_neg)
{
    a.hi = wide_redc(a, q, qinv_neg);
    a.lo = 0;
}

// products that may be added between folds: floor(2^64 / q), capped
__host__ __device__ __forceinline__ int wide_period(u64 ratio) { return ratio < 4096 ? (int)ratio : 4096; }

// ---- binary64 modular arithmetic for primes q < 2^41 ----
// Residues are integer-valued doubles.  Every integer below 2^53 is exact in
// binary64, and an FMA forms a * b - c with one rounding, so x w = hi + lo
// holds exactly with hi = fl(x w), lo = fma(x, w, -hi) (|lo| <= ulp(hi) / 2).
// With a quotient estimate qf = round(x w / q) (off by at most one), the
// remainder r = (hi - qf q) + lo is small, so fma(-qf, q, hi) is exact and so
// is the final addition: r is the integer x w - qf q, congruent to x w mod q,
// in (-0.7 q, 0.7 q) for |x| < 2^49.
struct FpModulus {
    double q, qinv;      // q and fl(1 / q)
    double ninv, ninvq;  // N^-1 mod q and fl(N^-1 / q)
    double rinv, rinvq;  // 2^-64 mod q and fl(2^-64 mod q / q) (undoes the Montgomery factor of stored operands)
    double pad0, pad1;
};

// fixed w in [0, q) with wq = fl(w / q)
__device__ __forceinline__ double fp_mulmod(double x, double w, double wq, double q)
{
    const double hi = x * w;
    const double lo = __builtin_fma(x, w, -hi);
    const double qf = __builtin_rint(x * wq);
    return __builtin_fma(-qf, q, hi) + lo;
}

// two variable operands (|x| < 2^49, 0 <= y < q): quotient from fl(x y) / q
__device__ __forceinline__ double fp_mulmod_var(double x, double y, double qinv, double q)
{
    const double hi = x * y;
    const double lo = __builtin_fma(x, y, -hi);
    const double qf = __builtin_rint(hi * qinv);
    return __builtin_fma(-qf, q, hi) + lo;
}

// integer below 2^53 -> binary64 (exact): high and low words converted apart
__device__ __forceinline__ double u2d(u64 x)
{
    return __builtin_fma((double)(u32)(x >> 32), 4294967296.0, (double)(u32)x);
}

// integer-valued double in [0, 2^53) -> integer
__device__ __forceinline__ u64 d2u(double x)
{
    const double h = __builtin_trunc(x * (1.0 / 4294967296.0));
    const double l = __builtin_fma(-h, 4294967296.0, x);
    return ((u64)(u32)h << 32) | (u32)l;
}

// canonical residue in [0, q) of an integer-valued double with |x| < 2^50
__device__ __forceinline__ u64 fp_canon(double x, double q, double qinv)
{
    double r = __builtin_fma(-__builtin_rint(x * qinv), q, x);  // in [-q/2, q/2] up to a rounding of the quotient
    r = r < 0.0 ? r + q : r;
    r = r >= q ? r - q : r;
    return d2u(r);
}
