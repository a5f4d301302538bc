// hsd_math.hpp -- device math for the MI355X direct-sum and NUFFT kernels.
//
// FP64 sine/cosine: Cody-Waite reduction by pi/2 (two-part constant, exact
// FMA products) followed by the Maclaurin series of sin and cos on
// [-pi/4, pi/4], truncated where the first omitted term is below 1e-19
// (x^19/19! and x^20/20! at pi/4).  The coefficients are 1/k!, generated at
// compile time; no tabulated constants beyond pi/2 itself.
//
// FP32 sine/cosine for the mixed form: the argument is reduced by pi/2 in
// FP64 and the series is summed in FP32 (sincos32_acc).  The hardware
// transcendental unit is not used: its absolute error (~1e-7) is a large
// relative error for the small angles of the divided differences.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

#define HSD_HD __host__ __device__ __forceinline__

namespace hsd {

// ---------------------------------------------------------------------------
// compile-time 1/k!
// ---------------------------------------------------------------------------
constexpr double inv_factorial(int k)
{
    double f = 1.0;
    for (int i = 2; i <= k; ++i) f *= (double)i;
    return 1.0 / f;
}

// pi/2 split into the nearest double and the (rounded) remainder; 2/pi.
constexpr double kPio2Hi = 1.5707963267948966;      // RN(pi/2)
constexpr double kPio2Lo = 6.123233995736766e-17;   // RN(pi/2 - kPio2Hi)
constexpr double kTwoOverPi = 0.6366197723675814;   // RN(2/pi)
constexpr double kPi = 3.141592653589793;
constexpr double kFourPi = 12.566370614359172;

// e^{-i theta} stored as (c, s) = (cos theta, sin theta).
struct cs64 { double c, s; };
struct cs32 { float c, s; };

// sin and cos of x (|x| < 2^20 * pi/2), FP64, error ~1 ulp.
HSD_HD cs64 sincos64(double x)
{
    const double q = __builtin_rint(x * kTwoOverPi);
    double r = __builtin_fma(-q, kPio2Hi, x);
    r = __builtin_fma(-q, kPio2Lo, r);
    const int iq = (int)q;
    const double r2 = r * r;
    // sin r = r + r^3 * (-1/3! + r^2 (1/5! + r^2 (-1/7! + ...)))
    double ps = inv_factorial(17);
    ps = __builtin_fma(ps, r2, -inv_factorial(15));
    ps = __builtin_fma(ps, r2, inv_factorial(13));
    ps = __builtin_fma(ps, r2, -inv_factorial(11));
    ps = __builtin_fma(ps, r2, inv_factorial(9));
    ps = __builtin_fma(ps, r2, -inv_factorial(7));
    ps = __builtin_fma(ps, r2, inv_factorial(5));
    ps = __builtin_fma(ps, r2, -inv_factorial(3));
    const double sn = __builtin_fma(ps * r2, r, r);
    // cos r = 1 + r^2 * (-1/2! + r^2 (1/4! + r^2 (-1/6! + ...)))
    double pc = -inv_factorial(18);
    pc = __builtin_fma(pc, r2, inv_factorial(16));
    pc = __builtin_fma(pc, r2, -inv_factorial(14));
    pc = __builtin_fma(pc, r2, inv_factorial(12));
    pc = __builtin_fma(pc, r2, -inv_factorial(10));
    pc = __builtin_fma(pc, r2, inv_factorial(8));
    pc = __builtin_fma(pc, r2, -inv_factorial(6));
    pc = __builtin_fma(pc, r2, inv_factorial(4));
    pc = __builtin_fma(pc, r2, -inv_factorial(2));
    const double cn = __builtin_fma(pc, r2, 1.0);
    // quadrant q mod 4: (sin, cos) of r + q pi/2
    const bool swap = (iq & 1) != 0;
    double s = swap ? cn : sn;
    double c = swap ? sn : cn;
    s = (iq & 2) ? -s : s;
    c = ((iq + 1) & 2) ? -c : c;
    return cs64{c, s};
}

// e^{i k pi/16} for k = 0..31 as (cos, sin): the eighth-quadrant values
// k = 0..7 from sincos64, the others by exact quarter-turn rotations, so that
// multiples of pi/2 give exact 0 and +-1.
HSD_HD cs64 turn16(int k)
{
    const int j = k & 7, quad = (k >> 3) & 3;
    const cs64 b = j == 0 ? cs64{1.0, 0.0} : sincos64((double)j * (kPio2Hi / 8.0));
    switch (quad) {
    case 0: return b;
    case 1: return cs64{-b.s, b.c};
    case 2: return cs64{-b.c, -b.s};
    default: return cs64{b.s, -b.c};
    }
}

// (cos x, sin x) with x reduced by pi/16 instead of pi/2: x = q pi/16 + r,
// |r| <= pi/32, then e^{ix} = T[q mod 32] e^{ir} with T = turn16 (tab holds
// its 32 entries).  The short interval needs sin r through r^9 and cos r
// through r^8 (first omitted terms below 3e-19 and 2.2e-17); one complex
// product replaces the quadrant logic.  For q = 0 the result is the
// polynomial itself, so small angles keep full relative accuracy.
HSD_HD cs64 sincos64_tab(double x, const cs64 *tab)
{
    constexpr double kPi16Hi = kPio2Hi / 8.0, kPi16Lo = kPio2Lo / 8.0;   // exact scalings
    const double q = __builtin_rint(x * (8.0 * kTwoOverPi));
    double r = __builtin_fma(-q, kPi16Hi, x);
    r = __builtin_fma(-q, kPi16Lo, r);
    const double r2 = r * r;
    double ps = inv_factorial(9);
    ps = __builtin_fma(ps, r2, -inv_factorial(7));
    ps = __builtin_fma(ps, r2, inv_factorial(5));
    ps = __builtin_fma(ps, r2, -inv_factorial(3));
    const double sn = __builtin_fma(ps * r2, r, r);
    double pc = inv_factorial(8);
    pc = __builtin_fma(pc, r2, -inv_factorial(6));
    pc = __builtin_fma(pc, r2, inv_factorial(4));
    pc = __builtin_fma(pc, r2, -0.5);
    const double cn = __builtin_fma(pc, r2, 1.0);
    const cs64 t = tab[(int)q & 31];
    return cs64{__builtin_fma(t.c, cn, -t.s * sn), __builtin_fma(t.s, cn, t.c * sn)};
}

// FP32 sin/cos of an angle x given in FP64, accurate to ~1 ulp of FP32 in
// the relative sense also near zero (the hardware unit is not: it carries an
// absolute error near 1e-7, i.e. ~1e-6 relative for small angles, which the
// closed-branch differences of the divided difference would amplify).  The
// angle is reduced by pi/2 in FP64 (Cody-Waite, as sincos64), rounded to
// FP32 in [-pi/4, pi/4], and the Maclaurin series is summed in FP32 through
// x^11 (sin) and x^12 (cos).
//
// Unbiased on average, not only small: the sums over many triangles cancel
// the random rounding errors but keep any systematic one, so the two
// largest correction terms (1/3! for sin, 1/4! for cos, and 1/5!) use a
// two-float coefficient hi + lo whose lo part is added to the varying
// product before the hi part (a lo part added to a rounded value would
// always be absorbed).  Rounding 1/3! to FP32 alone shrinks |sin| by ~3e-8
// x^2 relative; without the split the mean of (computed - exact) projected
// on the exact phase is about -2e-10 over uniformly spread angles, with it
// below 1e-11.
constexpr float f32_hi(double v) { return (float)v; }
constexpr float f32_lo(double v) { return (float)(v - (double)(float)v); }

HSD_HD cs32 sincos32_acc(double x)
{
    const double q = __builtin_rint(x * kTwoOverPi);
    double rd = __builtin_fma(-q, kPio2Hi, x);
    rd = __builtin_fma(-q, kPio2Lo, rd);
    const int iq = (int)q;
    const float r = (float)rd;
    const float r2 = r * r;
    float ps = (float)-inv_factorial(11);
    ps = __builtin_fmaf(ps, r2, (float)inv_factorial(9));
    ps = __builtin_fmaf(ps, r2, (float)-inv_factorial(7));
    ps = __builtin_fmaf(ps, r2, f32_lo(inv_factorial(5))) + f32_hi(inv_factorial(5));
    ps = __builtin_fmaf(ps, r2, f32_lo(-inv_factorial(3))) + f32_hi(-inv_factorial(3));
    const float sn = __builtin_fmaf(ps * r2, r, r);
    float pc = (float)inv_factorial(12);
    pc = __builtin_fmaf(pc, r2, (float)-inv_factorial(10));
    pc = __builtin_fmaf(pc, r2, (float)inv_factorial(8));
    pc = __builtin_fmaf(pc, r2, (float)-inv_factorial(6));
    pc = __builtin_fmaf(pc, r2, f32_lo(inv_factorial(4))) + f32_hi(inv_factorial(4));
    pc = __builtin_fmaf(pc, r2, -0.5f);
    const float cn = __builtin_fmaf(pc, r2, 1.0f);
    const bool swap = (iq & 1) != 0;
    float s = swap ? cn : sn;
    float c = swap ? sn : cn;
    s = (iq & 2) ? -s : s;
    c = ((iq + 1) & 2) ? -c : c;
    return cs32{c, s};
}

// 1/x for finite nonzero x: hardware estimate + two Newton steps (~1 ulp)
// on the device; a correctly rounded division in the host pass.
HSD_HD double rcp64(double x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    double y = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, y, 1.0);
    y = __builtin_fma(y, e, y);
    e = __builtin_fma(-x, y, 1.0);
    y = __builtin_fma(y, e, y);
    return y;
#else
    return 1.0 / x;
#endif
}

// Square root of x >= 0 (0 for x = 0) from the hardware reciprocal square
// root and two Newton-Raphson corrections of the root (Goldschmidt form),
// without the library's scaling for denormal and special inputs: used where
// x is a positive normal number or zero.
HSD_HD double sqrt_pos64(double x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, hh = 0.5 * y;
    const double e = __builtin_fma(-hh, g, 0.5);
    g = __builtin_fma(g, e, g);
    hh = __builtin_fma(hh, e, hh);
    double d = __builtin_fma(-g, g, x);
    g = __builtin_fma(d, hh, g);
    d = __builtin_fma(-g, g, x);
    g = __builtin_fma(d, hh, g);
    return x > 0.0 ? g : 0.0;
#else
    return __builtin_sqrt(x);
#endif
}

HSD_HD float rcp32(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    float y = __builtin_amdgcn_rcpf(x);
    float e = __builtin_fmaf(-x, y, 1.0f);
    return __builtin_fmaf(y, e, y);
#else
    return 1.0f / x;
#endif
}

// product of two unit phases e^{-i a} e^{-i b}
HSD_HD cs64 pmul(cs64 a, cs64 b)
{
    return cs64{__builtin_fma(a.c, b.c, -a.s * b.s), __builtin_fma(a.s, b.c, a.c * b.s)};
}
// e^{-i a} e^{+i b}
HSD_HD cs64 pmulc(cs64 a, cs64 b)
{
    return cs64{__builtin_fma(a.c, b.c, a.s * b.s), __builtin_fma(a.s, b.c, -a.c * b.s)};
}
HSD_HD cs32 pmul(cs32 a, cs32 b)
{
    return cs32{__builtin_fmaf(a.c, b.c, -a.s * b.s), __builtin_fmaf(a.s, b.c, a.c * b.s)};
}
HSD_HD cs32 pmulc(cs32 a, cs32 b)
{
    return cs32{__builtin_fmaf(a.c, b.c, a.s * b.s), __builtin_fmaf(a.s, b.c, -a.c * b.s)};
}

// Sorting network for three values: lo <= mid <= hi.
template <typename T>
HSD_HD void sort3(T x0, T x1, T x2, T &lo, T &mid, T &hi)
{
    T m1 = fmin(x0, x1), M1 = fmax(x0, x1);
    T m2 = fmin(M1, x2);
    hi = fmax(M1, x2);
    lo = fmin(m1, m2);
    mid = fmax(m1, m2);
}

// Power series of the second divided difference of exp at (i a, 0, -i b)
// (a, b >= 0): sum_n (-i)^n H_n / (n+2)!, H_n = sum_{m<=n} (-a)^m b^(n-m),
// summed through n = N; the first omitted term is below
// (N+2) G^(N+1) / (N+3)! with G = a + b (N = 9: 2e-21 at G = 0.05;
// N = 11: 5e-12 at G = 0.75).
template <int N = 9, typename T>
HSD_HD void dd2_series_dev(T a, T b, T &re, T &im);

template <typename T>
HSD_HD void dd2_series(T a, T b, T &re, T &im)
{
    dd2_series_dev(a, b, re, im);
    re += (T)0.5;
}

// The same series without its constant term 1/2 (re is Re - 1/2).  The
// mixed form adds the 1/2 term last, fused
// with the already summed rest: at the smallest radii the rest is below one
// FP32 ulp of 1/2, and adding it to a rounded 1/2-term would err the same way
// for every triangle of a node.
template <int N, typename T>
HSD_HD void dd2_series_dev(T a, T b, T &re, T &im)
{
    const T na = -a;
    T pw = (T)1.0, H = (T)1.0;
    T sre = (T)0.0, sim = (T)0.0;       // n = 0 term (1/2) left out
#pragma unroll
    for (int n = 1; n <= N; ++n) {
        pw *= na;
        H = H * b + pw;                 // H_n
        const T t = H * (T)inv_factorial(n + 2);
        switch (n & 3) {                // times (-i)^n
        case 1: sim -= t; break;
        case 2: sre -= t; break;
        case 3: sim += t; break;
        default: sre += t; break;
        }
    }
    re = sre;
    im = sim;
}

} // namespace hsd
