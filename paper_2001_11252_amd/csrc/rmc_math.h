// rmc_math.h -- double elementary functions of the double transport path,
// written for the arguments it produces and for a small register footprint:
// the general library forms carry reductions for arguments of any size
// (Payne-Hanek for the tangent) and special-case branches whose temporaries
// set the register peak of the double transport kernel.
//
//   tan_halfpi    tan(th), |th| <= pi/2       (the atom-velocity draw)
//   atan_any      atan(z), any z              (its envelope)
//   sincos_turns  sin and cos of 2 pi r       (azimuths, Box-Muller)
//   log_pos       log(x), x > 0 finite        (optical depths, Box-Muller)
//   exp_any       exp(x)                      (H(a,x), the draw's envelope)
//
// All are host and device functions with every multiply-add written as an
// fma and contraction off, so a host build gives the device's values bit
// for bit (the CPU tests measure their error against 40-digit references:
// under 2 ulp).
//
// Polynomials: Chebyshev interpolants of the series remainders on the
// reduced intervals, fitted at 60 digits and rounded to double; each fit
// reaches the rounding floor of its double coefficients (below 0.1 ulp of
// the result).
#pragma once
#include <hip/hip_runtime.h>

namespace rmc {

#pragma clang fp contract(off)

// sin and cos of r + rl for |r| <= pi/4 (rl a tail far below r's ulp), by
// the series remainders in r; rl enters the small terms to first order.
// cos is (1 - z/2) + z^2 C(z) - rl r with 1 - z/2 taken as a rounded head
// w and the exact tails of w and of z = r^2 carried into the small term;
// sin is r + (r z S(z) + rl w).
__host__ __device__ inline void sincos_reduced(double r, double rl, double *s, double *c) {
  const double z = r * r;
  double cp = -1.1382632425521717e-11;
  cp = fma(cp, z, 2.08761462684032e-09);
  cp = fma(cp, z, -2.7557317271729793e-07);
  cp = fma(cp, z, 2.480158729876569e-05);
  cp = fma(cp, z, -0.0013888888888887398);
  cp = fma(cp, z, 0.041666666666666664);
  const double hz = 0.5 * z;
  const double w = 1.0 - hz;
  const double tail = ((1.0 - w) - hz) - 0.5 * fma(r, r, -z) - rl * r;
  *c = w + fma(z * z, cp, tail);
  double sp = -7.586697117706918e-13;
  sp = fma(sp, z, 1.6058531618986147e-10);
  sp = fma(sp, z, -2.5052106232447578e-08);
  sp = fma(sp, z, 2.7557319219339167e-06);
  sp = fma(sp, z, -0.00019841269841265065);
  sp = fma(sp, z, 0.008333333333333331);
  sp = fma(sp, z, -0.16666666666666666);
  *s = r + fma(r * z, sp, rl * w);
}

// tan(th) for |th| <= pi/2 (rounded to double): with n = rint(2 th / pi)
// in {-1, 0, 1}, th - n pi/2 = r + rl where r = th - n PIO2_HI is exact
// (Sterbenz) and rl = -n PIO2_LO; then tan = s / c (n = 0) or -c / s
// (n odd).
__host__ __device__ inline double tan_halfpi(double th) {
  const double PIO2_HI = 1.5707963267948966, PIO2_LO = 6.123233995736766e-17;
  const double n = rint(th * 0.6366197723675814);
  double sn, cs;
  sincos_reduced(fma(-n, PIO2_HI, th), -n * PIO2_LO, &sn, &cs);
  return n == 0.0 ? sn / cs : -cs / sn;
}

// sin(2 pi r) and cos(2 pi r) for |r| <= 1: q = rint(4 r), t = r - q/4
// (exact: Sterbenz for q != 0), 2 pi t as a product with its exact fma
// tail and the tail of 2 pi, then the quadrant q mod 4.
__host__ __device__ inline void sincos_turns(double r, double *s, double *c) {
  const double TWOPI_HI = 6.283185307179586, TWOPI_LO = 2.4492935982947064e-16;
  const double q = rint(4.0 * r);
  const double t = fma(-0.25, q, r);
  const double th = t * TWOPI_HI;
  const double tl = fma(t, TWOPI_HI, -th) + t * TWOPI_LO;
  double sn, cs;
  sincos_reduced(th, tl, &sn, &cs);
  const int k = (int)q & 3;
  *s = k == 0 ? sn : (k == 1 ? cs : (k == 2 ? -sn : -cs));
  *c = k == 0 ? cs : (k == 1 ? -sn : (k == 2 ? -cs : sn));
}

// log(x) for finite x > 0: x = 2^e m with m in [sqrt(1/2), sqrt(2)),
// log m = 2 atanh(s), s = (m - 1)/(m + 1) (m - 1 exact), as 2s + 2s z A(z),
// z = s^2; then e log 2 with log 2 in two parts.
__host__ __device__ inline double log_pos(double x) {
  const double LN2_HI = 0.6931471805599453, LN2_LO = 2.3190468138462996e-17;
  int e;
  double m = frexp(x, &e);           // m in [1/2, 1)
  if (m < 0.7071067811865476) {
    m *= 2.0;
    --e;
  }
  const double f = m - 1.0;
  const double s = f / (2.0 + f);
  const double z = s * s;
  double a = 0.07308224842521703;
  a = fma(a, z, 0.07665860800278021);
  a = fma(a, z, 0.09091444562630861);
  a = fma(a, z, 0.1111110556739754);
  a = fma(a, z, 0.14285714312987743);
  a = fma(a, z, 0.19999999999949752);
  a = fma(a, z, 0.3333333333333335);
  const double s2 = 2.0 * s;
  const double de = (double)e;
  return fma(de, LN2_HI, s2 + fma(s2 * z, a, de * LN2_LO));
}

// exp(x): x = k log 2 + r with k = rint(x / log 2), |r| <= log(2)/2; log 2
// in two parts, the first with 32 significant bits so that x - k LN2_HI is
// exact (|k| <= 1076); exp r = 1 + (r + r^2 E(r)); then the scaling by 2^k
// (exact above the subnormal range).  0 below -746, inf above 710.
__host__ __device__ inline double exp_any(double x) {
  const double LN2_HI = 0.6931471803691238, LN2_LO = 1.9082149292705877e-10;
  if (!(x > -746.0)) return x != x ? x : 0.0;
  if (x > 710.0) return __builtin_inf();
  const double k = rint(x * 1.4426950408889634);
  const double r = fma(-k, LN2_LO, fma(-k, LN2_HI, x));
  double e = 1.6086622436215554e-10;
  e = fma(e, r, 2.0918129454967065e-09);
  e = fma(e, r, 2.5052071109214447e-08);
  e = fma(e, r, 2.755726330147475e-07);
  e = fma(e, r, 2.755731924720479e-06);
  e = fma(e, r, 2.480158733642132e-05);
  e = fma(e, r, 0.00019841269841263304);
  e = fma(e, r, 0.0013888888888879082);
  e = fma(e, r, 0.008333333333333333);
  e = fma(e, r, 0.04166666666666668);
  e = fma(e, r, 0.16666666666666666);
  e = fma(e, r, 0.5);
  return ldexp(1.0 + fma(r * r, e, r), (int)k);
}

// atan(z) for any double z: |z| > 1 through pi/2 - atan(1/|z|), then
// arguments above tan(pi/12) through pi/6 + atan((t sqrt3 - 1)/(t + sqrt3)),
// so the series remainder runs on |t| <= tan(pi/12).
__host__ __device__ inline double atan_any(double z) {
  const double PIO2_HI = 1.5707963267948966, PIO2_LO = 6.123233995736766e-17;
  const double PIO6_HI = 0.5235987755982989, PIO6_LO = -5.360408832255455e-17;
  const double SQ3_HI = 1.7320508075688772, SQ3_LO = 1.0035084221806903e-16;
  double t = fabs(z);
  const bool inv = t > 1.0;
  if (inv) t = 1.0 / t;
  const bool big = t > 0.2679491924311227;
  if (big) t = fma(t, SQ3_LO, fma(t, SQ3_HI, -1.0)) / (t + SQ3_HI);
  const double s = t * t;
  // atan t = t + t s P(s)
  double p = -0.03957893591546196;
  p = fma(p, s, 0.05716329894442852);
  p = fma(p, s, -0.06654945053677658);
  p = fma(p, s, 0.07691819638198708);
  p = fma(p, s, -0.09090897081592211);
  p = fma(p, s, 0.11111110944516939);
  p = fma(p, s, -0.14285714284553813);
  p = fma(p, s, 0.1999999999999688);
  p = fma(p, s, -0.3333333333333333);
  double r = fma(t * s, p, t);
  if (big) r = PIO6_HI + (r + PIO6_LO);
  if (inv) r = PIO2_HI - (r - PIO2_LO);
  return copysign(r, z);
}

#pragma clang fp contract(fast)

}  // namespace rmc
