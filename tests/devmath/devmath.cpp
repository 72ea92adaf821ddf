// Host build of the double elementary functions of rmc_math.h, for
// the CPU tests that measure their error: the functions are host and device
// functions with explicit fmas and contraction off, so these are the values
// the double kernels compute.
#include "rmc_math.h"

extern "C" void devmath_tan_halfpi(const double *x, double *y, long n) {
  for (long i = 0; i < n; ++i) y[i] = rmc::tan_halfpi(x[i]);
}

extern "C" void devmath_atan_any(const double *x, double *y, long n) {
  for (long i = 0; i < n; ++i) y[i] = rmc::atan_any(x[i]);
}

extern "C" void devmath_sincos_turns(const double *x, double *s, double *c, long n) {
  for (long i = 0; i < n; ++i) rmc::sincos_turns(x[i], s + i, c + i);
}

extern "C" void devmath_log_pos(const double *x, double *y, long n) {
  for (long i = 0; i < n; ++i) y[i] = rmc::log_pos(x[i]);
}

extern "C" void devmath_exp_any(const double *x, double *y, long n) {
  for (long i = 0; i < n; ++i) y[i] = rmc::exp_any(x[i]);
}
