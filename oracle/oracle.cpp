/*
 * oracle.cpp -- plain FP64 CPU oracle for Monte Carlo resonant-line transfer
 * (Michel-Dansac et al. 2020, "RASCAS", A&A 635 A154).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the GPU library.
 *
 * Each function names the passage of the paper it follows.  Where the paper
 * is silent or garbled the reading taken is stated at the point of use.
 * Build: g++ -O2 -std=c++17 -ffp-contract=off (no fast-math): the traversal
 * geometry relies on uncontracted IEEE arithmetic with explicit fma().
 */
#include "rmc_oracle.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <thread>
#include <unordered_map>
#include <vector>

namespace {

/* ---------------------------------------------------------------- constants
 * CGS values (CODATA 2018; the paper prints none of them). */
const double C_LIGHT = 2.99792458e10;     /* cm/s  */
const double H_PLANCK = 6.62607015e-27;   /* erg s */
const double K_BOLTZ = 1.380649e-16;      /* erg/K */
const double E_CHARGE = 4.80320471e-10;   /* esu   */
const double M_ELECTRON = 9.1093837015e-28; /* g   */
const double AMU_G = 1.66053906660e-24;   /* g     */
const double PI = 3.14159265358979323846;

/* ------------------------------------------------------------------ Philox
 * Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds of two
 * 32x32->64 multiplications with the published multipliers, the key bumped
 * by the published Weyl increments between rounds. */
void philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Uniform number j of one event.  Counter = (pid_lo, pid_hi, event, j/2),
 * key = (seed_lo, seed_hi); draw j takes the word pair 2(j%2), 2(j%2)+1,
 * keeps 52 bits and returns (2m+1) 2^-53, exactly representable and never
 * 0 or 1 (so -ln r is always finite). */
double uniform(uint64_t seed, uint64_t pid, uint32_t event, uint32_t j) {
  uint32_t ctr[4] = {(uint32_t)pid, (uint32_t)(pid >> 32), event, j >> 1};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t w[4];
  philox(ctr, key, w);
  uint32_t hi = w[2 * (j & 1)], lo = w[2 * (j & 1) + 1];
  uint64_t m = ((uint64_t)hi << 20) | (uint64_t)(lo >> 12);
  return (double)(2 * m + 1) * 0x1p-53;
}

/* Fixed slots of the uniforms used by one event.  Slots 6.. are shared by
 * branches that never occur in the same event (dust albedo, the |x| >= 8
 * Gaussian, the rejection rounds). */
enum {
  J_CHANNEL = 0,  /* dust or which line                        */
  J_MU = 1,       /* cosine of the scattering angle            */
  J_PHI = 2,      /* azimuth of the new direction              */
  J_TAU = 3,      /* optical depth to the next event           */
  J_PERP1 = 4,    /* Box-Muller pair for the two u_perp        */
  J_PERP2 = 5,
  J_ALBEDO = 6,   /* dust: scatter or absorb                   */
  J_GAUSS1 = 6,   /* line, |x| >= 8: Box-Muller pair           */
  J_GAUSS2 = 7,
  J_REJ = 6,      /* line, |x| < 8: round i uses 6+3i .. 8+3i  */
  J_SRC1 = 4,     /* emission (event 0): source-spectrum draws */
  J_SRC2 = 5,
  J_DECAY = 1 << 30 /* line: resonant or fluorescent decay; above
                       any rejection round (they stop at 2^20)    */
};

struct Rng {
  uint64_t seed, pid;
  uint32_t event;
  double u(uint32_t j) const { return uniform(seed, pid, event, j); }
};

/* ------------------------------------------------------ line quantities
 * Sect. 3.1.1: v_th = (2 k_B T / m_X)^1/2, Doppler width
 * dnu_D = nu_lu v_th / c, damping a = A_ul / (4 pi dnu_D), and the
 * line-centre cross-section sqrt(pi) e^2 f_lu / (m_e c dnu_D) (Eq. for
 * sigma with H = 1). */
struct LineQ {
  double nu0, vth, dnu, a, sigma0;
};

LineQ line_q(const orc_line &ln, double T) {
  LineQ q;
  q.nu0 = C_LIGHT / (ln.lambda0_A * 1e-8);
  q.vth = std::sqrt(2.0 * K_BOLTZ * T / (ln.mass_amu * AMU_G));
  q.dnu = q.nu0 * q.vth / C_LIGHT;
  q.a = ln.A_ul / (4.0 * PI * q.dnu);
  q.sigma0 = std::sqrt(PI) * E_CHARGE * E_CHARGE * ln.f_lu / (M_ELECTRON * C_LIGHT * q.dnu);
  return q;
}

/* ---------------------------------------------------------------- Voigt H
 * Sect. 3.3.2 names the Tasitsiomi (2006, Eqs. 7-8) approximation as the
 * simplest of the three RASCAS evaluators.  Its form:
 *   z = (x^2 - 0.855) / (x^2 + 3.42)
 *   q = 0 for z <= 0, else z (1 + 21/x^2) (a/pi) / (x^2 + 1) P(z),
 *       P(z) = 5.674 z^3 - 9.207 z^2 + 4.421 z + 0.1117
 *   H = sqrt(pi) q + exp(-x^2). */
double voigt_h(double a, double x) {
  double x2 = x * x;
  double z = (x2 - 0.855) / (x2 + 3.42);
  double q = 0.0;
  if (z > 0.0) {
    double P = 5.674 * z * z * z - 9.207 * z * z + 4.421 * z + 0.1117;
    q = z * (1.0 + 21.0 / x2) * (a / PI) / (x2 + 1.0) * P;
  }
  return std::sqrt(PI) * q + std::exp(-x2);
}

/* H from its definition (Sect. 3.1.1): H(a,x) = (a/pi) int e^{-y^2} /
 * ((y-x)^2 + a^2) dy, by adaptive Gauss-Legendre quadrature.  Within
 * |y - x| <= 1 the Lorentzian factor is removed by y = x + a tan(theta),
 * which turns that part into (1/pi) int e^{-(x + a tan theta)^2} dtheta;
 * outside it the integrand is smooth and is integrated in y over
 * |y| <= 10 (e^{-100} beyond), split at y = 0 where the Gaussian peaks.
 * Each panel is accepted when its 10- and 20-point Gauss-Legendre sums
 * agree to 1e-14 relative, else halved.  The nodes and weights come from
 * Newton's method on the Legendre polynomials. */
struct GaussLegendre {
  std::vector<double> t, w;
  explicit GaussLegendre(int n) : t(n), w(n) {
    /* P_n(r) and P_n'(r) by the three-term recurrence */
    auto legendre = [n](double r, double *dp) {
      double p0 = 1.0, p1 = r;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * r * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      *dp = n * (r * p1 - p0) / (r * r - 1.0);
      return p1;
    };
    for (int i = 0; i < n; ++i) {
      double r = std::cos(PI * (i + 0.75) / (n + 0.5)), dp = 0.0;
      for (int it = 0; it < 100; ++it) {
        double dr = legendre(r, &dp) / dp;
        r -= dr;
        if (std::fabs(dr) < 1e-16) break;
      }
      legendre(r, &dp);
      t[i] = r;
      w[i] = 2.0 / ((1.0 - r * r) * dp * dp);
    }
  }
  template <class F> double panel(const F &f, double lo, double hi) const {
    double m = 0.5 * (lo + hi), hw = 0.5 * (hi - lo), s = 0.0;
    for (size_t i = 0; i < t.size(); ++i) s += w[i] * f(m + hw * t[i]);
    return s * hw;
  }
};

template <class F> double adaptive(const F &f, double lo, double hi, double atol, int depth) {
  static const GaussLegendre g10(10), g20(20);
  double a = g10.panel(f, lo, hi), b = g20.panel(f, lo, hi);
  if (std::fabs(b - a) <= std::max(1e-14 * std::fabs(b), atol) || depth >= 60 || !(hi > lo)) return b;
  double m = 0.5 * (lo + hi);
  return adaptive(f, lo, m, atol, depth + 1) + adaptive(f, m, hi, atol, depth + 1);
}

/* integral over [lo, hi] split at the points of `cuts` inside it */
template <class F> double adaptive_cut(const F &f, double lo, double hi, double atol, std::vector<double> cuts) {
  if (!(hi > lo)) return 0.0;
  std::vector<double> e{lo};
  std::sort(cuts.begin(), cuts.end());
  for (double c : cuts)
    if (c > lo && c < hi) e.push_back(c);
  e.push_back(hi);
  double s = 0.0;
  for (size_t i = 0; i + 1 < e.size(); ++i) s += adaptive(f, e[i], e[i + 1], atol, 0);
  return s;
}

double voigt_h_exact(double a, double x) {
  const double W = 1.0, Y = 10.0;
  /* a panel whose two sums agree to 1e-18 of H (scale from the Tasitsiomi
   * form, within a few percent) is also accepted */
  const double atol = 1e-18 * voigt_h(a, x);
  /* inner part, theta in [-atan(W/a), atan(W/a)]; y = 0 at theta = atan(-x/a) */
  auto fin = [&](double th) { double y = x + a * std::tan(th); return std::exp(-y * y) / PI; };
  double tw = std::atan(W / a);
  double h = adaptive_cut(fin, -tw, tw, atol, {std::atan(-x / a), 0.0});
  /* outer parts in y */
  auto fout = [&](double y) { double d = y - x; return (a / PI) * std::exp(-y * y) / (d * d + a * a); };
  h += adaptive_cut(fout, -Y, std::min(x - W, Y), atol, {0.0});
  h += adaptive_cut(fout, std::max(x + W, -Y), Y, atol, {0.0});
  return h;
}

/* dH/dx of the same form, by the product and chain rules. */
double voigt_dhdx(double a, double x) {
  double x2 = x * x;
  double z = (x2 - 0.855) / (x2 + 3.42);
  double d = -2.0 * x * std::exp(-x2);
  if (z > 0.0) {
    double dz = 2.0 * x * (0.855 + 3.42) / ((x2 + 3.42) * (x2 + 3.42));
    double P = 5.674 * z * z * z - 9.207 * z * z + 4.421 * z + 0.1117;
    double dP = 3.0 * 5.674 * z * z - 2.0 * 9.207 * z + 4.421;
    double f1 = z, df1 = dz;
    double f2 = 1.0 + 21.0 / x2, df2 = -42.0 / (x2 * x);
    double f3 = (a / PI) / (x2 + 1.0), df3 = -(a / PI) * 2.0 * x / ((x2 + 1.0) * (x2 + 1.0));
    double f4 = P, df4 = dP * dz;
    double dq = df1 * f2 * f3 * f4 + f1 * df2 * f3 * f4 + f1 * f2 * df3 * f4 + f1 * f2 * f3 * df4;
    d += std::sqrt(PI) * dq;
  }
  return d;
}

/* ------------------------------------------------------------- samplers
 * Parallel atom velocity, Sect. 3.3.3: rejection sampling of
 * f(u) ~ exp(-u^2) / (a^2 + (x-u)^2) (Sect. 3.2.1) with the two-piece
 * Lorentzian comparison function split at u0, where u0(x, log10 a) is the
 * paper's fitted 2D polynomial.  Readings: the fit goes negative for small
 * x at small a, and the comparison function only bounds f for u0 >= 0, so
 * u0 is clamped at 0; for |x| >= 8 the draw is a Gaussian of variance 1/2
 * centred at 1/x; negative x is handled by the symmetry f(-u | -x) = f(u | x). */
double u0_fit(double x, double a) {
  double z = std::log10(a);
  double c0 = 2.648963 + 2.014446 * z + 0.351479 * z * z;
  double c1 = -4.058673 - 3.675859 * z - 0.640003 * z * z;
  double c2 = 3.017395 + 2.117133 * z + 0.370294 * z * z;
  double c3 = -0.869789 - 0.565886 * z - 0.096312 * z * z;
  double c4 = 0.110987 + 0.070103 * z + 0.011557 * z * z;
  double c5 = -0.005200 - 0.003240 * z - 0.000519 * z * z;
  return c0 + x * (c1 + x * (c2 + x * (c3 + x * (c4 + x * c5))));
}

/* returns false only if the rejection loop exceeds 2^20 rounds (the packet
 * then stops with status stuck) */
bool sample_upar(double x, double a, const Rng &rng, double *u_out) {
  if (std::fabs(x) >= 8.0) {
    double g = std::sqrt(-std::log(rng.u(J_GAUSS1))) * std::cos(2.0 * PI * rng.u(J_GAUSS2));
    *u_out = 1.0 / x + g;
    return true;
  }
  double s = (x < 0.0) ? -1.0 : 1.0;
  double xa = std::fabs(x);
  double u0 = u0_fit(xa, a);
  if (u0 < 0.0) u0 = 0.0;
  double th0 = std::atan((u0 - xa) / a);
  double e0 = std::exp(-u0 * u0);
  double p1 = (th0 + PI / 2.0) / ((1.0 - e0) * th0 + (1.0 + e0) * PI / 2.0);
  for (uint32_t it = 0; it < (1u << 20); ++it) {
    double r1 = rng.u(J_REJ + 3 * it);
    double r2 = rng.u(J_REJ + 3 * it + 1);
    double r3 = rng.u(J_REJ + 3 * it + 2);
    double th, u;
    if (r1 < p1) {
      th = -PI / 2.0 + r2 * (th0 + PI / 2.0);
      u = xa + a * std::tan(th);
      if (r3 < std::exp(-u * u)) { *u_out = s * u; return true; }
    } else {
      th = th0 + r2 * (PI / 2.0 - th0);
      u = xa + a * std::tan(th);
      if (r3 < std::exp(u0 * u0 - u * u)) { *u_out = s * u; return true; }
    }
  }
  *u_out = 0.0;
  return false;
}

/* Sect. 3.3.1: inverse CDFs.  Core and wing phase functions (Eqs. P_core,
 * P_wing) invert to mu = (A+B)^1/3 - (A-B)^1/3; Henyey-Greenstein
 * (Eq. P_HG) inverts to mu = [1 + g^2 - ((1-g^2)/(1-g+2gr))^2] / (2g).
 * Reading: the printed HG inverse lacks the square; the squared form is
 * the exact inverse of the HG CDF. */
double mu_core(double r) {
  double B = 6.0 * (2.0 * r - 1.0);
  double A = std::sqrt(B * B + 11.0 * 11.0 * 11.0 / 27.0);
  return std::cbrt(A + B) - std::cbrt(A - B);
}
double mu_wing(double r) {
  double B = 4.0 * r - 2.0;
  double A = std::sqrt(B * B + 1.0);
  return std::cbrt(A + B) - std::cbrt(A - B);
}
double mu_hg(double r, double g) {
  if (g == 0.0) return 2.0 * r - 1.0;
  double t = (1.0 - g * g) / (1.0 - g + 2.0 * g * r);
  return (1.0 + g * g - t * t) / (2.0 * g);
}
double p_core(double mu) { return 11.0 / 24.0 + 3.0 * mu * mu / 24.0; }
double p_wing(double mu) { return 3.0 * (1.0 + mu * mu) / 8.0; }
double p_hg(double mu, double g) {
  double d = 1.0 + g * g - 2.0 * g * mu;
  return 0.5 * (1.0 - g * g) / (d * std::sqrt(d));
}

/* Orthonormal pair perpendicular to k: e1 = normalize(k x z^), or
 * normalize(k x x^) when |k_z| > 0.9; e2 = k x e1. */
void perp_basis(const double k[3], double e1[3], double e2[3]) {
  double c[3];
  if (std::fabs(k[2]) > 0.9) {
    c[0] = 0.0; c[1] = k[2]; c[2] = -k[1];
  } else {
    c[0] = k[1]; c[1] = -k[0]; c[2] = 0.0;
  }
  double n = std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
  e1[0] = c[0] / n; e1[1] = c[1] / n; e1[2] = c[2] / n;
  e2[0] = k[1] * e1[2] - k[2] * e1[1];
  e2[1] = k[2] * e1[0] - k[0] * e1[2];
  e2[2] = k[0] * e1[1] - k[1] * e1[0];
}

double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* ------------------------------------------------------------------- mesh
 * Sect. 4.3: leaves of a graded octree.  The oracle keeps them in a hash
 * map keyed by (level, i, j, k) and finds the leaf holding a point by
 * probing every level from the root down. */
const int MAX_LEVEL = 18;
/* A packet or ray that has crossed this many leaves is stopped (a packet
 * gets status stuck): it bounds the walk of a ray running parallel to a
 * periodic slab. */
const int64_t MAX_CROSS = (int64_t)1 << 24;

uint64_t mkey(int lev, int64_t i, int64_t j, int64_t k) {
  return ((uint64_t)lev << 57) | ((uint64_t)i << 38) | ((uint64_t)j << 19) | (uint64_t)k;
}

struct Mesh {
  int L = 0;
  std::unordered_map<uint64_t, int64_t> map;
  std::vector<int> lev;
  std::vector<int64_t> ox, oy, oz; /* leaf origin in finest-level units */
};

int build_mesh(int64_t n, const int8_t *level, const int32_t *ijk, Mesh &m) {
  m.L = 0;
  for (int64_t c = 0; c < n; ++c) {
    if (level[c] < 0 || level[c] > MAX_LEVEL) return -1;
    m.L = std::max(m.L, (int)level[c]);
  }
  m.map.reserve((size_t)n * 2);
  m.lev.resize(n); m.ox.resize(n); m.oy.resize(n); m.oz.resize(n);
  for (int64_t c = 0; c < n; ++c) {
    int l = level[c];
    int64_t side = (int64_t)1 << l;
    int64_t i = ijk[3 * c], j = ijk[3 * c + 1], k = ijk[3 * c + 2];
    if (i < 0 || j < 0 || k < 0 || i >= side || j >= side || k >= side) return -1;
    if (!m.map.emplace(mkey(l, i, j, k), c).second) return -2;
    m.lev[c] = l;
    int sh = m.L - l;
    m.ox[c] = i << sh; m.oy[c] = j << sh; m.oz[c] = k << sh;
  }
  return 0;
}

int64_t find_leaf_int(const Mesh &m, int64_t X, int64_t Y, int64_t Z) {
  int64_t side = (int64_t)1 << m.L;
  if (X < 0 || Y < 0 || Z < 0 || X >= side || Y >= side || Z >= side) return -1;
  for (int l = 0; l <= m.L; ++l) {
    int sh = m.L - l;
    auto it = m.map.find(mkey(l, X >> sh, Y >> sh, Z >> sh));
    if (it != m.map.end()) return it->second;
  }
  return -1;
}

/* Point location with direction-biased ties: along an axis with k_d >= 0
 * the integer coordinate is floor(p_d 2^L), otherwise ceil(p_d 2^L) - 1,
 * so a point on a face belongs to the cell the packet is entering. */
int64_t locate(const Mesh &m, const double p[3], const double k[3]) {
  int64_t X[3];
  for (int d = 0; d < 3; ++d) {
    double s = std::ldexp(p[d], m.L);
    X[d] = (k[d] >= 0.0) ? (int64_t)std::floor(s) : (int64_t)std::ceil(s) - 1;
  }
  return find_leaf_int(m, X[0], X[1], X[2]);
}

/* Distance from p along k to the face the packet leaves leaf c through,
 * and the point on that face.  Exiting axes are snapped onto the face, the
 * others advanced with one fma and clamped into the leaf. */
double exit_step(const Mesh &m, int64_t c, const double p[3], const double k[3], double pn[3]) {
  int64_t o[3] = {m.ox[c], m.oy[c], m.oz[c]};
  int64_t s = (int64_t)1 << (m.L - m.lev[c]);
  double face[3], td[3], lo[3], hi[3];
  double t = INFINITY;
  for (int d = 0; d < 3; ++d) {
    lo[d] = std::ldexp((double)o[d], -m.L);
    hi[d] = std::ldexp((double)(o[d] + s), -m.L);
    if (k[d] > 0.0) { face[d] = hi[d]; td[d] = (face[d] - p[d]) / k[d]; }
    else if (k[d] < 0.0) { face[d] = lo[d]; td[d] = (face[d] - p[d]) / k[d]; }
    else { face[d] = 0.0; td[d] = INFINITY; }
    if (td[d] < t) t = td[d];
  }
  if (t < 0.0) t = 0.0;
  for (int d = 0; d < 3; ++d) {
    if (td[d] <= t) {
      pn[d] = face[d];
    } else {
      double q = std::fma(t, k[d], p[d]);
      pn[d] = std::min(std::max(q, lo[d]), hi[d]);
    }
  }
  return t;
}

/* Domain classes of Sect. 4: distance from p along k to the domain
 * border.  Box: the unit cube.  Slab: |z - zc| < half_z, periodic in x and
 * y.  Sphere: centre c, radius R, by the cancellation-free root of
 * t^2 + 2bt + q = 0. */
double domain_dist(const orc_problem &pb, const double p[3], const double k[3]) {
  double t = INFINITY;
  if (pb.domain_kind == ORC_DOM_BOX) {
    for (int d = 0; d < 3; ++d) {
      double td = INFINITY;
      if (k[d] > 0.0) td = (1.0 - p[d]) / k[d];
      else if (k[d] < 0.0) td = (0.0 - p[d]) / k[d];
      if (td < t) t = td;
    }
  } else if (pb.domain_kind == ORC_DOM_SLAB_Z) {
    double zc = pb.domain[0], hz = pb.domain[1];
    if (k[2] > 0.0) t = ((zc + hz) - p[2]) / k[2];
    else if (k[2] < 0.0) t = ((zc - hz) - p[2]) / k[2];
  } else {
    double dx = p[0] - pb.domain[0], dy = p[1] - pb.domain[1], dz = p[2] - pb.domain[2];
    double R = pb.domain[3];
    double b = dx * k[0] + dy * k[1] + dz * k[2];
    double q = dx * dx + dy * dy + dz * dz - R * R;
    double disc = b * b - q;
    if (disc < 0.0) return 0.0;
    double sq = std::sqrt(disc);
    t = (b > 0.0) ? -q / (b + sq) : -b + sq;
  }
  if (t < 0.0) t = 0.0;
  return t;
}

/* Periodic wrap of the slab's x and y after a face step. */
void wrap_slab(const orc_problem &pb, double p[3], const double k[3]) {
  if (pb.domain_kind != ORC_DOM_SLAB_Z) return;
  for (int d = 0; d < 2; ++d) {
    if (k[d] > 0.0 && p[d] >= 1.0) p[d] = 0.0;
    else if (k[d] < 0.0 && p[d] <= 0.0) p[d] = 1.0;
  }
}

/* --------------------------------------------------------------- opacity
 * Sect. 3.1: total opacity is the sum over lines plus dust, each line
 * evaluated at the photon frequency in the gas frame,
 * nu_cell = nu_ext / (1 + k.v/c) (the inverse of the printed frame relation
 * nu_ext = nu (1 + k.v/c)).
 *
 * Frequencies are carried as offsets dnu = nu - nu_ref from the reference
 * line centre (still in Hz): an absolute frequency of ~1e15 Hz would only
 * resolve x to ~5e-12, an offset resolves it to ~1e-15.  Every relation
 * below is the printed one rewritten for offsets. */
struct Problem {
  const orc_problem *pb;
  Mesh mesh;
  double nu_ref, dnu_ref;
  double lambda_ref_A;     /* rest wavelength of the reference line */
};

/* nu_i - nu_ref for line i, from the wavelengths (nu = c/lambda):
 * c (lambda_ref - lambda_i) / (lambda_i lambda_ref).  Differencing the two
 * absolute frequencies (~2.5e15 Hz for Lya) instead would leave ~0.25 Hz of
 * rounding, ~1e-11 of a narrow line's Doppler width. */
double lambda_offset(const Problem &P, double lambda_A) {
  return C_LIGHT * ((P.lambda_ref_A - lambda_A) / (lambda_A * P.lambda_ref_A)) * 1e8;
}
double line_offset(const Problem &P, const orc_line &ln) { return lambda_offset(P, ln.lambda0_A); }

/* Fluorescent re-emission (Sect. 3.2.1): the photon leaves along k at the
 * rest frequency nu_j of channel j in the frame of the scatterer (atom
 * velocity vatom), nu_cell = nu_j (1 + k.vatom/c), then to the external
 * frame through the cell velocity; returned as an offset from nu_ref. */
double to_external(const Problem &P, double dnu_cell, const double k[3], const double vc[3]);
double fluor_dnu_ext(const Problem &P, const orc_line &ln, int j, const double k[3], const double vatom[3],
                     const double vc[3]) {
  double off = lambda_offset(P, ln.fluor_lambda_A[j]);
  double nu_j = P.nu_ref + off;
  double dnu_cell = off + nu_j * (k[0] * vatom[0] + k[1] * vatom[1] + k[2] * vatom[2]) / C_LIGHT;
  return to_external(P, dnu_cell, k, vc);
}

struct Opac {
  double dnu_cell;
  double kd;
  double kl[4];
  double x[4];
  LineQ q[4];
  double ktot;
};

void opacity(const Problem &P, int64_t c, double dnu_ext, const double k[3], Opac &o) {
  const orc_problem &pb = *P.pb;
  double vc[3] = {pb.v[3 * c], pb.v[3 * c + 1], pb.v[3 * c + 2]};
  double beta = dot3(k, vc) / C_LIGHT;
  o.dnu_cell = (dnu_ext - P.nu_ref * beta) / (1.0 + beta);
  o.kd = pb.kappa_d[c];
  o.ktot = o.kd;
  for (int i = 0; i < pb.n_lines; ++i) {
    o.q[i] = line_q(pb.lines[i], pb.T[c]);
    o.x[i] = (o.dnu_cell - line_offset(P, pb.lines[i])) / o.q[i].dnu;
    double H = pb.voigt_exact ? voigt_h_exact(o.q[i].a, o.x[i]) : voigt_h(o.q[i].a, o.x[i]);
    o.kl[i] = pb.n_hi[c] * pb.lines[i].abundance * o.q[i].sigma0 * H;
    o.ktot += o.kl[i];
  }
}

double dnu_from_x(const Problem &P, double x) { return x * P.dnu_ref; }
double x_from_dnu(const Problem &P, double dnu) { return dnu / P.dnu_ref; }

/* external-frame offset of a packet with cell-frame offset dnu_cell moving
 * along k through gas of velocity vc: nu_ext = nu_cell (1 + k.v/c) */
double to_external(const Problem &P, double dnu_cell, const double k[3], const double vc[3]) {
  double beta = dot3(k, vc) / C_LIGHT;
  return dnu_cell + (P.nu_ref + dnu_cell) * beta;
}

/* Eq. for nu_out (Sect. 3.2.1): coherent in the atom frame,
 * nu_out = nu_in [1 + (k_out - k_in).v_X/c] / [1 + (1-mu) h nu_in/(m_X c^2)],
 * the denominator being recoil; returned as an offset from nu_ref. */
double scatter_dnu(const Problem &P, double dnu_in, const double kin[3], const double kout[3],
                   const double vatom[3], const orc_line &ln) {
  double nu_in = P.nu_ref + dnu_in;
  double dk[3] = {kout[0] - kin[0], kout[1] - kin[1], kout[2] - kin[2]};
  double shift = nu_in * dot3(dk, vatom) / C_LIGHT;
  double R = 0.0;
  if (ln.recoil) {
    double mu = dot3(kin, kout);
    R = (1.0 - mu) * H_PLANCK * nu_in / (ln.mass_amu * AMU_G * C_LIGHT * C_LIGHT);
  }
  return (dnu_in + shift - P.nu_ref * R) / (1.0 + R);
}

/* --------------------------------------------------------- ray casting
 * Optical depth from p along k to the domain border at a fixed external
 * frequency (the peel-off integral and the tau probe).  Every visited
 * leaf adds kappa * l * box.  `visit` receives (leaf, segment, Opac). */
template <class F>
double ray_tau(const Problem &P, const double p0[3], const double k[3], double dnu_ext,
               int64_t *ncross, F visit, double tau_stop = HUGE_VAL) {
  const orc_problem &pb = *P.pb;
  double p[3] = {p0[0], p0[1], p0[2]};
  int64_t c = locate(P.mesh, p, k);
  double tau = 0.0;
  Opac o;
  int64_t steps = 0;
  while (c >= 0 && steps++ < MAX_CROSS && !(tau >= tau_stop)) {
    opacity(P, c, dnu_ext, k, o);
    double pn[3];
    double te = exit_step(P.mesh, c, p, k, pn);
    double tdom = domain_dist(pb, p, k);
    ++*ncross;
    if (tdom <= te) {
      tau += o.ktot * tdom * pb.box_cm;
      visit(c, tdom, o);
      break;
    }
    tau += o.ktot * te * pb.box_cm;
    visit(c, te, o);
    p[0] = pn[0]; p[1] = pn[1]; p[2] = pn[2];
    wrap_slab(pb, p, k);
    c = locate(P.mesh, p, k);
  }
  return tau;
}

/* Image basis of an observer at k: e1 = normalize(z^ x k) (x^ when k is
 * along z), e2 = k x e1; pixel coordinates are (p - 1/2).e1, (p - 1/2).e2. */
void image_basis(const double k[3], double e1[3], double e2[3]) {
  if (k[0] == 0.0 && k[1] == 0.0) {
    e1[0] = 1.0; e1[1] = 0.0; e1[2] = 0.0;
  } else {
    double n = std::sqrt(k[1] * k[1] + k[0] * k[0]);
    e1[0] = -k[1] / n; e1[1] = k[0] / n; e1[2] = 0.0;
  }
  e2[0] = k[1] * e1[2] - k[2] * e1[1];
  e2[1] = k[2] * e1[0] - k[0] * e1[2];
  e2[2] = k[0] * e1[1] - k[1] * e1[0];
}

/* pixel index of position p, or -1 if outside the field of view */
int64_t pixel_of(const orc_observer &ob, const double p[3]) {
  double e1[3], e2[3];
  image_basis(ob.k, e1, e2);
  double q[3] = {p[0] - 0.5, p[1] - 0.5, p[2] - 0.5};
  double u = q[0] * e1[0] + q[1] * e1[1] + q[2] * e1[2];
  double v = q[0] * e2[0] + q[1] * e2[1] + q[2] * e2[2];
  double fu = (u - ob.fov[0]) / (ob.fov[1] - ob.fov[0]) * ob.nx;
  double fv = (v - ob.fov[2]) / (ob.fov[3] - ob.fov[2]) * ob.ny;
  if (!(fu >= 0.0 && fu < ob.nx && fv >= 0.0 && fv < ob.ny)) return -1;
  int64_t ix = (int64_t)std::floor(fu), iy = (int64_t)std::floor(fv);
  if (ix >= ob.nx || iy >= ob.ny) return -1;
  return iy * ob.nx + ix;
}

int64_t bin_of(const orc_observer &ob, double x) {
  double fb = (x - ob.x_min) / (ob.x_max - ob.x_min) * ob.nbins;
  if (!(fb >= 0.0 && fb < ob.nbins)) return -1;
  int64_t b = (int64_t)std::floor(fb);
  if (b >= ob.nbins) return -1;
  return b;
}

struct ThreadOut {
  std::vector<std::vector<double>> cubes;
  orc_stats st;
};

/* Peel-off (Sect. 5.1, the peeling algorithm of Yusef-Zadeh et al. and
 * Zheng & Miralda-Escude): at each emission or scattering the packet sends
 * weight P(mu_o)/(2 pi) exp(-tau_o) per steradian toward each observer,
 * where P is the event's own phase function normalised over mu in [-1,1]
 * (1/(4 pi) at an isotropic emission), tau_o the optical depth to the
 * domain border at the frequency the packet would have after scattering
 * into k_o. */
void peel_deposit(const Problem &P, int n_obs, const orc_observer *obs, ThreadOut &to,
                  const double p[3], int kind, const double kin[3], double dnu_in_cell,
                  const double vatom[3], const orc_line *ln, int core, const double vcell[3],
                  double dnu_ext_emit) {
  const orc_problem &pb = *P.pb;
  for (int o = 0; o < n_obs; ++o) {
    const orc_observer &ob = obs[o];
    const double *ko = ob.k;
    double weight, dnu_ext_o;
    if (kind == 0) { /* emission */
      weight = 1.0 / (4.0 * PI);
      dnu_ext_o = dnu_ext_emit;
    } else if (kind == 3) { /* fluorescent re-emission, isotropic; `core` is the channel */
      weight = 1.0 / (4.0 * PI);
      dnu_ext_o = fluor_dnu_ext(P, *ln, core, ko, vatom, vcell);
    } else if (kind == 1) { /* line scattering, same atom velocity */
      double mu = dot3(kin, ko);
      double P_ = (ln->phase == ORC_PHASE_ISO) ? 0.5 : (core ? p_core(mu) : p_wing(mu));
      weight = P_ / (2.0 * PI);
      double dnu_out = scatter_dnu(P, dnu_in_cell, kin, ko, vatom, *ln);
      dnu_ext_o = to_external(P, dnu_out, ko, vcell);
    } else { /* dust scattering: coherent in the cell frame */
      double mu = dot3(kin, ko);
      weight = p_hg(mu, pb.g_hg) / (2.0 * PI);
      dnu_ext_o = to_external(P, dnu_in_cell, ko, vcell);
    }
    int64_t nc = 0;
    /* with peel_tau_cut > 0 the walk stops once tau reaches it; from 746 on
     * exp(-tau) rounds to exactly 0 in double, so the deposit is the same */
    const double stop = pb.peel_tau_cut > 0.0 ? pb.peel_tau_cut : HUGE_VAL;
    double tau = ray_tau(P, p, ko, dnu_ext_o, &nc, [](int64_t, double, const Opac &) {}, stop);
    to.st.peel_rays += 1;
    to.st.peel_crossings += nc;
    double w = weight * std::exp(-tau);
    int64_t pix = pixel_of(ob, p);
    int64_t b = bin_of(ob, x_from_dnu(P, dnu_ext_o));
    if (pix < 0 || b < 0) { to.st.peel_dropped += 1; continue; }
    to.cubes[o][(size_t)pix * ob.nbins + b] += w;
  }
}

/* Core-skipping (Sect. 3.2.1 names the acceleration: the frequency
 * redistribution is biased so that a packet deep in the line core of an
 * optically thick cell jumps to the wing at once, Ahn et al. 2002,
 * Laursen et al. 2009).  The perpendicular velocity of the scattering atom
 * is drawn from the Gaussian restricted to |u_perp| >= x_crit: the 2-D
 * density exp(-u^2)/pi on u^2 >= x_crit^2 has radial CDF
 * 1 - exp(x_crit^2 - u^2), so |u_perp| = sqrt(x_crit^2 - ln r).  The paper
 * takes x_crit from Smith et al. 2015; this library's criterion is its own,
 * from the cell alone, with tau_cell = n_X sigma0(T) h the line-centre
 * optical depth across the cell's edge:
 *   x_crit = min( sqrt(ln(tau_cell / tau_skip)),  f (a tau_cell)^(1/3) ),
 * the first term the frequency below which the cell stays optically thick
 * by the factor tau_skip in the Gaussian core, the second a fraction f of
 * the frequency at which packets leave a medium as thick as the cell
 * (wings at |x| ~ (a tau)^(1/3)), so that a skip never carries a packet
 * past the frequencies it would escape at.  The draw is biased only while
 * |x| < x_crit.  Returns x_crit^2 for the draw, 0 when not skipping. */
double core_skip_x2(double tau_skip, double frac, double a, double tau_cell, double x) {
  if (!(tau_skip > 0.0) || !(tau_cell > tau_skip)) return 0.0;
  double xt = std::sqrt(std::log(tau_cell / tau_skip));
  double xw = frac * std::cbrt(a * tau_cell);
  double xc = std::min(xt, xw);
  return std::fabs(x) < xc ? xc * xc : 0.0;
}

/* ------------------------------------------------------------ transport
 * Sect. 3 (tau_event = -ln r, cell-by-cell subtraction), Sect. 3.2
 * (interaction choice by opacity fractions, resonant scattering with
 * recoil, dust absorption or HG scattering), Sect. 4.3 (moving from leaf
 * to leaf).  Position, path length and tau are double throughout. */
struct PacketOut {
  int32_t status;
  double x, k[3], pos[3], path;
  int32_t nscat;
};

/* Source spectrum (Sect. 2.1): the emitted frequency, as an offset in Hz
 * added to the source's own x.  Monochromatic: 0.  Gaussian line: the
 * Box-Muller draw sqrt(-2 ln r1) cos(2 pi r2) times the standard deviation
 * (given in Doppler widths of the reference line).  Power-law continuum
 * F_lambda ~ lambda^beta on [lambda_min, lambda_max]: the photon-number
 * distribution lambda F_lambda has the inverse CDF
 *   lambda = [lambda_min^(2+b) + r (lambda_max^(2+b) - lambda_min^(2+b))]^(1/(2+b)),
 *   lambda = lambda_min exp(r ln(lambda_max/lambda_min))  (b = -2),
 * and nu - nu_ref = c (lambda_ref - lambda) / (lambda lambda_ref). */
double spectrum_offset(const Problem &P, const Rng &rng) {
  const orc_problem &pb = *P.pb;
  if (pb.spec_kind == 1) {
    double g = std::sqrt(-2.0 * std::log(rng.u(J_SRC1))) * std::cos(2.0 * PI * rng.u(J_SRC2));
    return g * pb.spec_p[0] * P.dnu_ref;
  }
  if (pb.spec_kind == 3) {
    /* tabulated continuum: between neighbouring points F_lambda is the
     * power law through them; the photon count of bin i is the integral of
     * lambda F_lambda over it; a packet takes bin i with probability
     * N_i / sum N, then lambda inside it by the power-law inverse CDF */
    const int m = pb.spec_n;
    std::vector<double> beta(m - 1), cum(m, 0.0);
    for (int i = 0; i + 1 < m; ++i) {
      double l0 = pb.spec_lambda[i], l1 = pb.spec_lambda[i + 1];
      double b = std::log(pb.spec_flux[i + 1] / pb.spec_flux[i]) / std::log(l1 / l0);
      beta[i] = b;
      /* int_l0^l1 lambda F_i (lambda/l0)^b dlambda, in ratios (steep
       * slopes between close points would overflow lambda^(b+2)) */
      double n = (b == -2.0) ? pb.spec_flux[i] * l0 * l0 * std::log(l1 / l0)
                             : pb.spec_flux[i] * l0 * l0 * (std::pow(l1 / l0, b + 2.0) - 1.0) / (b + 2.0);
      cum[i + 1] = cum[i] + n;
    }
    double r1 = rng.u(J_SRC1) * cum[m - 1];
    int i = (int)(std::upper_bound(cum.begin() + 1, cum.end() - 1, r1) - (cum.begin() + 1));
    double l0 = pb.spec_lambda[i], l1 = pb.spec_lambda[i + 1], b = beta[i], r = rng.u(J_SRC2), lam;
    if (b == -2.0) {
      lam = l0 * std::exp(r * std::log(l1 / l0));
    } else {
      double e = 2.0 + b;
      lam = l0 * std::pow(1.0 + r * (std::pow(l1 / l0, e) - 1.0), 1.0 / e);
    }
    return C_LIGHT * ((P.lambda_ref_A - lam) / (lam * P.lambda_ref_A)) * 1e8;
  }
  if (pb.spec_kind == 2) {
    double lmin = pb.spec_p[0], lmax = pb.spec_p[1], b = pb.spec_p[2], r = rng.u(J_SRC1), lam;
    if (b == -2.0) {
      lam = lmin * std::exp(r * std::log(lmax / lmin));
    } else {
      double e = 2.0 + b;
      lam = std::pow(std::pow(lmin, e) + r * (std::pow(lmax, e) - std::pow(lmin, e)), 1.0 / e);
    }
    return C_LIGHT * ((P.lambda_ref_A - lam) / (lam * P.lambda_ref_A)) * 1e8;
  }
  return 0.0;
}

void transport_packet(const Problem &P, uint64_t seed, uint64_t pid, const double src_p[3],
                      const double *src_k, double src_x, int n_obs, const orc_observer *obs,
                      ThreadOut &to, PacketOut &out) {
  const orc_problem &pb = *P.pb;
  Rng rng{seed, pid, 0};
  double p[3] = {src_p[0], src_p[1], src_p[2]};
  double k[3];
  if (src_k) {
    k[0] = src_k[0]; k[1] = src_k[1]; k[2] = src_k[2];
  } else { /* isotropic emission, Sect. 2 */
    double mu = 2.0 * rng.u(J_MU) - 1.0;
    double phi = 2.0 * PI * rng.u(J_PHI);
    double s = std::sqrt(1.0 - mu * mu);
    k[0] = s * std::cos(phi); k[1] = s * std::sin(phi); k[2] = mu;
  }
  double dnu_ext = dnu_from_x(P, src_x) + spectrum_offset(P, rng);
  double tau_ev = -std::log(rng.u(J_TAU));
  double path = 0.0;
  int32_t nscat = 0;
  to.st.emitted += 1;
  {
    double zero[3] = {0.0, 0.0, 0.0};
    peel_deposit(P, n_obs, obs, to, p, 0, k, 0.0, zero, nullptr, 0, zero, dnu_ext);
  }
  int64_t c = locate(P.mesh, p, k);
  uint32_t event = 0;
  int64_t ncross_pk = 0;
  out.status = ORC_ST_ESCAPED;
  Opac o;
  while (true) {
    if (c < 0) { /* left the octree's cube on a non-periodic axis */
      out.status = ORC_ST_ESCAPED;
      break;
    }
    opacity(P, c, dnu_ext, k, o);
    double pn[3];
    double te = exit_step(P.mesh, c, p, k, pn);
    double tdom = domain_dist(pb, p, k);
    double lmax = std::min(te, tdom);
    double tau_seg = o.ktot * lmax * pb.box_cm;
    if (tau_ev < tau_seg) {
      /* interaction inside this leaf */
      double dist = tau_ev / (o.ktot * pb.box_cm);
      {
        int64_t s = (int64_t)1 << (P.mesh.L - P.mesh.lev[c]);
        int64_t org[3] = {P.mesh.ox[c], P.mesh.oy[c], P.mesh.oz[c]};
        for (int d = 0; d < 3; ++d) {
          double lo = std::ldexp((double)org[d], -P.mesh.L);
          double hi = std::ldexp((double)(org[d] + s), -P.mesh.L);
          double q = std::fma(dist, k[d], p[d]);
          p[d] = std::min(std::max(q, lo), hi);
        }
      }
      path += dist;
      ++event;
      if (pb.max_events > 0 && (int64_t)event >= pb.max_events) {
        out.status = ORC_ST_STUCK;
        break;
      }
      rng.event = event;
      double vc[3] = {pb.v[3 * c], pb.v[3 * c + 1], pb.v[3 * c + 2]};
      double r = rng.u(J_CHANNEL) * o.ktot;
      if (r < o.kd) {
        /* dust: absorbed with probability 1 - albedo (Sect. 3.2.2) */
        if (rng.u(J_ALBEDO) >= pb.albedo) {
          out.status = ORC_ST_ABSORBED;
          break;
        }
        to.st.dust_scatterings += 1;
        double kin[3] = {k[0], k[1], k[2]};
        double zero[3] = {0.0, 0.0, 0.0};
        peel_deposit(P, n_obs, obs, to, p, 2, kin, o.dnu_cell, zero, nullptr, 0, vc, 0.0);
        if (!pb.forward_only) {
          double mu = mu_hg(rng.u(J_MU), pb.g_hg);
          double phi = 2.0 * PI * rng.u(J_PHI);
          double e1[3], e2[3];
          perp_basis(kin, e1, e2);
          double s = std::sqrt(std::max(0.0, 1.0 - mu * mu));
          for (int d = 0; d < 3; ++d)
            k[d] = mu * kin[d] + s * (std::cos(phi) * e1[d] + std::sin(phi) * e2[d]);
          dnu_ext = to_external(P, o.dnu_cell, k, vc);
        }
      } else {
        /* resonant scattering in line i (Sect. 3.2.1) */
        r -= o.kd;
        int i = 0;
        while (i < pb.n_lines - 1 && r >= o.kl[i]) { r -= o.kl[i]; ++i; }
        const orc_line &ln = pb.lines[i];
        const LineQ &q = o.q[i];
        double dnu_in = o.dnu_cell;
        double x_in = o.x[i];
        double upar;
        if (!sample_upar(x_in, q.a, rng, &upar)) { out.status = ORC_ST_STUCK; break; }
        double tau_cell = pb.n_hi[c] * ln.abundance * q.sigma0 *
                          std::ldexp(pb.box_cm, -(int)P.mesh.lev[c]);
        double xc2 = core_skip_x2(pb.core_skip_tau, pb.core_skip_frac, q.a, tau_cell, x_in);
        double rr = std::sqrt(xc2 - std::log(rng.u(J_PERP1)));
        double ph = 2.0 * PI * rng.u(J_PERP2);
        double up1 = rr * std::cos(ph), up2 = rr * std::sin(ph);
        double kin[3] = {k[0], k[1], k[2]};
        double e1[3], e2[3];
        perp_basis(kin, e1, e2);
        double vatom[3];
        for (int d = 0; d < 3; ++d) vatom[d] = (upar * kin[d] + up1 * e1[d] + up2 * e2[d]) * q.vth;
        /* core or wing, from the frequency seen by the atom,
         * nu_scat,in = nu_in (1 - k_in . v_X / c), within 0.2 dnu_D of nu_lu */
        double off = (dnu_in - line_offset(P, ln)) - (P.nu_ref + dnu_in) * dot3(kin, vatom) / C_LIGHT;
        int core = std::fabs(off) < 0.2 * q.dnu;
        /* decay channel (Sect. 3.2.1): resonant with probability
         * A_ul / (A_ul + sum A_j), else fluorescent channel j by the
         * cumulative ratios */
        int fch = -1;
        if (ln.n_fluor > 0 && !pb.forward_only) {
          double a_tot = ln.A_ul + ln.fluor_A_ul[0] + (ln.n_fluor > 1 ? ln.fluor_A_ul[1] : 0.0);
          double u = rng.u(J_DECAY);
          if (u >= ln.A_ul / a_tot) fch = (ln.n_fluor > 1 && u >= (ln.A_ul + ln.fluor_A_ul[0]) / a_tot) ? 1 : 0;
        }
        nscat += 1;
        to.st.scatterings += 1;
        if (fch >= 0) {
          peel_deposit(P, n_obs, obs, to, p, 3, kin, dnu_in, vatom, &ln, fch, vc, 0.0);
          double mu = 2.0 * rng.u(J_MU) - 1.0;
          double phi = 2.0 * PI * rng.u(J_PHI);
          double s = std::sqrt(std::max(0.0, 1.0 - mu * mu));
          for (int d = 0; d < 3; ++d)
            k[d] = mu * kin[d] + s * (std::cos(phi) * e1[d] + std::sin(phi) * e2[d]);
          dnu_ext = fluor_dnu_ext(P, ln, fch, k, vatom, vc);
          tau_ev = -std::log(rng.u(J_TAU));
          continue;
        }
        peel_deposit(P, n_obs, obs, to, p, 1, kin, dnu_in, vatom, &ln, core, vc, 0.0);
        if (!pb.forward_only) {
          double ru = rng.u(J_MU);
          double mu = (ln.phase == ORC_PHASE_ISO) ? 2.0 * ru - 1.0 : (core ? mu_core(ru) : mu_wing(ru));
          double phi = 2.0 * PI * rng.u(J_PHI);
          double s = std::sqrt(std::max(0.0, 1.0 - mu * mu));
          for (int d = 0; d < 3; ++d)
            k[d] = mu * kin[d] + s * (std::cos(phi) * e1[d] + std::sin(phi) * e2[d]);
          double dnu_out = scatter_dnu(P, dnu_in, kin, k, vatom, ln);
          dnu_ext = to_external(P, dnu_out, k, vc);
        }
      }
      tau_ev = -std::log(rng.u(J_TAU));
      continue;
    }
    tau_ev -= tau_seg;
    path += lmax;
    to.st.crossings += 1;
    if (++ncross_pk >= MAX_CROSS) {
      out.status = ORC_ST_STUCK;
      break;
    }
    if (tdom <= te) {
      for (int d = 0; d < 3; ++d) p[d] = std::fma(tdom, k[d], p[d]);
      out.status = ORC_ST_ESCAPED;
      break;
    }
    p[0] = pn[0]; p[1] = pn[1]; p[2] = pn[2];
    wrap_slab(pb, p, k);
    c = locate(P.mesh, p, k);
  }
  if (out.status == ORC_ST_ESCAPED) to.st.escaped += 1;
  else if (out.status == ORC_ST_ABSORBED) to.st.absorbed += 1;
  else to.st.stuck += 1;
  out.x = x_from_dnu(P, dnu_ext);
  for (int d = 0; d < 3; ++d) { out.k[d] = k[d]; out.pos[d] = p[d]; }
  out.path = path;
  out.nscat = nscat;
}

int setup_problem(const orc_problem *pb, Problem &P) {
  if (!pb || pb->n_lines < 0 || pb->n_lines > 4) return -10;
  P.pb = pb;
  int rc = build_mesh(pb->n_leaves, pb->level, pb->ijk, P.mesh);
  if (rc) return rc;
  if (pb->n_lines > 0) {
    LineQ q = line_q(pb->lines[0], pb->T_ref);
    P.nu_ref = q.nu0;
    P.dnu_ref = q.dnu;
    P.lambda_ref_A = pb->lines[0].lambda0_A;
  } else { /* continuum: x is measured in units of 1e-5 of an arbitrary
              1215.67 A reference */
    P.nu_ref = C_LIGHT / 1215.67e-8;
    P.dnu_ref = P.nu_ref * 1e-5;
    P.lambda_ref_A = 1215.67;
  }
  return 0;
}

void add_stats(orc_stats &a, const orc_stats &b) {
  a.emitted += b.emitted; a.escaped += b.escaped; a.absorbed += b.absorbed; a.stuck += b.stuck;
  a.scatterings += b.scatterings; a.dust_scatterings += b.dust_scatterings;
  a.crossings += b.crossings; a.peel_rays += b.peel_rays; a.peel_crossings += b.peel_crossings;
  a.peel_dropped += b.peel_dropped;
}

int nthreads_of(int n) {
  if (n > 0) return n;
  unsigned h = std::thread::hardware_concurrency();
  return h ? (int)h : 1;
}

} /* namespace */

/* ================================================================ C API */
extern "C" {

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  philox(ctr, key, out);
}

double orc_uniform(uint64_t seed, uint64_t pid, uint32_t event, uint32_t j) {
  return uniform(seed, pid, event, j);
}

void orc_line_quantities(const orc_line *ln, double T, double out[5]) {
  LineQ q = line_q(*ln, T);
  out[0] = q.nu0; out[1] = q.vth; out[2] = q.dnu; out[3] = q.a; out[4] = q.sigma0;
}

double orc_voigt_h(double a, double x) { return voigt_h(a, x); }
double orc_voigt_dhdx(double a, double x) { return voigt_dhdx(a, x); }
double orc_voigt_h_exact(double a, double x) { return voigt_h_exact(a, x); }

void orc_sample_upar(int64_t n, double x, double a, uint64_t seed, double *out) {
  for (int64_t i = 0; i < n; ++i) {
    Rng rng{seed, (uint64_t)i, 1};
    sample_upar(x, a, rng, &out[i]);
  }
}

void orc_sample_mu(int64_t n, int kind, double g, uint64_t seed, double *out) {
  for (int64_t i = 0; i < n; ++i) {
    double r = uniform(seed, (uint64_t)i, 1, J_MU);
    if (kind == 0) out[i] = mu_core(r);
    else if (kind == 1) out[i] = mu_wing(r);
    else if (kind == 2) out[i] = mu_hg(r, g);
    else out[i] = 2.0 * r - 1.0;
  }
}

void orc_sample_uperp(int64_t n, double x_crit, uint64_t seed, double *out) {
  for (int64_t i = 0; i < n; ++i) {
    Rng rng{seed, (uint64_t)i, 1};
    double rr = std::sqrt(x_crit * x_crit - std::log(rng.u(J_PERP1)));
    double ph = 2.0 * PI * rng.u(J_PERP2);
    out[2 * i] = rr * std::cos(ph);
    out[2 * i + 1] = rr * std::sin(ph);
  }
}

void orc_single_scatter(int64_t n, const orc_line *ln, double T, double x_in, uint64_t seed,
                        double *x_out) {
  LineQ q = line_q(*ln, T);
  Problem P;
  P.pb = nullptr;
  P.nu_ref = q.nu0;
  P.dnu_ref = q.dnu;
  P.lambda_ref_A = ln->lambda0_A;
  double dnu_in = x_in * q.dnu;
  for (int64_t i = 0; i < n; ++i) {
    Rng rng{seed, (uint64_t)i, 1};
    /* incoming direction drawn isotropically so the pinned basis is
     * exercised in every orientation */
    Rng r0{seed, (uint64_t)i, 0};
    double mu0 = 2.0 * r0.u(J_MU) - 1.0, ph0 = 2.0 * PI * r0.u(J_PHI);
    double s0 = std::sqrt(1.0 - mu0 * mu0);
    double kin[3] = {s0 * std::cos(ph0), s0 * std::sin(ph0), mu0};
    double upar;
    sample_upar(x_in, q.a, rng, &upar);
    double rr = std::sqrt(-std::log(rng.u(J_PERP1)));
    double ph = 2.0 * PI * rng.u(J_PERP2);
    double up1 = rr * std::cos(ph), up2 = rr * std::sin(ph);
    double e1[3], e2[3];
    perp_basis(kin, e1, e2);
    double vatom[3];
    for (int d = 0; d < 3; ++d) vatom[d] = (upar * kin[d] + up1 * e1[d] + up2 * e2[d]) * q.vth;
    double off = dnu_in - (q.nu0 + dnu_in) * dot3(kin, vatom) / C_LIGHT;
    int core = std::fabs(off) < 0.2 * q.dnu;
    double ru = rng.u(J_MU);
    double mu = (ln->phase == ORC_PHASE_ISO) ? 2.0 * ru - 1.0 : (core ? mu_core(ru) : mu_wing(ru));
    double phi = 2.0 * PI * rng.u(J_PHI);
    double s = std::sqrt(std::max(0.0, 1.0 - mu * mu));
    double k[3];
    for (int d = 0; d < 3; ++d) k[d] = mu * kin[d] + s * (std::cos(phi) * e1[d] + std::sin(phi) * e2[d]);
    x_out[i] = scatter_dnu(P, dnu_in, kin, k, vatom, *ln) / q.dnu;
  }
}

int orc_mesh_validate(int64_t n, const int8_t *level, const int32_t *ijk) {
  Mesh m;
  int rc = build_mesh(n, level, ijk, m);
  if (rc) return rc;
  /* overlap: no ancestor of a leaf may itself be a leaf */
  for (int64_t c = 0; c < n; ++c) {
    int l = m.lev[c];
    int64_t i = ijk[3 * c], j = ijk[3 * c + 1], k = ijk[3 * c + 2];
    for (int a = 0; a < l; ++a) {
      int sh = l - a;
      if (m.map.count(mkey(a, i >> sh, j >> sh, k >> sh))) return -2;
    }
  }
  /* cover: with no overlap the volumes must add up to the whole cube */
  unsigned __int128 vol = 0, full = (unsigned __int128)1 << (3 * m.L);
  for (int64_t c = 0; c < n; ++c) vol += (unsigned __int128)1 << (3 * (m.L - m.lev[c]));
  if (vol != full) return -3;
  /* 2:1 grading across faces: the leaf holding the same-size face
   * neighbour region is at most one level coarser */
  for (int64_t c = 0; c < n; ++c) {
    int l = m.lev[c];
    int64_t side = (int64_t)1 << l;
    int64_t ii[3] = {ijk[3 * c], ijk[3 * c + 1], ijk[3 * c + 2]};
    for (int d = 0; d < 3; ++d) {
      for (int sgn = -1; sgn <= 1; sgn += 2) {
        int64_t nb[3] = {ii[0], ii[1], ii[2]};
        nb[d] += sgn;
        if (nb[d] < 0 || nb[d] >= side) continue;
        for (int a = l; a >= 0; --a) {
          int sh = l - a;
          if (m.map.count(mkey(a, nb[0] >> sh, nb[1] >> sh, nb[2] >> sh))) {
            if (a < l - 1) return -4;
            break;
          }
        }
      }
    }
  }
  return 0;
}

int64_t orc_locate(const orc_problem *pb, const double p[3], const double k[3]) {
  Mesh m;
  if (build_mesh(pb->n_leaves, pb->level, pb->ijk, m)) return -1;
  return locate(m, p, k);
}

int orc_trace(const orc_problem *pb, int64_t n, const double *orig, const double *dir,
              int32_t max_cells, int32_t *leaf_out, double *seg_out, int32_t *n_out) {
  Problem P;
  int rc = setup_problem(pb, P);
  if (rc) return rc;
  for (int64_t r = 0; r < n; ++r) {
    const double *k = dir + 3 * r;
    double p[3] = {orig[3 * r], orig[3 * r + 1], orig[3 * r + 2]};
    int64_t c = locate(P.mesh, p, k);
    int32_t cnt = 0;
    while (c >= 0 && cnt < max_cells) {
      double pn[3];
      double te = exit_step(P.mesh, c, p, k, pn);
      double tdom = domain_dist(*pb, p, k);
      leaf_out[(size_t)r * max_cells + cnt] = (int32_t)c;
      if (tdom <= te) {
        seg_out[(size_t)r * max_cells + cnt] = tdom;
        ++cnt;
        break;
      }
      seg_out[(size_t)r * max_cells + cnt] = te;
      ++cnt;
      p[0] = pn[0]; p[1] = pn[1]; p[2] = pn[2];
      wrap_slab(*pb, p, k);
      c = locate(P.mesh, p, k);
    }
    n_out[r] = cnt;
  }
  return 0;
}

int orc_tau(const orc_problem *pb, int64_t n, const double *orig, const double *dir,
            const double *x_ext, double *tau_out) {
  Problem P;
  int rc = setup_problem(pb, P);
  if (rc) return rc;
  for (int64_t r = 0; r < n; ++r) {
    int64_t nc = 0;
    tau_out[r] = ray_tau(P, orig + 3 * r, dir + 3 * r, dnu_from_x(P, x_ext[r]), &nc,
                         [](int64_t, double, const Opac &) {});
  }
  return 0;
}

int orc_run(const orc_problem *pb, int64_t n_src, const double *src_pos, const double *src_dir,
            const double *src_x, uint64_t seed, int64_t first, int64_t n, int n_obs,
            const orc_observer *obs, double *const *cubes, int32_t *status, double *x_out,
            double *k_out, double *pos_out, int32_t *n_scat, double *path_out, int n_threads,
            orc_stats *stats) {
  Problem P;
  int rc = setup_problem(pb, P);
  if (rc) return rc;
  if (n_src <= 0 || first < 0 || n < 0 || first + n > n_src) return -11;
  int nt = nthreads_of(n_threads);
  std::vector<ThreadOut> outs(nt);
  for (auto &t : outs) {
    t.cubes.resize(n_obs);
    for (int o = 0; o < n_obs; ++o)
      t.cubes[o].assign((size_t)obs[o].nx * obs[o].ny * obs[o].nbins, 0.0);
    std::memset(&t.st, 0, sizeof(t.st));
  }
  std::atomic<int64_t> next(0);
  auto work = [&](int tid) {
    ThreadOut &to = outs[tid];
    while (true) {
      int64_t i = next.fetch_add(1);
      if (i >= n) break;
      int64_t pid = first + i;
      PacketOut po;
      transport_packet(P, seed, (uint64_t)pid, src_pos + 3 * pid, src_dir ? src_dir + 3 * pid : nullptr,
                       src_x[pid], n_obs, obs, to, po);
      if (status) status[i] = po.status;
      if (x_out) x_out[i] = po.x;
      if (k_out) for (int d = 0; d < 3; ++d) k_out[3 * i + d] = po.k[d];
      if (pos_out) for (int d = 0; d < 3; ++d) pos_out[3 * i + d] = po.pos[d];
      if (n_scat) n_scat[i] = po.nscat;
      if (path_out) path_out[i] = po.path;
    }
  };
  std::vector<std::thread> th;
  for (int t = 0; t < nt; ++t) th.emplace_back(work, t);
  for (auto &t : th) t.join();
  orc_stats tot;
  std::memset(&tot, 0, sizeof(tot));
  for (auto &t : outs) add_stats(tot, t.st);
  for (int o = 0; o < n_obs; ++o) {
    if (!cubes || !cubes[o]) continue;
    size_t sz = (size_t)obs[o].nx * obs[o].ny * obs[o].nbins;
    for (size_t b = 0; b < sz; ++b) {
      double s = 0.0;
      for (auto &t : outs) s += t.cubes[o][b];
      cubes[o][b] += s;
    }
  }
  if (stats) *stats = tot;
  return 0;
}

int orc_raycast_image(const orc_problem *pb, const orc_observer *ob, int64_t n_rays,
                      const double *orig, const double *x_ext, const double *w, double *image,
                      const double *grad_image, double *g_nhi, double *g_kd, double *g_vlos,
                      int n_threads, int64_t *n_crossings) {
  /* the gradient uses the dH/dx of the Tasitsiomi form */
  if (grad_image && pb->voigt_exact) return -5;
  Problem P;
  int rc = setup_problem(pb, P);
  if (rc) return rc;
  struct Rec { int64_t c; double gn, gk, gv; };
  std::vector<double> tau(n_rays, 0.0);
  std::vector<int64_t> pix(n_rays, -1);
  std::vector<std::vector<Rec>> recs(grad_image ? n_rays : 0);
  int nt = nthreads_of(n_threads);
  std::atomic<int64_t> next(0);
  std::atomic<int64_t> total_cross(0);
  auto work = [&]() {
    while (true) {
      int64_t r = next.fetch_add(1);
      if (r >= n_rays) break;
      const double *p = orig + 3 * r;
      pix[r] = pixel_of(*ob, p);
      double dnu = dnu_from_x(P, x_ext[r]);
      int64_t nc = 0;
      std::vector<std::pair<int64_t, double>> cross;
      tau[r] = ray_tau(P, p, ob->k, dnu, &nc, [&](int64_t c, double seg, const Opac &) {
        cross.emplace_back(c, seg);
      });
      total_cross += nc;
      if (!grad_image || pix[r] < 0) continue;
      /* dL/dtau_r = -G_p w_r exp(-tau_r); dtau_r/dtheta_c summed over
       * the crossings of c (one per visit) */
      double g = -grad_image[pix[r]] * w[r] * std::exp(-tau[r]);
      for (auto &cs : cross) {
        int64_t c = cs.first;
        double l = cs.second * pb->box_cm;
        Opac o;
        opacity(P, c, dnu, ob->k, o);
        double vc[3] = {pb->v[3 * c], pb->v[3 * c + 1], pb->v[3 * c + 2]};
        double beta = dot3(ob->k, vc) / C_LIGHT;
        double dn = 0.0, dv = 0.0;
        for (int i = 0; i < pb->n_lines; ++i) {
          double ab = pb->lines[i].abundance;
          dn += ab * o.q[i].sigma0 * voigt_h(o.q[i].a, o.x[i]);
          /* x = (nu_ext/(1+beta) - nu0)/dnu_D  =>
           * dx/dv_los = -nu_ext / (c (1+beta)^2 dnu_D) */
          double nu_ext = P.nu_ref + dnu;
          double dxdv = -nu_ext / (C_LIGHT * (1.0 + beta) * (1.0 + beta) * o.q[i].dnu);
          dv += pb->n_hi[c] * ab * o.q[i].sigma0 * voigt_dhdx(o.q[i].a, o.x[i]) * dxdv;
        }
        recs[r].push_back(Rec{c, g * l * dn, g * l, g * l * dv});
      }
    }
  };
  std::vector<std::thread> th;
  for (int t = 0; t < nt; ++t) th.emplace_back(work);
  for (auto &t : th) t.join();
  for (int64_t r = 0; r < n_rays; ++r)
    if (pix[r] >= 0) image[pix[r]] += w[r] * std::exp(-tau[r]);
  if (grad_image) {
    for (int64_t r = 0; r < n_rays; ++r)
      for (auto &e : recs[r]) {
        g_nhi[e.c] += e.gn;
        g_kd[e.c] += e.gk;
        g_vlos[e.c] += e.gv;
      }
  }
  if (n_crossings) *n_crossings = total_cross.load();
  return 0;
}

} /* extern "C" */
