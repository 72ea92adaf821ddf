// rmc_device.h -- device-side data layout and building blocks of the
// resonant-line Monte Carlo kernels (gfx950).
//
// Method: Michel-Dansac et al. 2020 (RASCAS).  Frequencies are carried as
// x_ext, the external-frame offset from the first line's rest frequency in
// Doppler widths of that line at T_ref; every per-cell quantity is expressed
// relative to T_ref so that all float work stays O(1):
//   per leaf   nl = n_HI box / rho, irho = 1/rho, rho = sqrt(T/T_ref),
//              kd = kappa_d box, u = v / v_th,ref
//   per line   s = nu_ref/nu_i, delta = (s-1)/b_ref, inv_mu = sqrt(m_i/m_ref),
//              alpha = a_i(T_ref), kfac = abundance sigma0_i(T_ref)
// so that in a leaf, for a packet moving along k with w = k.u,
//   x_i = (delta + s x_ext - w) irho inv_mu / (1 + b_ref w)
//   kappa_i box = nl kfac H(alpha irho, x_i)
// (Sect. 3.1.1 cross-section, Sect. 3 frame relation nu_ext = nu(1+k.v/c)).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rmc_math.h"

namespace rmc {

constexpr int MAX_LEVEL = 16;
// Level of the table of cells that point location starts from, and where a
// table entry for a leaf keeps the leaf's level (the leaf index below it)
constexpr int TOP_LEVEL = 6;
constexpr int TOP_LEVEL_SHIFT = 27;
constexpr int MAX_LINES = 4;
constexpr int MAX_OBS = 4;
constexpr int LEAF_STRIDE = 8;   // values per leaf record (6 used, padded)
// A packet or ray that has crossed this many leaves is stopped (a packet
// gets status stuck): it bounds the walk of a ray parallel to a periodic slab.
constexpr uint32_t MAX_CROSS = 1u << 24;
constexpr double PI_D = 3.14159265358979323846;

enum { DOM_BOX = 0, DOM_SLAB_Z = 1, DOM_SPHERE = 2 };
enum { PHASE_LYA = 0, PHASE_ISO = 1 };
enum { ST_NONE = 0, ST_ESCAPED = 1, ST_ABSORBED = 2, ST_STUCK = 3 };
enum {
  S_EMITTED = 0, S_ESCAPED, S_ABSORBED, S_STUCK, S_SCAT, S_DUST_SCAT, S_CROSS,
  S_PEEL_RAYS, S_PEEL_CROSS, S_PEEL_DROPPED, N_STATS
};

struct LineK {
  double delta, s, inv_s, inv_mu, mu, alpha, kfac;
  double lalpha;   // log10 alpha
  double ibmu;     // 1 / (b_ref mu): v_th,line / c is b_ref mu rho
  double rec;      // h nu_i / (m_i c^2)
  int phase, recoil;
  // fluorescent channels: decay through channel j when the draw u lies at
  // or above a_res (j = 0) / a_cum0 (j = 1); the photon leaves at
  // x_ext = xf0[j] + sf[j] (b_a + b_c + b_a b_c) / b_ref with b_a, b_c the
  // atom's and the cell's k.v/c, xf0 = (lambda_ref - lambda_j)/(lambda_j b_ref),
  // sf = lambda_ref / lambda_j (nu_j / nu_ref)
  int n_fluor;
  double a_res, a_cum0, xf0[2], sf[2];
  // the same constants rounded to float on the host (as a conversion on the
  // device would round them), for the float path
  struct {
    float delta, s, inv_s, inv_mu, mu, alpha, kfac, ibmu, rec, a_res, a_cum0, xf0[2], sf[2];
  } f;
};

// A constant in the path's precision: the double, or its float copy.
template <class R> __device__ __forceinline__ R cst(double d, float f);
template <> __device__ __forceinline__ double cst<double>(double d, float) { return d; }
template <> __device__ __forceinline__ float cst<float>(double, float f) { return f; }

struct ObsK {
  double k[3], e1[3], e2[3];
  double u0, uspan, v0, vspan, x_min, xspan;
  double su, sv, sx;   // nx/uspan, ny/vspan, nbins/xspan (float path binning)
  double kinv[3];      // 1/k (0 where k is 0; float path ray walks)
  float kf[3];         // k rounded to float
  int nx, ny, nbins, pad;
  void *cube;      // [ny][nx][nbins], float or double by precision
};

// A peel-off ray queued for the ray-cast pass that follows each transport
// launch: cube element | observer << 40 | problem << 44 in dst.  Double
// path: the point where the ray enters its next leaf (or its start), the
// optical depth so far and the leaves crossed so far (64 B).  Float path:
// the ray's start, its frequency and weight in float (40 B); its cube
// element is left 0 and found by the pass from the start and frequency.
template <class R> struct PeelJob;
template <> struct PeelJob<double> {
  double p[3];
  double tau;
  double x;                 // x_ext of the ray (frequency toward the observer)
  double weight;            // phase-function weight of the deposit
  unsigned long long dst;
  uint32_t steps, pad;
};
template <> struct PeelJob<float> {
  double p[3];
  unsigned long long dst;
  float x, weight;
};
constexpr int PQ_OBS_SHIFT = 40, PQ_PROB_SHIFT = 44;
constexpr unsigned long long PQ_ELEM_MASK = (1ull << PQ_OBS_SHIFT) - 1ull;

struct PeelQueue {
  void *jobs;                     // PeelJob<R> [n_regions][cap]: one region per transport wave
  uint32_t *counts;               // [n_regions]: pushes of each region in the last launch
  unsigned long long cap;         // jobs per region (a wave stops its slice before it)
  unsigned long long n_regions;
  unsigned long long pushes;      // pushes of the launch
  unsigned long long max_region;  // largest region push count of the launch
  unsigned long long take;        // regions handed out by the ray-cast pass
  unsigned long long lost;        // pushes that found their region full (an error)
};

// Crossing lists ("tape") of the rays of one image pass, for the adjoint.
// The rays of a wave (64 consecutive rays) walk in step; the wave keeps a
// linked list of chunks of TAPE_CHUNK wave iterations, each lane-
// interleaved (entry of iteration i, lane l at (i % TAPE_CHUNK) * 64 + l),
// so a wave stores and loads whole 256-B runs of leaf indices and segments.
constexpr int TAPE_CHUNK = 32;
constexpr int TAPE_ENTRIES = TAPE_CHUNK * 64;
struct TapeK {
  int32_t *leaf;             // [cap][TAPE_ENTRIES] leaf crossed
  void *seg;                 // [cap][TAPE_ENTRIES] segment (box units), float or double
  int64_t *next;             // [cap] next chunk of the same wave, -1 at its end
  int64_t *first;            // [waves] first chunk of the wave, -1 none
  int32_t *count;            // [rays] crossings recorded for the ray
  int32_t *pix;              // [rays] image pixel, -1 outside
  double *wt;                // [rays] w exp(-tau); 0 where exp(-tau) is zero
  double *x;                 // [rays] x_ext
  unsigned long long *ctl;   // [0]: chunks requested (beyond cap: none given)
  unsigned long long cap;    // chunks
};

struct ProblemK {
  const int32_t *nodes;     // [n_nodes][8]: >=0 child node, <0: -(leaf+1)
  const void *leaves;       // [n_leaves][LEAF_STRIDE] float or double
  int L;                    // deepest leaf level
  // the cells of level top_level (z-major, x fastest): >= 0 the node there,
  // < 0 -(leaf | level << TOP_LEVEL_SHIFT) - 1 for the leaf (of level
  // <= top_level) covering it; null: every descent starts at the root
  const int32_t *top;
  int top_level;
  int n_lines;
  LineK lines[MAX_LINES];
  double b_ref;             // v_th(T_ref, line 0) / c
  double box_cm;
  int domain;
  double dom[4];
  double albedo, g_hg;
  float b_ref_f, albedo_f, g_hg_f;  // b_ref, albedo and g_hg rounded to float
  int forward_only;
  int64_t max_events;
  double skip_tau, skip_frac; // core-skipping (skip_tau > 0: on)
  int voigt_exact;          // 1: H from voigt_h_exact, 0: the Tasitsiomi form
  int spec_kind;            // source spectrum: 0 monochromatic, 1 Gaussian, 2 power law
  double spec_p[3];         // sigma_x | lambda_min, lambda_max (A), beta
  double lambda_ref;        // rest wavelength of line 0 (A)
  // tabulated continuum (spec_kind 3): tab_n wavelengths, the power-law
  // slope of F_lambda in each of the tab_n - 1 bins, cumulative photon counts
  int tab_n;
  const double *tab_lam, *tab_beta, *tab_cum;
  // sources (device)
  const double *src_pos, *src_dir, *src_x;
  int64_t first, n;         // packet range of this run
  uint64_t seed;
  // per-packet outputs, indexed pid - first
  int32_t *status, *nscat;
  double *x_out, *k_out, *pos_out, *path_out;
  int n_obs;
  ObsK obs[MAX_OBS];
  unsigned long long *stats; // [N_STATS]
  PeelQueue *pq;            // deferred peel-off rays (null: traced inline)
  int index;                // position in the launch's problem array
};

// ------------------------------------------------------------------ Philox
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11).  Each round's two
// 32x32-bit products are taken whole as 64-bit products: one
// v_mad_u64_u32 gives both halves, where separate high and low multiplies
// cost two multi-pass instructions.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint2 k) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    c = make_uint4(hi1 ^ c.y ^ k.x, lo1, hi0 ^ c.w ^ k.y, lo0);
    k.x += 0x9E3779B9u;
    k.y += 0xBB67AE85u;
  }
  return c;
}

// Slots of the uniforms of one event (counter = pid, event, block).
enum {
  J_CHANNEL = 0,  // dust or which line
  J_MU = 1,       // scattering-angle cosine (emission: direction cosine)
  J_PHI = 2,      // azimuth
  J_TAU = 3,      // optical depth to the next event
  J_PERP1 = 4,    // Box-Muller pair for the two perpendicular atom velocities
  J_PERP2 = 5,
  J_ALBEDO = 6,   // dust: scatter or absorb
  J_GAUSS1 = 6,   // line, |x| >= 8: Box-Muller pair for the Gaussian
  J_GAUSS2 = 7,
  J_REJ = 6,      // line, |x| < 8: rejection round i uses J_REJ+3i .. +2
                  // (double) or J_REJ+2i, +1 (float)
  J_SRC1 = 4,     // emission (event 0): source-spectrum draws
  J_SRC2 = 5,
  J_DECAY = 1 << 30  // line: resonant or fluorescent decay (far above any
                     // rejection round, which stops at 2^20)
};

// Uniforms of one event.  Double: draw j uses the word pair (2(j%2),
// 2(j%2)+1) of block j/2 and returns (2m+1) 2^-53 with m the top 52 bits.
// Float: (2m+1) 2^-24 with m 23 bits of the blocks' words, placed below.
// Both lie strictly inside (0,1).
template <class R> struct EventRng;

template <> struct EventRng<double> {
  uint2 key;
  uint32_t plo, phi, ev;
  uint32_t cur;
  uint4 w;
  __device__ EventRng(uint64_t seed, uint64_t pid, uint32_t event)
      : key(make_uint2((uint32_t)seed, (uint32_t)(seed >> 32))), plo((uint32_t)pid),
        phi((uint32_t)(pid >> 32)), ev(event), cur(0xffffffffu) {}
  __device__ double u(uint32_t j) {
    const uint32_t b = j >> 1;
    if (b != cur) {
      w = philox4x32_10(make_uint4(plo, phi, ev, b), key);
      cur = b;
    }
    const uint32_t hi = (j & 1) ? w.z : w.x;
    const uint32_t lo = (j & 1) ? w.w : w.y;
    const uint64_t m = ((uint64_t)hi << 20) | (uint64_t)(lo >> 12);
    return (double)(2 * m + 1) * 0x1p-53;
  }
  // 2^-52 spacing resolves any probability the path compares with
  __device__ double u_small(uint32_t j) { return u(j); }
};

// Float: a draw takes 23 bits, so a 32-bit word has 9 to spare.  Two blocks
// hold every draw of an event up to its second rejection round:
//   block 0  word 0 the channel (all 32 bits), the top 23 bits of word 1
//            tau_event, of words 2 and 3 the first rejection round (or the
//            albedo test, or the |x| >= 8 Gaussian pair); the direction
//            cosine from the low 9 bits of words 1, 2, 3 (the top 23 of 27)
//   block 1  the top 23 bits of words 0 and 1 the second rejection round,
//            of words 2 and 3 the perpendicular velocities (emission: the
//            source-spectrum pair); the azimuth from the low 9 bits of words
//            0, 1, 2
//   block b  (b >= 2) the top 23 bits of words 0 and 1 rejection round
//            2b - 2, of words 2 and 3 round 2b - 1
// so the second rejection round costs no block of its own.  Draw j >= 8
// (rounds beyond the first, and the decay draw far above them) belongs to
// round k = (j - 6) / 2 (its first or second draw as j is even or odd).
template <> struct EventRng<float> {
  uint2 key;
  uint32_t plo, phi, ev;
  uint4 b0, b1;
  bool have1;
  __device__ EventRng(uint64_t seed, uint64_t pid, uint32_t event)
      : key(make_uint2((uint32_t)seed, (uint32_t)(seed >> 32))), plo((uint32_t)pid),
        phi((uint32_t)(pid >> 32)), ev(event), have1(false) {
    b0 = block(0);
  }
  __device__ uint4 block(uint32_t b) const { return philox4x32_10(make_uint4(plo, phi, ev, b), key); }
  // block 1, computed once (where every lane of a branch that needs it is
  // active, the block is computed once per wave)
  __device__ void need1() {
    if (!have1) {
      b1 = block(1);
      have1 = true;
    }
  }
  static __device__ __forceinline__ float top(uint32_t w) { return (float)(2u * (w >> 9) + 1u) * 0x1p-24f; }
  static __device__ __forceinline__ float low(uint32_t a, uint32_t b, uint32_t c) {
    const uint32_t m = ((a & 511u) << 14) | ((b & 511u) << 5) | ((c & 511u) >> 4);
    return (float)(2u * m + 1u) * 0x1p-24f;
  }
  // the pair of rejection round k (draws J_REJ + 2k and J_REJ + 2k + 1)
  __device__ void round(uint32_t k, float *r1, float *r3) {
    uint32_t x, y;
    if (k == 0) {
      x = b0.z;
      y = b0.w;
    } else if (k == 1) {
      need1();
      x = b1.x;
      y = b1.y;
    } else {
      const uint4 w = block(1 + k / 2);
      x = (k & 1) ? w.z : w.x;
      y = (k & 1) ? w.w : w.y;
    }
    *r1 = top(x);
    *r3 = top(y);
  }
  __device__ float u(uint32_t j) {
    switch (j) {
      case J_CHANNEL: return top(b0.x);
      case J_TAU: return top(b0.y);
      case J_MU: return low(b0.y, b0.z, b0.w);
      case J_PHI: need1(); return low(b1.x, b1.y, b1.z);
      case J_PERP1: need1(); return top(b1.z);
      case J_PERP2: need1(); return top(b1.w);
      case J_REJ: return top(b0.z);
      case J_REJ + 1: return top(b0.w);
      default: {
        float r1, r3;
        round((j - J_REJ) >> 1, &r1, &r3);
        return (j & 1) ? r3 : r1;
      }
    }
  }
  // The channel draw, compared with a probability that may be far below
  // the 2^-23 spacing of u (kappa_d / kappa in an optically thick line
  // core): the whole 32-bit word, so near zero the draw is resolved to
  // 2^-32.  Lies in [0, 1].
  __device__ float u_small(uint32_t) { return (float)b0.x * 0x1p-32f; }
};

// ------------------------------------------------------------ math policy
template <class R> struct M;
template <> struct M<double> {
  static __device__ __forceinline__ double exp(double x) { return exp_any(x); }
  static __device__ __forceinline__ double log(double x) { return log_pos(x); }
  static __device__ __forceinline__ double log10(double x) { return ::log10(x); }
  static __device__ __forceinline__ double sqrt(double x) { return ::sqrt(x); }
  static __device__ __forceinline__ double cbrt(double x) { return ::cbrt(x); }
  // exp, log, the draw's arctangent and its tangent of |th| <= pi/2, and
  // the sine and cosine of 2 pi r: the forms of rmc_math.h
  static __device__ __forceinline__ double atan(double x) { return atan_any(x); }
  static __device__ __forceinline__ double tan(double x) { return tan_halfpi(x); }
  static __device__ __forceinline__ void sincos2pi(double r, double *s, double *c) { sincos_turns(r, s, c); }
  static __device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
  static __device__ __forceinline__ double rsqrt(double x) { return 1.0 / ::sqrt(x); }
  static __device__ __forceinline__ double div(double a, double b) { return a / b; }
  static __device__ __forceinline__ double cbrt_pos(double x) { return ::cbrt(x); }
};
// The float path uses the hardware transcendental instructions (log2,
// exp2, sqrt, rcp, sin and cos in turns, each within a few ulp); its
// arguments here are normal numbers (uniforms >= 2^-24, positive sums).
template <> struct M<float> {
  static __device__ __forceinline__ float exp(float x) { return __expf(x); }
  static __device__ __forceinline__ float log(float x) {
    return __builtin_amdgcn_logf(x) * 0.69314718055994531f;
  }
  static __device__ __forceinline__ float log10(float x) {
    return __builtin_amdgcn_logf(x) * 0.30102999566398120f;
  }
  static __device__ __forceinline__ float sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
  static __device__ __forceinline__ float cbrt(float x) { return ::cbrtf(x); }
  static __device__ __forceinline__ float atan(float x) { return ::atanf(x); }
  static __device__ __forceinline__ float tan(float x) {
    float s, c;
    __sincosf(x, &s, &c);
    return s * __builtin_amdgcn_rcpf(c);
  }
  // the hardware sine and cosine take their argument in turns
  static __device__ __forceinline__ void sincos2pi(float r, float *s, float *c) {
    *s = __builtin_amdgcn_sinf(r);
    *c = __builtin_amdgcn_cosf(r);
  }
  static __device__ __forceinline__ float rcp(float x) { return __frcp_rn(x); }
  static __device__ __forceinline__ float rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
  // a times the hardware reciprocal of b (about 1 ulp)
  static __device__ __forceinline__ float div(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
  // cube root of a positive normal number from the hardware log2 and exp2
  static __device__ __forceinline__ float cbrt_pos(float x) {
    return __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(x) * (1.0f / 3.0f));
  }
};

// ---------------------------------------------------------------- Voigt H
// Tasitsiomi (2006) form named in Sect. 3.3.2:
//   z = (x^2 - 0.855)/(x^2 + 3.42); q = 0 (z <= 0) else
//   z (1 + 21/x^2) (a/pi)/(x^2+1) (((5.674 z - 9.207) z + 4.421) z + 0.1117)
//   H = sqrt(pi) q + exp(-x^2)
template <class R> __device__ __forceinline__ R voigt_h(R a, R x) {
  const R x2 = x * x;
  const R z = M<R>::div(x2 - R(0.855), x2 + R(3.42));
  R h = M<R>::exp(-x2);
  if (z > R(0)) {
    const R P = ((R(5.674) * z - R(9.207)) * z + R(4.421)) * z + R(0.1117);
    R q;
    if constexpr (sizeof(R) == 4) {
      // (1 + 21/x^2) / (x^2 + 1) as one quotient: one reciprocal
      q = M<R>::div(z * (x2 + R(21)) * (a * R(1.0 / PI_D)), x2 * (x2 + R(1))) * P;
    } else {
      q = M<R>::div(z * (R(1) + M<R>::div(R(21), x2)) * (a * R(1.0 / PI_D)), x2 + R(1)) * P;
    }
    h += R(1.7724538509055160273) * q;
  }
  return h;
}

// H(a, x) = Re w(x + ia) in double to ~1e-14 relative (the accurate
// evaluator Sect. 3.3.2 measures its fast forms against; H from its
// Sect. 3.1.1 definition).  For Im z > 0, w(z) = (i/pi) int e^{-t^2} /
// (z - t) dt.  The trapezoidal rule with step s = 1/2 converges like
// e^{-pi^2/s^2} once the pole at t = z is accounted for:
//   w(z) ~ (i s/pi) sum_n e^{-t_n^2}/(z - t_n) + 2 e^{-z^2}/(1 -+ e^{-2 pi i z/s}),
// nodes t_n = n s ("-") or (n - 1/2) s ("+"), whichever set keeps x at
// least s/4 from every node (the two parts of the formula then stay
// moderate).  Pairing t and -t, the real part of the sum is
//   (s/pi) a sum_n e^{-t_n^2} (x^2 + a^2 + t_n^2) / ((x^2 - t_n^2 - a^2)^2 + 4 a^2 x^2),
// a sum of positive terms (the t = 0 node contributes 1/(x^2 + a^2) once).
// For |x| >= 30 the asymptotic series w ~ (i/sqrt(pi)) sum_k (2k-1)!!/2^k
// z^-(2k+1) is used (the imaginary parts of its powers share one sign).
__device__ __attribute__((noinline)) double voigt_h_exact(double a, double x) {
  const double ax = fabs(x);
  if (ax >= 30.0) {
    const double d = x * x + a * a;
    const double ur = x / d, ui = -a / d;                      // 1/z
    const double vr = ur * ur - ui * ui, vi = 2.0 * ur * ui;  // 1/z^2
    double tr = ur, ti = ui, si = ui;
    for (int k = 1; k < 12; ++k) {
      const double c = (2.0 * k - 1.0) * 0.5;
      const double nr = (tr * vr - ti * vi) * c, ni = (tr * vi + ti * vr) * c;
      tr = nr;
      ti = ni;
      si += ti;
    }
    return -si * 0.56418958354775628695;  // 1/sqrt(pi)
  }
  const double q = 2.0 * ax;  // |x| / s
  const double fr = q - floor(q);
  const bool mid = fr < 0.25 || fr > 0.75;
  const double a2 = a * a, x2a2 = x * x + a2, fa2x2 = 4.0 * a2 * x * x;
  double sum = mid ? 0.0 : 1.0 / x2a2;
  // e^{-t_n^2} by ratios: nodes n/2 have e^{-n^2/4}, ratio e^{-(2n-1)/4};
  // half-nodes (2n-1)/4 have e^{-(2n-1)^2/16}, ratio e^{-(n-1)/2}
  double c = mid ? 0.93941306281347578612 : 0.77880078307140486825;   // e^{-1/16}, e^{-1/4}
  double rho = mid ? 0.60653065971263342360 : 0.47236655274101470714;  // e^{-1/2}, e^{-3/4}
  for (int n = 1; n <= 14; ++n) {
    const double t = mid ? 0.5 * n - 0.25 : 0.5 * n;
    const double dd = (ax - t) * (ax + t) - a2;
    sum += 2.0 * c * (x2a2 + t * t) / (dd * dd + fa2x2);
    c *= rho;
    rho *= 0.60653065971263342360;  // e^{-1/2}
  }
  double h = 0.15915494309189533577 * a * sum;  // s/pi = 1/(2 pi)
  const double g = exp(a2 - x * x);
  if (g > 0.0 && a < 20.0) {  // (the pole term is below e^{-37} for a > 3)
    // Re[2 E / D], E = e^{-z^2} = g (cos 2ax - i sin 2ax),
    // D = 1 - sg e^{4 pi a} (cos 4 pi x - i sin 4 pi x), sg = +1 ("-"), -1 ("+")
    double s1, c1, s2, c2;
    sincos(2.0 * a * x, &s1, &c1);
    sincospi(4.0 * x, &s2, &c2);
    const double e = (mid ? -1.0 : 1.0) * exp(12.566370614359172954 * a);
    const double dr = 1.0 - e * c2, di = e * s2;
    h += 2.0 * g * (c1 * dr - s1 * di) / (dr * dr + di * di);
  }
  return h;
}

// dH/dx of the same form.
template <class R> __device__ __forceinline__ R voigt_dhdx(R a, R x) {
  const R x2 = x * x;
  const R z = M<R>::div(x2 - R(0.855), x2 + R(3.42));
  R d = R(-2) * x * M<R>::exp(-x2);
  if (z > R(0)) {
    const R den = x2 + R(3.42);
    const R dz = M<R>::div(R(2) * x * R(4.275), den * den);
    const R P = ((R(5.674) * z - R(9.207)) * z + R(4.421)) * z + R(0.1117);
    const R dP = (R(17.022) * z - R(18.414)) * z + R(4.421);
    const R f2 = R(1) + M<R>::div(R(21), x2), df2 = M<R>::div(R(-42), x2 * x);
    const R f3 = M<R>::div(a * R(1.0 / PI_D), x2 + R(1));
    const R df3 = M<R>::div(-f3 * R(2) * x, x2 + R(1));
    const R dq = dz * f2 * f3 * P + z * df2 * f3 * P + z * f2 * df3 * P + z * f2 * f3 * dP * dz;
    d += R(1.7724538509055160273) * dq;
  }
  return d;
}

// ---------------------------------------------------- atom velocity draw
// Sect. 3.3.3: rejection sampling of f(u) ~ exp(-u^2)/(a^2+(x-u)^2) with a
// two-piece Lorentzian envelope split at u0(x, log10 a) (the paper's fit,
// clamped at 0 where it goes negative); |x| >= 8: Gaussian of variance 1/2
// centred at 1/x; negative x by symmetry.
#pragma clang fp contract(on)
template <class R> __device__ __forceinline__ R u0_fit(R x, R la) {
  const R c0 = R(2.648963) + la * (R(2.014446) + la * R(0.351479));
  const R c1 = R(-4.058673) + la * (R(-3.675859) + la * R(-0.640003));
  const R c2 = R(3.017395) + la * (R(2.117133) + la * R(0.370294));
  const R c3 = R(-0.869789) + la * (R(-0.565886) + la * R(-0.096312));
  const R c4 = R(0.110987) + la * (R(0.070103) + la * R(0.011557));
  const R c5 = R(-0.005200) + la * (R(-0.003240) + la * R(-0.000519));
  return c0 + x * (c1 + x * (c2 + x * (c3 + x * (c4 + x * c5))));
}

// Rejection rounds allowed per draw; a packet that exhausts them stops
// with status stuck (never reached for finite x and a > 0).
constexpr uint32_t MAX_REJECT = 1u << 20;

// The draw's envelope at (x, a), then single rounds of it.  Contraction
// within a statement only (from u0_fit on), so that the same expressions
// give the same values wherever the functions are inlined (the
// one-round-per-pass transport and the looping sampler then draw identical
// velocities).
template <class R> struct UparEnv {
  R sg, xa, th0, u02, p1, s1, s2;
};

template <class R> __device__ __forceinline__ UparEnv<R> upar_env(R x, R a, R la) {
  UparEnv<R> e;
  e.sg = x < R(0) ? R(-1) : R(1);
  e.xa = fabs(x);
  R u0 = u0_fit(e.xa, la);
  u0 = u0 < R(0) ? R(0) : u0;
  e.th0 = M<R>::atan(M<R>::div(u0 - e.xa, a));
  const R e0 = M<R>::exp(-u0 * u0);
  const R hp = R(0.5 * PI_D);
  const R D = (R(1) - e0) * e.th0 + (R(1) + e0) * hp;
  e.p1 = M<R>::div(e.th0 + hp, D);
  e.u02 = u0 * u0;
  // float: one uniform picks the piece and, rescaled within it, the angle
  // (the same distribution with two uniforms per round, so that an event
  // whose draw ends by its second round fits in two Philox blocks); double:
  // three per round.
  // The scales (th0 + pi/2)/p1 and (pi/2 - th0)/(1 - p1) are D and D/e0
  // (1 - p1 = e0 (pi/2 - th0)/D); the second is not used when p1 is 1.
  e.s1 = D;
  e.s2 = e.p1 < R(1) ? M<R>::div(D, e0) : R(0);
  return e;
}

// One float round from its pair: r1 picks the piece and, rescaled within
// it, the angle; r3 accepts or rejects.
__device__ __forceinline__ bool upar_try_pair(const UparEnv<float> &e, float a, float r1, float r3, float *out) {
  const float hp = float(0.5 * PI_D);
  float th, lim;
  if (r1 < e.p1) {
    th = -hp + r1 * e.s1;
    lim = 0.0f;
  } else {
    th = e.th0 + (r1 - e.p1) * e.s2;
    lim = e.u02;
  }
  const float u = e.xa + a * M<float>::tan(th);
  *out = e.sg * u;
  return r3 < M<float>::exp(lim - u * u);
}

// Round `it` of the rejection draw (|x| < 8): true when it accepts, with
// the velocity in *out.
template <class R>
__device__ __forceinline__ bool upar_try(const UparEnv<R> &e, R a, EventRng<R> &rng, uint32_t it, R *out) {
  if constexpr (sizeof(R) == 4) {
    float r1, r3;
    rng.round(it, &r1, &r3);
    return upar_try_pair(e, a, r1, r3, out);
  } else {
    const R hp = R(0.5 * PI_D);
    R th, lim;
    const R r1 = rng.u(J_REJ + 3 * it);
    const R r2 = rng.u(J_REJ + 3 * it + 1);
    const R r3 = rng.u(J_REJ + 3 * it + 2);
    if (r1 < e.p1) {
      th = -hp + r2 * (e.th0 + hp);
      lim = R(0);
    } else {
      th = e.th0 + r2 * (hp - e.th0);
      lim = e.u02;
    }
    const R u = e.xa + a * M<R>::tan(th);
    *out = e.sg * u;
    return r3 < M<R>::exp(lim - u * u);
  }
}

// The |x| >= 8 branch: Gaussian of variance 1/2 centred at 1/x.
template <class R> __device__ __forceinline__ R upar_gauss(R x, EventRng<R> &rng) {
  R s, c;
  M<R>::sincos2pi(rng.u(J_GAUSS2), &s, &c);
  return M<R>::div(R(1), x) + M<R>::sqrt(-M<R>::log(rng.u(J_GAUSS1))) * c;
}
#pragma clang fp contract(fast)

template <class R>
__device__ __forceinline__ bool sample_upar(R x, R a, R la, EventRng<R> &rng, R *out) {
  if (fabs(x) >= R(8)) {
    *out = upar_gauss(x, rng);
    return true;
  }
  const UparEnv<R> e = upar_env(x, a, la);
  uint32_t it = 0;
  if constexpr (sizeof(R) == 4) {
    // float: the first two rounds side by side (their draws are in blocks 0
    // and 1, which the event computes anyway): a wave in which a few lanes
    // reject the first round would run the second for them alone
    float r1, r3, q1, q3, v0, v1;
    rng.round(0, &r1, &r3);
    rng.round(1, &q1, &q3);
    const bool a0 = upar_try_pair(e, a, r1, r3, &v0);
    const bool a1 = upar_try_pair(e, a, q1, q3, &v1);
    if (a0 || a1) {
      *out = a0 ? v0 : v1;
      return true;
    }
    // then two rounds per block
    for (it = 2; it < MAX_REJECT; it += 2) {
      const uint4 w = rng.block(1 + it / 2);
      if (upar_try_pair(e, a, EventRng<float>::top(w.x), EventRng<float>::top(w.y), out)) return true;
      if (upar_try_pair(e, a, EventRng<float>::top(w.z), EventRng<float>::top(w.w), out)) return true;
    }
  } else {
    for (; it < MAX_REJECT; ++it) {
      if (upar_try(e, a, rng, it, out)) return true;
    }
  }
  *out = R(0);
  return false;
}

// Round `it` alone of the same draw, the envelope rebuilt from x and a
// (exact functions of the packet's state): true and *out when round `it`
// accepts (the |x| >= 8 Gaussian accepts at round 0).  Running rounds 0, 1,
// 2, ... one per call gives sample_upar's result with the same draws, so a
// lane whose round is rejected can take its next round at a later pass of
// the transport loop, together with the first rounds of other lanes,
// instead of holding its wave in a loop of its own.
template <class R>
__device__ __forceinline__ bool upar_round(R x, R a, R la, EventRng<R> &rng, uint32_t it, R *out) {
  if (fabs(x) >= R(8)) {
    *out = upar_gauss(x, rng);
    return true;
  }
  return upar_try(upar_env(x, a, la), a, rng, it, out);
}

// Sect. 3.3.1 inverse CDFs.  Both are cbrt(A + B) - cbrt(A - B) with
// A = sqrt(B^2 + C): core B = 6 (2r - 1), C = 11^3/27; wing B = 2 (2r - 1)
// (= 4r - 2 exactly), C = 1.  One evaluation with the lane's constants, so
// that a wave holding core and wing scatterings runs the cube roots once.
template <class R> __device__ __forceinline__ R mu_dipole(R r, bool core) {
  const R B = (core ? R(6) : R(2)) * (R(2) * r - R(1));
  const R A = M<R>::sqrt(B * B + (core ? R(11.0 * 11.0 * 11.0 / 27.0) : R(1)));
  if constexpr (sizeof(R) == 4) {
    // (A + B)(A - B) = C, so cbrt(A - B) = cbrt(C) / cbrt(A + B), with
    // cbrt(C) = 11/3 (core) or 1 (wing): one cube root and a reciprocal
    const R y = M<R>::cbrt_pos(A + B);
    return y - M<R>::div(core ? R(11.0 / 3.0) : R(1), y);
  } else {
    return M<R>::cbrt_pos(A + B) - M<R>::cbrt_pos(A - B);
  }
}
// Henyey-Greenstein inverse, with the square of the exact inverse.
template <class R> __device__ __forceinline__ R mu_hg(R r, R g) {
  if (g == R(0)) return R(2) * r - R(1);
  const R t = M<R>::div(R(1) - g * g, R(1) - g + R(2) * g * r);
  return M<R>::div(R(1) + g * g - t * t, R(2) * g);
}
template <class R> __device__ __forceinline__ R p_core(R mu) { return R(11.0 / 24.0) + R(3.0 / 24.0) * mu * mu; }
template <class R> __device__ __forceinline__ R p_wing(R mu) { return R(3.0 / 8.0) * (R(1) + mu * mu); }
template <class R> __device__ __forceinline__ R p_hg(R mu, R g) {
  const R d = R(1) + g * g - R(2) * g * mu;
  return M<R>::div(R(0.5) * (R(1) - g * g), d * M<R>::sqrt(d));
}

// Orthonormal pair perpendicular to k: e1 = normalize(k x z) (k x x when
// |k_z| > 0.9), e2 = k x e1.
template <class R> __device__ __forceinline__ void perp_basis(const R k[3], R e1[3], R e2[3]) {
  R c0, c1, c2;
  if (fabs(k[2]) > R(0.9)) { c0 = R(0); c1 = k[2]; c2 = -k[1]; }
  else { c0 = k[1]; c1 = -k[0]; c2 = R(0); }
  const R n = M<R>::rsqrt(c0 * c0 + c1 * c1 + c2 * c2);
  e1[0] = c0 * n; e1[1] = c1 * n; e1[2] = c2 * n;
  e2[0] = k[1] * e1[2] - k[2] * e1[1];
  e2[1] = k[2] * e1[0] - k[0] * e1[2];
  e2[2] = k[0] * e1[1] - k[1] * e1[0];
}

// ------------------------------------------------------------- geometry
// All traversal arithmetic is double, uncontracted, with the fma written
// out, so that the cell sequence is an exact function of the inputs.
#pragma clang fp contract(off)

struct Cell {
  int leaf;        // leaf index
  int level;       // leaf level
  int ox, oy, oz;  // origin in deepest-level integer units
};

// Distance along k from p to the face through which the packet leaves the
// cell; exit axes are flagged in *emask.  With kinv (1/k, float path only)
// the per-axis distances are products instead of correctly rounded
// quotients.
__device__ __forceinline__ double exit_dist(const Cell &c, int L, const double p[3],
                                            const double k[3], double face[3], double lo[3],
                                            double hi[3], int *emask, const double *kinv = nullptr) {
  const double inv = ldexp(1.0, -L);
  const int s = 1 << (L - c.level);
  const int o[3] = {c.ox, c.oy, c.oz};
  double td[3];
  double t = __builtin_inf();
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    lo[d] = (double)o[d] * inv;
    hi[d] = (double)(o[d] + s) * inv;
    if (k[d] > 0.0) { face[d] = hi[d]; td[d] = kinv ? (face[d] - p[d]) * kinv[d] : (face[d] - p[d]) / k[d]; }
    else if (k[d] < 0.0) { face[d] = lo[d]; td[d] = kinv ? (face[d] - p[d]) * kinv[d] : (face[d] - p[d]) / k[d]; }
    else { face[d] = 0.0; td[d] = __builtin_inf(); }
    t = td[d] < t ? td[d] : t;
  }
  if (t < 0.0) t = 0.0;
  int m = 0;
#pragma unroll
  for (int d = 0; d < 3; ++d) m |= (td[d] <= t) ? (1 << d) : 0;
  *emask = m;
  return t;
}

// Bounds of cell c, as exit_dist computes them.
__device__ __forceinline__ void cell_bounds(const Cell &c, int L, double lo[3], double hi[3]) {
  const double inv = ldexp(1.0, -L);
  const int s = 1 << (L - c.level);
  const int o[3] = {c.ox, c.oy, c.oz};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    lo[d] = (double)o[d] * inv;
    hi[d] = (double)(o[d] + s) * inv;
  }
}

// Distance from p (inside cell c) to the nearest face of the cell, shrunk by
// 2^-40: no ray from p leaves the cell sooner than this, whatever its
// direction, with exit_dist's rounding (which divides the same face - p
// differences by |k_d| <= 1 + 2^-52) included.
__device__ __forceinline__ double inner_dist(const double lo[3], const double hi[3], const double p[3]) {
  double m = __builtin_inf();
#pragma unroll
  for (int d = 0; d < 3; ++d) m = fmin(m, fmin(p[d] - lo[d], hi[d] - p[d]));
  return fmax(m, 0.0) * (1.0 - 0x1p-40);
}
__device__ __forceinline__ double inner_dist(const Cell &c, int L, const double p[3]) {
  double lo[3], hi[3];
  cell_bounds(c, L, lo, hi);
  return inner_dist(lo, hi, p);
}

// The point where the packet leaves: exit axes snapped onto the face, the
// others advanced by one fma and clamped into the cell.
__device__ __forceinline__ void exit_point(double t, int emask, const double p[3], const double k[3],
                                           const double face[3], const double lo[3],
                                           const double hi[3], double pn[3]) {
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (emask & (1 << d)) pn[d] = face[d];
    else {
      const double q = fma(t, k[d], p[d]);
      pn[d] = fmin(fmax(q, lo[d]), hi[d]);
    }
  }
}

// Distance along k to the domain border (Sect. 4 domain classes).
__device__ __forceinline__ double domain_dist(int kind, const double dom[4], const double p[3],
                                              const double k[3]) {
  double t = __builtin_inf();
  if (kind == DOM_BOX) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      double td = __builtin_inf();
      if (k[d] > 0.0) td = (1.0 - p[d]) / k[d];
      else if (k[d] < 0.0) td = (0.0 - p[d]) / k[d];
      t = td < t ? td : t;
    }
  } else if (kind == DOM_SLAB_Z) {
    if (k[2] > 0.0) t = ((dom[0] + dom[1]) - p[2]) / k[2];
    else if (k[2] < 0.0) t = ((dom[0] - dom[1]) - p[2]) / k[2];
  } else {
    const double dx = p[0] - dom[0], dy = p[1] - dom[1], dz = p[2] - dom[2];
    const double R = dom[3];
    const double b = dx * k[0] + dy * k[1] + dz * k[2];
    const double q = dx * dx + dy * dy + dz * dz - R * R;
    const double disc = b * b - q;
    if (disc < 0.0) return 0.0;
    const double sq = sqrt(disc);
    t = (b > 0.0) ? -q / (b + sq) : -b + sq;
  }
  return t < 0.0 ? 0.0 : t;
}

__device__ __forceinline__ void wrap_slab(int kind, double p[3], const double k[3]) {
  if (kind != DOM_SLAB_Z) return;
#pragma unroll
  for (int d = 0; d < 2; ++d) {
    if (k[d] > 0.0 && p[d] >= 1.0) p[d] = 0.0;
    else if (k[d] < 0.0 && p[d] <= 0.0) p[d] = 1.0;
  }
}

// Integer point location: floor(p 2^L) along k_d >= 0, ceil(p 2^L) - 1
// otherwise; false if outside the unit cube.
__device__ __forceinline__ bool int_coords(int L, const double p[3], const double k[3], int X[3]) {
  const double sc = (double)(1 << L);
  const int side = 1 << L;
  bool in = true;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double s = p[d] * sc;
    const double f = (k[d] >= 0.0) ? floor(s) : ceil(s) - 1.0;
    in = in && (f >= 0.0) && (f < (double)side);
    X[d] = in ? (int)f : 0;
  }
  return in;
}

// Descend the breadth-first node array from `node` at `level` to the leaf
// holding integer point X, recording the nodes passed in the per-lane LDS
// stack (stack[level*stride]).
__device__ __forceinline__ void descend(const int32_t *__restrict__ nodes, int L, int node, int level,
                                        const int X[3], int *stack, int stride, Cell &c) {
  if (L == 0) {  // a single leaf covers the cube
    c.leaf = 0; c.level = 0; c.ox = c.oy = c.oz = 0;
    return;
  }
  while (true) {
    stack[level * stride] = node;
    const int sh = L - level - 1;
    const int oct = ((X[0] >> sh) & 1) | (((X[1] >> sh) & 1) << 1) | (((X[2] >> sh) & 1) << 2);
    const int ch = nodes[node * 8 + oct];
    ++level;
    if (ch < 0) {
      c.leaf = -ch - 1;
      c.level = level;
      const int clr = ~((1 << (L - level)) - 1);
      c.ox = X[0] & clr; c.oy = X[1] & clr; c.oz = X[2] & clr;
      return;
    }
    node = ch;
  }
}

// Descend to the leaf holding X from its ancestor at level `from` (0: the
// root).  Above the level-T table the start is X's entry in the table:
// either the leaf covering X's level-T cell (a leaf of level <= T) or the
// node there; below it, the ancestor recorded in the LDS stack.  With a
// table the stack holds the nodes of levels T and deeper on the way to the
// current leaf, and levels below T are never read (a move that leaves the
// level-T cell starts from the table again).
__device__ __forceinline__ void descend_from(const int32_t *__restrict__ nodes, const int32_t *__restrict__ top,
                                             int T, int L, int from, const int X[3], int *stack, int stride,
                                             Cell &c) {
  int node = 0, level = 0;
  if (top != nullptr && from < T) {
    const int sh = L - T;
    const int e = top[((X[2] >> sh) << (2 * T)) | ((X[1] >> sh) << T) | (X[0] >> sh)];
    if (e < 0) {
      const int v = -e - 1;
      c.leaf = v & ((1 << TOP_LEVEL_SHIFT) - 1);
      c.level = v >> TOP_LEVEL_SHIFT;
      const int clr = ~((1 << (L - c.level)) - 1);
      c.ox = X[0] & clr; c.oy = X[1] & clr; c.oz = X[2] & clr;
      return;
    }
    node = e;
    level = T;
  } else if (from > 0) {
    node = stack[from * stride];
    level = from;
  }
  descend(nodes, L, node, level, X, stack, stride, c);
}

// The leaf holding X.
__device__ __forceinline__ void locate(const int32_t *__restrict__ nodes, const int32_t *__restrict__ top, int T,
                                       int L, const int X[3], int *stack, int stride, Cell &c) {
  descend_from(nodes, top, T, L, 0, X, stack, stride, c);
}

// Move to the leaf holding X after leaving cell c: restart the descent at
// the deepest common ancestor of c and X.
__device__ __forceinline__ void relocate(const int32_t *__restrict__ nodes, const int32_t *__restrict__ top, int T,
                                         int L, const int X[3], int *stack, int stride, Cell &c) {
  const unsigned diff = (unsigned)((X[0] ^ c.ox) | (X[1] ^ c.oy) | (X[2] ^ c.oz));
  if (diff == 0u) return;
  const int b = 31 - __builtin_clz(diff);
  descend_from(nodes, top, T, L, L - 1 - b, X, stack, stride, c);   // from the common ancestor's level
}

__device__ __forceinline__ void locate(const ProblemK &pb, const int X[3], int *stack, int stride, Cell &c) {
  locate(pb.nodes, pb.top, pb.top_level, pb.L, X, stack, stride, c);
}
__device__ __forceinline__ void relocate(const ProblemK &pb, const int X[3], int *stack, int stride, Cell &c) {
  relocate(pb.nodes, pb.top, pb.top_level, pb.L, X, stack, stride, c);
}

#pragma clang fp contract(fast)

// ------------------------------------------------------------- leaf data
// bnd != 0 marks a leaf that reaches the domain border (or lies outside
// the domain); from a leaf strictly inside, every ray leaves the leaf
// before the domain, so its domain distance is never the smaller one.
template <class R> struct LeafRec {
  R nl, irho, kd, ux, uy, uz, bnd;
  R lg;   // log10(irho) (double records; the float path takes its own logarithm)
};

template <class R>
__device__ __forceinline__ LeafRec<R> load_leaf(const void *leaves, int i) {
  LeafRec<R> r;
  const R *p = (const R *)leaves + (size_t)i * LEAF_STRIDE;
  if constexpr (sizeof(R) == 4) {
    const float4 a = *(const float4 *)p;
    const float4 b = *(const float4 *)(p + 4);
    r.nl = a.x; r.irho = a.y; r.kd = a.z; r.ux = a.w; r.uy = b.x; r.uz = b.y; r.bnd = b.z; r.lg = 0.0f;
  } else {
    const double2 a = *(const double2 *)p;
    const double2 b = *(const double2 *)(p + 2);
    const double2 c = *(const double2 *)(p + 4);
    const double2 d = *(const double2 *)(p + 6);
    r.nl = a.x; r.irho = a.y; r.kd = b.x; r.ux = b.y; r.uy = c.x; r.uz = c.y; r.bnd = d.x; r.lg = d.y;
  }
  return r;
}

// Domain distance where it can matter (see LeafRec::bnd).
template <class R>
__device__ __forceinline__ double domain_dist_leaf(const LeafRec<R> &lf, int kind, const double dom[4],
                                                   const double p[3], const double k[3]) {
  return lf.bnd != R(0) ? domain_dist(kind, dom, p, k) : __builtin_inf();
}

// Opacity (times box size) of a leaf for a packet at x_ext along k; NL
// bounds the number of lines (1 for single-line problems, MAX_LINES else).
template <class R, int NL = MAX_LINES> struct Opac {
  R kd, kl[NL], x[NL], ktot, w;
};

// The numerator delta + s x_ext - w is formed in double in both precisions:
// for gas moving many thermal widths it is a small difference of large
// terms, and float would lose the core of the profile.
template <class R, int NL>
__device__ __forceinline__ void opacity(const ProblemK &pb, const LeafRec<R> &lf, double x_ext, const R k[3],
                                        Opac<R, NL> &o) {
  const double wd = (double)k[0] * (double)lf.ux + (double)k[1] * (double)lf.uy + (double)k[2] * (double)lf.uz;
  o.w = (R)wd;
  const R inv_den = M<R>::div(R(1), R(1) + cst<R>(pb.b_ref, pb.b_ref_f) * o.w);
  o.kd = lf.kd;
  o.ktot = lf.kd;
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    o.x[i] = R(0);
    o.kl[i] = R(0);
    if (NL == 1 || i < pb.n_lines) {
      const LineK &ln = pb.lines[i];
      o.x[i] = (R)(ln.delta + ln.s * x_ext - wd) * lf.irho * cst<R>(ln.inv_mu, ln.f.inv_mu) * inv_den;
      const R a = cst<R>(ln.alpha, ln.f.alpha) * lf.irho;
      R H;
      // the accurate H is a double-path option (the float kernels stay free of it)
      if constexpr (sizeof(R) == 8)
        H = pb.voigt_exact ? voigt_h_exact(a, o.x[i]) : voigt_h<R>(a, o.x[i]);
      else
        H = voigt_h<R>(a, o.x[i]);
      o.kl[i] = lf.nl * cst<R>(ln.kfac, ln.f.kfac) * H;
      o.ktot += o.kl[i];
    }
  }
}

// Core-skipping (Sect. 3.2.1): while a packet sits deep in the line core of
// a cell that is optically thick even well off line centre, the scattering
// atom's perpendicular velocity is drawn with |u_perp| >= x_crit, which moves
// the packet to the wing in one step instead of many local core scatterings.
// x_crit comes from the cell: tau_c = n_X sigma0(T) h is its line-centre
// optical depth across the edge; x_crit is the smaller of
// sqrt(ln(tau_c / skip_tau)) (where the Gaussian core of the cell is still
// skip_tau thick) and skip_frac (a tau_c)^(1/3) (a fraction of the wing
// frequency at which a medium of the cell's depth lets packets out).
// Returns x_crit^2 while |x| < x_crit, else 0 (the unbiased draw).
template <class R>
__device__ __forceinline__ R core_skip_x2(const ProblemK &pb, const LineK &ln, const LeafRec<R> &lf, int level,
                                          R a, R x) {
  const R tc = lf.nl * cst<R>(ln.kfac, ln.f.kfac) * (R)ldexp(1.0, -level);
  const R ts = R(pb.skip_tau);
  if (!(tc > ts)) return R(0);
  const R xt2 = M<R>::log(M<R>::div(tc, ts));
  const R xw = R(pb.skip_frac) * M<R>::cbrt(a * tc);
  const R x2 = fmin(xt2, xw * xw);
  return x * x < x2 ? x2 : R(0);
}

}  // namespace rmc
