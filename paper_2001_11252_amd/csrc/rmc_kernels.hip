// rmc_kernels.hip -- gfx950 kernels of the resonant-line Monte Carlo path.
//
// k_transport   persistent per-packet propagation loop (Sect. 3, 3.2, 4.3)
//               with peel-off toward observers at each emission and
//               scattering (Sect. 5.1); one packet per lane, lanes of a
//               wave refilled from a global queue with one atomic per wave
//               (ballot + mbcnt compaction of the idle lanes).  Each
//               peel-off ray is decided in the scattering's own leaf or
//               queued in the wave's region of the peel-off queue.
// k_peel_drain  ray-cast pass over the queued peel-off rays after each
//               transport launch (lanes refilled per ray), k_peel_reset
//               its bookkeeping
// k_trace       deterministic cell sequence of rays (probe)
// k_tau         optical depth of rays to the domain border (probe)
// k_image_fwd   peel-off image of fixed rays
// k_image_bwd   its adjoint with respect to per-leaf n_HI, kappa_d, v_los
// k_hist        spectrum of escaped packets
#include <mutex>

#include "rmc_device.h"
#include "rmc_launch.h"

namespace rmc {

// exp(-tau) is exactly zero (round to nearest) from these optical depths
// on: a ray may stop integrating there without changing any deposit.
template <class R> struct TauCut;
template <> struct TauCut<double> { static constexpr double v = 746.0; };
template <> struct TauCut<float> { static constexpr double v = 104.0; };

__device__ __forceinline__ void atomic_add_real(float *p, float v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void atomic_add_real(double *p, double v) { unsafeAtomicAdd(p, v); }

// --------------------------------------------------------------- ray cast
// A point strictly inside a cell is located in that cell whatever the
// direction, so a ray starting there needs no descent from the root.
__device__ __forceinline__ bool strictly_inside(const Cell &c, int L, const double p[3]) {
  const double inv = ldexp(1.0, -L);
  const int s = 1 << (L - c.level);
  const int o[3] = {c.ox, c.oy, c.oz};
  bool in = true;
#pragma unroll
  for (int d = 0; d < 3; ++d) in = in && (p[d] > (double)o[d] * inv) && (p[d] < (double)(o[d] + s) * inv);
  return in;
}

// Where a peel-off ray may start: the packet's current cell, its leaf
// record and the LDS stack of its ancestors.
template <class R> struct StartCell {
  const Cell *c;
  const LeafRec<R> *lf;
  const int *stk;
};

// Walks a ray at fixed x_ext from p (inside cell c) leaf by leaf, adding
// kappa * segment to tau, until it reaches the domain border or tau >=
// tau_cut.  steps counts the leaves crossed so far (at most MAX_CROSS).  With
// borrowed, sc lends the first leaf's record and ancestor stack.
template <class R, int NL>
__device__ double ray_walk(const ProblemK &pb, double p[3], const double k[3], double x_ext, double tau,
                           uint32_t steps, double tau_cut, int *stk, int stride, uint32_t *ncross, Cell &c,
                           const StartCell<R> *sc, bool borrowed, const double *kinv = nullptr) {
  const R kr[3] = {(R)k[0], (R)k[1], (R)k[2]};
  bool first = borrowed;
  bool start = true;
  for (; steps < MAX_CROSS; ++steps) {
    const LeafRec<R> lf = first ? *sc->lf : load_leaf<R>(pb.leaves, c.leaf);
    Opac<R, NL> o;
    opacity(pb, lf, x_ext, kr, o);
    // Only the start point can lie inside a leaf: later leaves are entered
    // on a face (inner distance 0, where the test is tau >= tau_cut, which
    // the previous leaf already ruled out).
    if (start && lf.bnd == R(0)) {
      if (tau + (double)o.ktot * inner_dist(c, pb.L, p) >= tau_cut) {
        // the cut is reached inside this leaf whatever the exit distance
        ++*ncross;
        tau = tau_cut;
        break;
      }
    }
    start = false;
    double face[3], lo[3], hi[3];
    int em;
    const double te = exit_dist(c, pb.L, p, k, face, lo, hi, &em, kinv);
    const double td = domain_dist_leaf(lf, pb.domain, pb.dom, p, k);
    ++*ncross;
    if (td <= te) {
      tau += (double)o.ktot * td;
      break;
    }
    tau += (double)o.ktot * te;
    if (tau >= tau_cut) break;
    double pn[3];
    exit_point(te, em, p, k, face, lo, hi, pn);
    p[0] = pn[0]; p[1] = pn[1]; p[2] = pn[2];
    wrap_slab(pb.domain, p, k);
    int X[3];
    if (!int_coords(pb.L, p, k, X)) break;
    if (first) {
      // first move out of the borrowed cell: copy its ancestors
      for (int l = 0; l < c.level; ++l) stk[l * stride] = sc->stk[l * stride];
    }
    first = false;
    relocate(pb, X, stk, stride, c);
  }
  return tau;
}

// Optical depth from p along k to the domain border at fixed x_ext (the
// peel-off integral); stops once tau >= tau_cut.  Uses its own LDS stack.
template <class R, int NL = MAX_LINES>
__device__ double ray_tau(const ProblemK &pb, const double p0[3], const double k[3], double x_ext,
                          double tau_cut, int *stk, int stride, uint32_t *ncross,
                          const StartCell<R> *sc, const double *kinv = nullptr) {
  double p[3] = {p0[0], p0[1], p0[2]};
  Cell c;
  const bool reuse = sc && strictly_inside(*sc->c, pb.L, p);
  if (reuse) {
    c = *sc->c;
  } else {
    int X[3];
    if (!int_coords(pb.L, p, k, X)) return 0.0;
    locate(pb, X, stk, stride, c);
  }
  return ray_walk<R, NL>(pb, p, k, x_ext, 0.0, 0u, tau_cut, stk, stride, ncross, c, sc, reuse, kinv);
}

// Pixel of position p in observer ob's image, -1 outside.  The double path
// bins exactly as the oracle does (divide by the span); the float path
// multiplies by the precomputed cells per unit (a point within an ulp of a
// pixel edge may fall on the other side).
template <bool FAST = false>
__device__ __forceinline__ int pixel_of(const ObsK &ob, const double p[3]) {
#pragma clang fp contract(off)
  const double q0 = p[0] - 0.5, q1 = p[1] - 0.5, q2 = p[2] - 0.5;
  const double u = q0 * ob.e1[0] + q1 * ob.e1[1] + q2 * ob.e1[2];
  const double v = q0 * ob.e2[0] + q1 * ob.e2[1] + q2 * ob.e2[2];
  const double fu = FAST ? (u - ob.u0) * ob.su : (u - ob.u0) / ob.uspan * ob.nx;
  const double fv = FAST ? (v - ob.v0) * ob.sv : (v - ob.v0) / ob.vspan * ob.ny;
  if (!(fu >= 0.0 && fu < ob.nx && fv >= 0.0 && fv < ob.ny)) return -1;
  const int ix = (int)floor(fu), iy = (int)floor(fv);
  if (ix >= ob.nx || iy >= ob.ny) return -1;
  return iy * ob.nx + ix;
}

template <bool FAST = false>
__device__ __forceinline__ int bin_of(const ObsK &ob, double x) {
#pragma clang fp contract(off)
  const double fb = FAST ? (x - ob.x_min) * ob.sx : (x - ob.x_min) / ob.xspan * ob.nbins;
  if (!(fb >= 0.0 && fb < ob.nbins)) return -1;
  const int b = (int)floor(fb);
  return b >= ob.nbins ? -1 : b;
}

struct LaneCount {
  uint32_t cross, peel_rays, peel_cross, peel_drop, dust_scat;
};

// What a scattering (or emission) needs to be redone toward an observer.
template <class R> struct PeelSrc {
  int kind;        // 0 emission, 1 line, 2 dust, 3 fluorescent re-emission
  R kin[3];
  R x;             // emission / dust: x_ext of the packet; line: cell-frame x
  R w;             // k_in . u of the cell (dust)
  R U[3];          // atom velocity / v_th of the line (line)
  R bc;            // v_th,line,cell / c (line)
  R rho;           // sqrt(T/T_ref) (line)
  R irho;          // 1/rho (line)
  int line, core;  // (fluorescent: core holds the channel)
  R ux, uy, uz;    // cell bulk velocity / v_th,ref
};

// Where a transport wave queues its deferred peel-off rays: its own region
// of the queue and the region's fill count, kept in LDS (one per wave, so
// no global atomics).  The wave stops taking events before the region
// could overflow, so a push always finds room.
template <class R> struct PeelSink {
  PeelJob<R> *region;
  int *count;
  uint32_t cap;
  unsigned long long *lost;   // pushes that found no room (never expected)
};

// First-leaf test of a peel-off ray toward observer ob from p, in the
// scattering's own leaf (its record is in the lane's registers; the leaf
// lies strictly inside the domain): true if the optical depth to the exit
// face along k_obs already reaches the cut, where exp(-tau) is zero and no
// deposit changes.  Without EXIT (float path) that distance alone is
// computed; with EXIT (double path, deferred rays) the nearest face is
// tried first, and a ray that goes on gets where it leaves the leaf (q,
// wrapped through periodic borders) and the optical depth so far.
template <class R, int NL, bool EXIT>
__device__ __forceinline__ bool peel_first_leaf(const ProblemK &pb, const double p[3], const ObsK &ob,
                                                const R ko[3], R xo, const StartCell<R> *sc, double q[3],
                                                double *qtau) {
  Opac<R, NL> o;
  opacity(pb, *sc->lf, (double)xo, ko, o);
  const double kt = (double)o.ktot;
  if constexpr (!EXIT) {
    // the distance to the leaf's face ahead along k_obs, as exit_dist
    // computes it (the observer's direction is uniform across the wave)
    const double inv = ldexp(1.0, -pb.L);
    const int sz = 1 << (pb.L - sc->c->level);
    const int o3[3] = {sc->c->ox, sc->c->oy, sc->c->oz};
    double te = __builtin_inf();
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      if (ob.k[d] != 0.0) {
        const double f = (double)(ob.k[d] > 0.0 ? o3[d] + sz : o3[d]) * inv;
        const double t = (f - p[d]) * ob.kinv[d];
        te = t < te ? t : te;
      }
    }
    return kt * (te < 0.0 ? 0.0 : te) >= TauCut<R>::v;
  }
  if (kt * inner_dist(*sc->c, pb.L, p) >= TauCut<R>::v) return true;
  double face[3], lo[3], hi[3];
  int em;
  const double te = exit_dist(*sc->c, pb.L, p, ob.k, face, lo, hi, &em, sizeof(R) == 4 ? ob.kinv : nullptr);
  const double t1 = kt * te;
  if (t1 >= TauCut<R>::v) return true;
  if constexpr (EXIT) {
    exit_point(te, em, p, ob.k, face, lo, hi, q);
    wrap_slab(pb.domain, q, ob.k);
    *qtau = t1;
  }
  return false;
}

// Queue a peel-off ray for the ray-cast pass, which makes every deposit:
// the float path queues it from its start (the pass walks the first leaf
// again, which keeps this kernel's registers low enough for four waves per
// SIMD), the double path, when its first leaf was tested, from where it
// leaves that leaf with the optical depth so far (qsteps = 1).  One LDS
// atomic per wave reserves the slots of the lanes pushing here.
template <class R>
__device__ __forceinline__ void peel_push(const ProblemK &pb, const double q[3], double qtau, uint32_t qsteps,
                                          R xo, R weight, size_t elem, int oi, const PeelSink<R> &snk) {
  const unsigned long long m = __ballot(true);
  const int lane = __lane_id();
  const int leader = __ffsll((long long)m) - 1;
  int base = 0;
  if (lane == leader) base = atomicAdd(snk.count, __popcll(m));
  base = __shfl(base, leader);
  const uint32_t slot = (uint32_t)base + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
  if (slot < snk.cap) {
    PeelJob<R> &j = snk.region[slot];
    j.p[0] = q[0]; j.p[1] = q[1]; j.p[2] = q[2];
    j.x = xo;
    j.weight = weight;
    j.dst = (unsigned long long)elem | ((unsigned long long)oi << PQ_OBS_SHIFT) |
            ((unsigned long long)pb.index << PQ_PROB_SHIFT);
    if constexpr (sizeof(R) == 8) {
      j.tau = qtau;
      j.steps = qsteps;
    }
  } else {
    atomicAdd(snk.lost, 1ull);
  }
}

// Peel-off of one event toward every observer (Sect. 5.1).  A ray from a
// leaf strictly inside the domain is first tested in that leaf, before its
// weight, pixel and bin are computed: most rays from optically thick gas
// end there with no deposit.  A ray that goes on is binned (deposits
// outside the cube are dropped and counted) and, with DEFER, queued for the
// ray-cast pass (peel_push), else walked here; the float path queues it
// unbinned, and the pass bins it.  Emission rays (sc null: no
// leaf located yet) and rays from leaves the domain border may cut skip the
// first-leaf test.
template <class R, bool DEFER, int NL>
__device__ void peel_all(const ProblemK &pb, const double p[3], const PeelSrc<R> &s, int *stk,
                         int stride, LaneCount &cnt, const PeelSink<R> &snk, const StartCell<R> *sc = nullptr) {
  for (int oi = 0; oi < pb.n_obs; ++oi) {
    const ObsK &ob = pb.obs[oi];
    const R ko[3] = {cst<R>(ob.k[0], ob.kf[0]), cst<R>(ob.k[1], ob.kf[1]), cst<R>(ob.k[2], ob.kf[2])};
    R xo, mu = R(0);
    if (s.kind == 0) {
      xo = s.x;
    } else if (NL > 1 && s.kind == 3) {
      // fluorescent re-emission: isotropic, at the channel's rest frequency
      // in the atom frame, then through the cell's velocity
      const LineK &ln = pb.lines[s.line];
      const R ba = s.bc * (ko[0] * s.U[0] + ko[1] * s.U[1] + ko[2] * s.U[2]);
      const R bw = cst<R>(pb.b_ref, pb.b_ref_f) * (ko[0] * s.ux + ko[1] * s.uy + ko[2] * s.uz);
      xo = cst<R>(ln.xf0[s.core], ln.f.xf0[s.core]) + M<R>::div(cst<R>(ln.sf[s.core], ln.f.sf[s.core]) * (ba + bw + ba * bw), cst<R>(pb.b_ref, pb.b_ref_f));
    } else if (s.kind == 1) {
      const LineK &ln = pb.lines[s.line];
      mu = s.kin[0] * ko[0] + s.kin[1] * ko[1] + s.kin[2] * ko[2];
      const R dkU = (ko[0] - s.kin[0]) * s.U[0] + (ko[1] - s.kin[1]) * s.U[1] + (ko[2] - s.kin[2]) * s.U[2];
      const R g1 = R(1) + s.bc * s.x;
      const R Rr = ln.recoil ? (R(1) - mu) * cst<R>(ln.rec, ln.f.rec) * g1 : R(0);
      R xc;
      if constexpr (sizeof(R) == 4) {
        // Rr < 3e-8 for any line and scatterer (h nu <= 13.6 eV, m c^2 >=
        // 938 MeV): 1/(1 + Rr) = 1 - Rr to float precision, and
        // Rr/bc = Rr irho / (b_ref mu)
        xc = (s.x + g1 * dkU - Rr * cst<R>(ln.ibmu, ln.f.ibmu) * s.irho) * (R(1) - Rr);
      } else {
        xc = M<R>::div(s.x + g1 * dkU - M<R>::div(Rr, s.bc), R(1) + Rr);
      }
      const R wo = ko[0] * s.ux + ko[1] * s.uy + ko[2] * s.uz;
      xo = (-cst<R>(ln.delta, ln.f.delta) + cst<R>(ln.mu, ln.f.mu) * s.rho * xc * (R(1) + cst<R>(pb.b_ref, pb.b_ref_f) * wo) + wo) * cst<R>(ln.inv_s, ln.f.inv_s);
    } else {
      mu = s.kin[0] * ko[0] + s.kin[1] * ko[1] + s.kin[2] * ko[2];
      const R wo = ko[0] * s.ux + ko[1] * s.uy + ko[2] * s.uz;
      const R b = cst<R>(pb.b_ref, pb.b_ref_f);
      xo = M<R>::div(s.x + wo + b * s.x * wo - s.w, R(1) + b * s.w);
    }
    ++cnt.peel_rays;
    constexpr bool EXIT = DEFER && sizeof(R) == 8;
    double q[3] = {p[0], p[1], p[2]}, qtau = 0.0;
    uint32_t qsteps = 0;
    if (sc && sc->lf->bnd == R(0)) {
      if (peel_first_leaf<R, NL, EXIT>(pb, p, ob, ko, xo, sc, q, &qtau)) {
        ++cnt.peel_cross;
        continue;
      }
      qsteps = EXIT ? 1u : 0u;
    }
    R weight;
    if (s.kind == 0 || (NL > 1 && s.kind == 3)) {
      weight = R(1.0 / (4.0 * PI_D));
    } else if (s.kind == 1) {
      const LineK &ln = pb.lines[s.line];
      const R P = ln.phase == PHASE_ISO ? R(0.5) : (s.core ? p_core(mu) : p_wing(mu));
      weight = P * R(1.0 / (2.0 * PI_D));
    } else {
      weight = p_hg(mu, cst<R>(pb.g_hg, pb.g_hg_f)) * R(1.0 / (2.0 * PI_D));
    }
    if constexpr (DEFER && sizeof(R) == 4) {
      // the float ray-cast pass bins the ray from its start (and counts
      // the deposits outside the cube)
      peel_push<R>(pb, q, 0.0, 0u, xo, weight, 0, oi, snk);
      continue;
    }
    const int pix = pixel_of<sizeof(R) == 4>(ob, p);
    const int bin = bin_of<sizeof(R) == 4>(ob, (double)xo);
    if (pix < 0 || bin < 0) {
      ++cnt.peel_drop;
      continue;
    }
    const size_t elem = (size_t)pix * ob.nbins + bin;
    if constexpr (DEFER) {
      if (qsteps) ++cnt.peel_cross;
      peel_push<R>(pb, q, qtau, qsteps, xo, weight, elem, oi, snk);
    } else {
      uint32_t nc = 0;
      const double tau = ray_tau<R, NL>(pb, p, ob.k, (double)xo, TauCut<R>::v, stk, stride, &nc, sc,
                                        sizeof(R) == 4 ? ob.kinv : nullptr);
      cnt.peel_cross += nc;
      if (tau < TauCut<R>::v) atomic_add_real((R *)ob.cube + elem, weight * M<R>::exp((R)(-tau)));
    }
  }
}

// ------------------------------------------------------------- transport
template <class R> struct Lane {
  int64_t pid;
  double p[3];
  R k[3];
  double kd[3];    // direction used for geometry (unit in double)
  R x;
  double tau, path;
  uint32_t event;
  uint32_t rej;    // regrouped loop: rejection rounds already run by the pending
                   // line scattering at p (0: none pending)
  int32_t nscat;
  Cell c;
  LeafRec<R> lf;
  LaneCount cnt;
};

// Geometry direction: the float direction of the bulk path is renormalised
// in double so that a packet's displacement equals its path length.
template <class R> __device__ __forceinline__ void set_geom_dir(Lane<R> &s) {
  if constexpr (sizeof(R) == 4) {
    const double a = s.k[0], b = s.k[1], c = s.k[2];
    // |k|^2 = 1 + e with |e| of order the float rounding: 1/sqrt(1+e) by its
    // series to e^3 (remainder below 2^-53 for |e| < 2^-16), else exactly
    const double e = fma(a, a, fma(b, b, fma(c, c, -1.0)));
    const double inv = fabs(e) < 0x1p-16 ? 1.0 + e * (-0.5 + e * (0.375 - 0.3125 * e)) : 1.0 / sqrt(1.0 + e);
    s.kd[0] = a * inv; s.kd[1] = b * inv; s.kd[2] = c * inv;
  } else {
    s.kd[0] = s.k[0]; s.kd[1] = s.k[1]; s.kd[2] = s.k[2];
  }
}

// Record a packet that ended (escaped, absorbed or stuck): its outputs, its
// counts in the problem's totals, and, in the launch's slice counters, the
// packet and its status (its dropped peel-off deposits are reported in the
// slice where it ends).
// Record a finished packet and count it.  The counts of the lanes that
// finish here together are summed over the wave first, one atomic per
// counter and wave: packets that end at once (short walks, a whole wave of
// them per loop pass) would otherwise queue on the same few addresses, one
// atomic per packet and counter.  Single-problem launches publish the
// packets' work (scatterings, crossings, peel-off rays) with the launch's
// slice totals at the end of the kernel; in batches, whose lanes change
// problem, each packet adds its own to its problem's totals here.
template <class R, bool BATCH>
__device__ void finish(const ProblemK &pb, Lane<R> &s, int status, unsigned long long *slice) {
  const int64_t i = s.pid - pb.first;
  pb.status[i] = status;
  pb.x_out[i] = (double)s.x;
  pb.k_out[3 * i] = (double)s.k[0];
  pb.k_out[3 * i + 1] = (double)s.k[1];
  pb.k_out[3 * i + 2] = (double)s.k[2];
  pb.pos_out[3 * i] = s.p[0];
  pb.pos_out[3 * i + 1] = s.p[1];
  pb.pos_out[3 * i + 2] = s.p[2];
  pb.nscat[i] = s.nscat;
  pb.path_out[i] = s.path;
  unsigned long long *st = pb.stats;
  const int sk = status == ST_ESCAPED ? S_ESCAPED : (status == ST_ABSORBED ? S_ABSORBED : S_STUCK);
  const unsigned long long m = __ballot(true);
  const unsigned long long me = __ballot(status == ST_ESCAPED), ma = __ballot(status == ST_ABSORBED);
  const unsigned long long ms = m & ~(me | ma);
  if (__lane_id() == __ffsll((long long)m) - 1) {
    atomicAdd(slice + S_EMITTED, (unsigned long long)__popcll(m));
    if (me) atomicAdd(slice + S_ESCAPED, (unsigned long long)__popcll(me));
    if (ma) atomicAdd(slice + S_ABSORBED, (unsigned long long)__popcll(ma));
    if (ms) atomicAdd(slice + S_STUCK, (unsigned long long)__popcll(ms));
    if (!BATCH) {
      atomicAdd(st + S_EMITTED, (unsigned long long)__popcll(m));
      if (me) atomicAdd(st + S_ESCAPED, (unsigned long long)__popcll(me));
      if (ma) atomicAdd(st + S_ABSORBED, (unsigned long long)__popcll(ma));
      if (ms) atomicAdd(st + S_STUCK, (unsigned long long)__popcll(ms));
    }
  }
  if (BATCH) {
    atomicAdd(st + S_EMITTED, 1ull);
    atomicAdd(st + sk, 1ull);
    atomicAdd(st + S_SCAT, (unsigned long long)s.nscat);
    if (s.cnt.dust_scat) atomicAdd(st + S_DUST_SCAT, (unsigned long long)s.cnt.dust_scat);
    atomicAdd(st + S_CROSS, (unsigned long long)s.cnt.cross);
    if (s.cnt.peel_rays) atomicAdd(st + S_PEEL_RAYS, (unsigned long long)s.cnt.peel_rays);
    if (s.cnt.peel_cross) atomicAdd(st + S_PEEL_CROSS, (unsigned long long)s.cnt.peel_cross);
  }
  if (s.cnt.peel_drop) {
    atomicAdd(st + S_PEEL_DROPPED, (unsigned long long)s.cnt.peel_drop);
    atomicAdd(slice + S_PEEL_DROPPED, (unsigned long long)s.cnt.peel_drop);
  }
}

// Emission (Sect. 2): position and frequency from the source list,
// isotropic direction unless given, tau_event = -ln r.
// Source spectrum (Sect. 2.1), added to the source's own x, in double in
// both precisions, by a pass before the transport (k_source_x) so that the
// transport kernels carry none of it.  Gaussian line: Box-Muller draw times
// sigma (Doppler widths of the reference line).  Power-law continuum,
// F_lambda ~ lambda^beta on [lambda_min, lambda_max]: inverse CDF of the
// photon-number distribution lambda F_lambda, then
// x = (lambda_ref - lambda) / (lambda b_ref)  (nu = c / lambda).
// r1, r2: the packet's emission draws J_SRC1, J_SRC2.
__device__ inline double source_spectrum_x(const ProblemK &pb, double r1, double r2) {
  if (pb.spec_kind == 1) return pb.spec_p[0] * sqrt(-2.0 * log(r1)) * cospi(2.0 * r2);
  if (pb.spec_kind == 3) {
    // tabulated continuum: bin i with probability (cum[i+1] - cum[i]) / cum[n-1]
    // (bisection), then the bin's power law by its inverse CDF in ratio form
    const double t = r1 * pb.tab_cum[pb.tab_n - 1];
    int lo = 0, hi = pb.tab_n - 2;  // the bin: first i with t < cum[i+1]
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (t < pb.tab_cum[mid + 1]) hi = mid; else lo = mid + 1;
    }
    const double l0 = pb.tab_lam[lo], l1 = pb.tab_lam[lo + 1], b = pb.tab_beta[lo];
    double lam;
    if (b == -2.0) {
      lam = l0 * exp(r2 * log(l1 / l0));
    } else {
      const double e = 2.0 + b;
      lam = l0 * pow(1.0 + r2 * (pow(l1 / l0, e) - 1.0), 1.0 / e);
    }
    return (pb.lambda_ref - lam) / (lam * pb.b_ref);
  }
  const double lmin = pb.spec_p[0], lmax = pb.spec_p[1], beta = pb.spec_p[2];
  const double r = r1;
  double lam;
  if (beta == -2.0) {
    lam = lmin * exp(r * log(lmax / lmin));
  } else {
    const double e = 2.0 + beta, a = pow(lmin, e);
    lam = pow(a + r * (pow(lmax, e) - a), 1.0 / e);
  }
  return (pb.lambda_ref - lam) / (lam * pb.b_ref);
}

// x_out[pid] = src_x[pid] + the packet's spectral draw, for pid in
// [first, first + n): the same counter-based emission draws (event 0,
// slots J_SRC1 and J_SRC2) the transport's precision would take.
template <class R>
__global__ void __launch_bounds__(256) k_source_x(const ProblemK pb, const double *__restrict__ src_x,
                                                  double *__restrict__ x_out, int64_t first, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t pid = first + i;
  EventRng<R> rng(pb.seed, (uint64_t)pid, 0u);
  const double r1 = (double)rng.u(J_SRC1), r2 = (double)rng.u(J_SRC2);
  x_out[pid] = src_x[pid] + source_spectrum_x(pb, r1, r2);
}

hipError_t launch_source_x(bool f32, const ProblemK &pb, const double *src_x, double *x_out, int64_t first,
                           int64_t n, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)((n + 255) / 256);
  if (f32)
    hipLaunchKernelGGL(k_source_x<float>, dim3(blocks), dim3(256), 0, stream, pb, src_x, x_out, first, n);
  else
    hipLaunchKernelGGL(k_source_x<double>, dim3(blocks), dim3(256), 0, stream, pb, src_x, x_out, first, n);
  return hipGetLastError();
}

template <class R, bool DEFER, int NL>
__device__ void emit(const ProblemK &pb, int64_t pid, Lane<R> &s, int *stk, int *pstk, int stride,
                     const PeelSink<R> &snk) {
  s.pid = pid;
  s.p[0] = pb.src_pos[3 * pid];
  s.p[1] = pb.src_pos[3 * pid + 1];
  s.p[2] = pb.src_pos[3 * pid + 2];
  EventRng<R> rng(pb.seed, (uint64_t)pid, 0u);
  if (pb.src_dir) {
    s.k[0] = (R)pb.src_dir[3 * pid];
    s.k[1] = (R)pb.src_dir[3 * pid + 1];
    s.k[2] = (R)pb.src_dir[3 * pid + 2];
  } else {
    const R mu = R(2) * rng.u(J_MU) - R(1);
    R sp, cp;
    M<R>::sincos2pi(rng.u(J_PHI), &sp, &cp);
    const R st = M<R>::sqrt(R(1) - mu * mu);
    s.k[0] = st * cp;
    s.k[1] = st * sp;
    s.k[2] = mu;
  }
  set_geom_dir(s);
  s.x = (R)pb.src_x[pid];
  s.tau = -(double)M<R>::log(rng.u(J_TAU));
  s.path = 0.0;
  s.event = 0;
  s.nscat = 0;
  s.rej = 0;
  s.cnt = LaneCount{0, 0, 0, 0, 0};
  if (pb.n_obs) {
    PeelSrc<R> ps;
    ps.kind = 0;
    ps.x = s.x;
    peel_all<R, DEFER, NL>(pb, s.p, ps, pstk, stride, s.cnt, snk);
  }
}

// Interaction at the current position (Sect. 3.2).  Returns the packet's
// status (ST_NONE while it lives).
// With REGROUP a line scattering runs one rejection round of its u_par
// draw per call: a rejected round leaves the event pending (s.rej rounds
// run) and the packet where it is, and the next pass of the transport loop
// calls again for the next round (the same draws as the looping sampler).
template <class R, bool DEFER, int NL, bool REGROUP = false>
__device__ int interact(const ProblemK &pb, Lane<R> &s, const Opac<R, NL> &o, int *pstk, const int *stk,
                        const PeelSink<R> &snk, int stride) {
  const StartCell<R> sc{&s.c, &s.lf, stk};
  if (!REGROUP || s.rej == 0) {
    ++s.event;
    if (pb.max_events > 0 && (int64_t)s.event >= pb.max_events) return ST_STUCK;
  }
  EventRng<R> rng(pb.seed, (uint64_t)s.pid, s.event);
  // kappa_d / kappa reaches ~1e-8 in optically thick line cores
  R r = rng.u_small(J_CHANNEL) * o.ktot;
  // the double generator keeps one Philox block: the draw of the channel's
  // block that the event uses last (the scattering angle) is taken now, so
  // that no block of the event is computed twice; the float path takes the
  // draws of block 0 it needs late now (tau_event and the scattering angle),
  // which leaves that block's words dead after the first rejection round
  const R r_late = rng.u(sizeof(R) == 4 ? J_TAU : J_MU);
  R r_mu = R(0);
  if constexpr (sizeof(R) == 4) r_mu = rng.u(J_MU);
  auto u_mu = [&]() { return sizeof(R) == 8 ? r_late : r_mu; };
  auto u_tau = [&]() { return sizeof(R) == 4 ? r_late : rng.u(J_TAU); };
  const R kin[3] = {s.k[0], s.k[1], s.k[2]};
  // the pair perpendicular to k_in is formed where it is used (after the
  // atom-velocity draw on the line branch, whose register peak it would
  // otherwise raise)
  R e1[3], e2[3];
  PeelSrc<R> ps;
  ps.kin[0] = kin[0]; ps.kin[1] = kin[1]; ps.kin[2] = kin[2];
  ps.ux = s.lf.ux; ps.uy = s.lf.uy; ps.uz = s.lf.uz;
  ps.w = o.w;
  if (r < o.kd) {
    // dust (Sect. 3.2.2): absorbed with probability 1 - albedo, else HG
    if (rng.u(J_ALBEDO) >= cst<R>(pb.albedo, pb.albedo_f)) return ST_ABSORBED;
    ++s.cnt.dust_scat;
    if (pb.n_obs) {
      ps.kind = 2;
      ps.x = s.x;
      peel_all<R, DEFER, NL>(pb, s.p, ps, pstk, stride, s.cnt, snk, &sc);
    }
    if (!pb.forward_only) {
      perp_basis(kin, e1, e2);
      const R mu = mu_hg(u_mu(), cst<R>(pb.g_hg, pb.g_hg_f));
      R sp, cp;
      M<R>::sincos2pi(rng.u(J_PHI), &sp, &cp);
      const R st = M<R>::sqrt(fmax(R(0), R(1) - mu * mu));
#pragma unroll
      for (int d = 0; d < 3; ++d) s.k[d] = mu * kin[d] + st * (cp * e1[d] + sp * e2[d]);
      set_geom_dir(s);
      // coherent in the cell frame
      const R wn = s.k[0] * s.lf.ux + s.k[1] * s.lf.uy + s.k[2] * s.lf.uz;
      const R b = cst<R>(pb.b_ref, pb.b_ref_f);
      s.x = M<R>::div(s.x + wn + b * s.x * wn - o.w, R(1) + b * o.w);
    }
  } else {
    // resonant scattering in line i (Sect. 3.2.1)
    r -= o.kd;
    // first line whose cumulative opacity exceeds r (the last line takes
    // any rounding remainder)
    int i = 0;
    R x = o.x[0];
    bool found = false;
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      if (!found && q < pb.n_lines) {
        if (r < o.kl[q] || q == pb.n_lines - 1) {
          i = q;
          x = o.x[q];
          found = true;
        } else {
          r -= o.kl[q];
        }
      }
    }
    const LineK &ln = pb.lines[i];
    const R a = cst<R>(ln.alpha, ln.f.alpha) * s.lf.irho;
    // log10 a for the envelope: the double path adds the line's log10 alpha
    // and the leaf's log10(1/rho) (its record holds it)
    const R la = sizeof(R) == 8 ? R(ln.lalpha) + s.lf.lg : M<R>::log10(a);
    // float: block 1 (the second rejection round, the perpendicular
    // velocities and the azimuth) for every lane of the branch at once, its
    // outgoing draws taken now so that its words are dead after the
    // sampler's second round
    R r_p1 = R(0), r_p2 = R(0), r_phi = R(0);
    if constexpr (sizeof(R) == 4) {
      rng.need1();
      r_p1 = rng.u(J_PERP1);
      r_p2 = rng.u(J_PERP2);
      r_phi = rng.u(J_PHI);
    }
    auto u_p1 = [&]() { return sizeof(R) == 4 ? r_p1 : rng.u(J_PERP1); };
    auto u_p2 = [&]() { return sizeof(R) == 4 ? r_p2 : rng.u(J_PERP2); };
    auto u_phi = [&]() { return sizeof(R) == 4 ? r_phi : rng.u(J_PHI); };
    R upar;
    if constexpr (REGROUP) {
      if (!upar_round<R>(x, a, la, rng, s.rej, &upar)) {
        if (++s.rej >= MAX_REJECT) return ST_STUCK;
        return ST_NONE;
      }
      s.rej = 0;
    } else {
      if (!sample_upar<R>(x, a, la, rng, &upar)) return ST_STUCK;
    }
    // Gaussian u_perp (Box-Muller), restricted to |u_perp| >= x_crit while
    // core-skipping applies
    const R xc2 = pb.skip_tau > 0.0 ? core_skip_x2<R>(pb, ln, s.lf, s.c.level, a, x) : R(0);
    perp_basis(kin, e1, e2);
    R sp, cp;
    M<R>::sincos2pi(u_p2(), &sp, &cp);
    const R rr = M<R>::sqrt(xc2 - M<R>::log(u_p1()));
    const R up1 = rr * cp, up2 = rr * sp;
    R U[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) U[d] = upar * kin[d] + up1 * e1[d] + up2 * e2[d];
    const R rho = M<R>::div(R(1), s.lf.irho);
    const R bc = cst<R>(pb.b_ref, pb.b_ref_f) * cst<R>(ln.mu, ln.f.mu) * rho;
    // frequency seen by the atom, nu_in (1 - k_in.v/c), within 0.2 dnu_D
    const R g1 = R(1) + bc * x;
    const int core = fabs(x - g1 * upar) < R(0.2);
    // decay channel (Sect. 3.2.1): fluorescent channel j when the draw lies
    // at or above A_ul / sum A (then (A_ul + A_0) / sum A for j = 1); lines
    // with channels run in the multi-line kernels only
    int fch = -1;
    if constexpr (NL > 1) {
      if (ln.n_fluor > 0 && !pb.forward_only) {
        const R ud = rng.u(J_DECAY);
        if (ud >= cst<R>(ln.a_res, ln.f.a_res)) fch = (ln.n_fluor > 1 && ud >= cst<R>(ln.a_cum0, ln.f.a_cum0)) ? 1 : 0;
      }
    }
    ++s.nscat;
    if (NL > 1 && fch >= 0) {
      if (pb.n_obs) {
        ps.kind = 3;
        ps.U[0] = U[0]; ps.U[1] = U[1]; ps.U[2] = U[2];
        ps.bc = bc;
        ps.line = i;
        ps.core = fch;
        peel_all<R, DEFER, NL>(pb, s.p, ps, pstk, stride, s.cnt, snk, &sc);
      }
      const R mu = R(2) * u_mu() - R(1);
      M<R>::sincos2pi(u_phi(), &sp, &cp);
      const R st = M<R>::sqrt(fmax(R(0), R(1) - mu * mu));
#pragma unroll
      for (int d = 0; d < 3; ++d) s.k[d] = mu * kin[d] + st * (cp * e1[d] + sp * e2[d]);
      set_geom_dir(s);
      const R ba = bc * (s.k[0] * U[0] + s.k[1] * U[1] + s.k[2] * U[2]);
      const R bw = cst<R>(pb.b_ref, pb.b_ref_f) * (s.k[0] * s.lf.ux + s.k[1] * s.lf.uy + s.k[2] * s.lf.uz);
      s.x = cst<R>(ln.xf0[fch], ln.f.xf0[fch]) + M<R>::div(cst<R>(ln.sf[fch], ln.f.sf[fch]) * (ba + bw + ba * bw), cst<R>(pb.b_ref, pb.b_ref_f));
      s.tau = -(double)M<R>::log(u_tau());
      return ST_NONE;
    }
    if (pb.n_obs) {
      ps.kind = 1;
      ps.x = x;
      ps.U[0] = U[0]; ps.U[1] = U[1]; ps.U[2] = U[2];
      ps.bc = bc;
      ps.rho = rho;
      ps.irho = s.lf.irho;
      ps.line = i;
      ps.core = core;
      peel_all<R, DEFER, NL>(pb, s.p, ps, pstk, stride, s.cnt, snk, &sc);
    }
    if (!pb.forward_only) {
      const R ru = u_mu();
      const R mu = ln.phase == PHASE_ISO ? R(2) * ru - R(1) : mu_dipole(ru, core != 0);
      M<R>::sincos2pi(u_phi(), &sp, &cp);
      const R st = M<R>::sqrt(fmax(R(0), R(1) - mu * mu));
#pragma unroll
      for (int d = 0; d < 3; ++d) s.k[d] = mu * kin[d] + st * (cp * e1[d] + sp * e2[d]);
      set_geom_dir(s);
      // outgoing frequency, coherent in the atom frame, recoil in the
      // denominator (Eq. for nu_out), then back to the external frame
      const R dkU = (s.k[0] - kin[0]) * U[0] + (s.k[1] - kin[1]) * U[1] + (s.k[2] - kin[2]) * U[2];
      const R Rr = ln.recoil ? (R(1) - mu) * cst<R>(ln.rec, ln.f.rec) * g1 : R(0);
      R xc;
      if constexpr (sizeof(R) == 4) {
        // as in the peel-off: 1/(1 + Rr) = 1 - Rr and Rr/bc = Rr irho/(b_ref mu)
        xc = (x + g1 * dkU - Rr * cst<R>(ln.ibmu, ln.f.ibmu) * s.lf.irho) * (R(1) - Rr);
      } else {
        xc = M<R>::div(x + g1 * dkU - M<R>::div(Rr, bc), R(1) + Rr);
      }
      const R wn = s.k[0] * s.lf.ux + s.k[1] * s.lf.uy + s.k[2] * s.lf.uz;
      s.x = (-cst<R>(ln.delta, ln.f.delta) + cst<R>(ln.mu, ln.f.mu) * rho * xc * (R(1) + cst<R>(pb.b_ref, pb.b_ref_f) * wn) + wn) * cst<R>(ln.inv_s, ln.f.inv_s);
    }
  }
  s.tau = -(double)M<R>::log(u_tau());
  return ST_NONE;
}

// Packet state kept in HBM between launches (one slot per lane of the
// grid): a run is a sequence of bounded launches, each lane resuming the
// packet it held, so no launch waits for the longest random walk and each
// launch can be replayed from a captured graph.
struct SlotState {
  double p[3], k[3];
  double x, tau, path;
  int64_t pid;
  int32_t prob, active, event, nscat;
  int32_t leaf, level, ox, oy, oz;
  uint32_t dust, cross, peel_rays, peel_cross, peel_drop;
  uint32_t rej;
};

template <class R>
__device__ __forceinline__ void save_slot(SlotState &q, const Lane<R> &s, int prob) {
  for (int d = 0; d < 3; ++d) { q.p[d] = s.p[d]; q.k[d] = (double)s.k[d]; }
  q.x = (double)s.x; q.tau = s.tau; q.path = s.path; q.pid = s.pid;
  q.prob = prob; q.active = 1; q.event = (int32_t)s.event; q.nscat = s.nscat;
  q.leaf = s.c.leaf; q.level = s.c.level; q.ox = s.c.ox; q.oy = s.c.oy; q.oz = s.c.oz;
  q.dust = s.cnt.dust_scat; q.cross = s.cnt.cross; q.peel_rays = s.cnt.peel_rays;
  q.peel_cross = s.cnt.peel_cross; q.peel_drop = s.cnt.peel_drop;
  q.rej = s.rej;
}

template <class R>
__device__ __forceinline__ void load_slot(const SlotState &q, Lane<R> &s, int *prob) {
  for (int d = 0; d < 3; ++d) { s.p[d] = q.p[d]; s.k[d] = (R)q.k[d]; }
  s.x = (R)q.x; s.tau = q.tau; s.path = q.path; s.pid = q.pid;
  *prob = q.prob; s.event = (uint32_t)q.event; s.nscat = q.nscat;
  s.c.leaf = q.leaf; s.c.level = q.level; s.c.ox = q.ox; s.c.oy = q.oy; s.c.oz = q.oz;
  s.cnt.dust_scat = q.dust; s.cnt.cross = q.cross; s.cnt.peel_rays = q.peel_rays;
  s.cnt.peel_cross = q.peel_cross; s.cnt.peel_drop = q.peel_drop;
  s.rej = q.rej;
  set_geom_dir(s);
}

// Counters of work done inside one launch, summed over the wave and
// published at the kernel's end (the packets that end in it are counted by
// finish).
struct SliceCount {
  uint32_t scat, dust, cross, peel_rays, peel_cross;
};

template <class R>
__device__ __forceinline__ void add_delta(SliceCount &a, const Lane<R> &s, const Lane<R> &z) {
  a.scat += (uint32_t)(s.nscat - z.nscat);
  a.dust += s.cnt.dust_scat - z.cnt.dust_scat;
  a.cross += s.cnt.cross - z.cnt.cross;
  a.peel_rays += s.cnt.peel_rays - z.cnt.peel_rays;
  a.peel_cross += s.cnt.peel_cross - z.cnt.peel_cross;
}

// Waves per SIMD the transport kernel is compiled for (register budget,
// chosen by measurement): the float single-problem kernels with deferred
// peel-off run four (about 30 registers spill with one line, 40 with four,
// and they are 8-9% faster than at three), the other float kernels three
// (no spills; at four the batch kernels spill 50-90 registers and the batch
// runs slower), the single-problem double kernels with deferred peel-off
// two (40-55 registers spill, and the dusty sphere runs 38% faster than at
// one, where nothing spills), the other double kernels (batch, inline
// walker; 90-200 registers would spill at two) one.
#ifndef RMC_WAVES_F32_LEAN
#define RMC_WAVES_F32_LEAN 4
#endif
#ifndef RMC_WAVES_F32
#define RMC_WAVES_F32 3
#endif
#ifndef RMC_WAVES_F32_MULTI
#define RMC_WAVES_F32_MULTI 4
#endif
#ifndef RMC_WAVES_F64
#define RMC_WAVES_F64 2
#endif
#ifndef RMC_WAVES_F64_WIDE
#define RMC_WAVES_F64_WIDE 1
#endif
template <class R, bool BATCH, bool DEFER, int NL> struct WavesPerEU;
template <bool BATCH, bool DEFER, int NL> struct WavesPerEU<float, BATCH, DEFER, NL> {
  static constexpr int v = (!BATCH && DEFER) ? (NL == 1 ? RMC_WAVES_F32_LEAN : RMC_WAVES_F32_MULTI) : RMC_WAVES_F32;
};
template <bool BATCH, bool DEFER, int NL> struct WavesPerEU<double, BATCH, DEFER, NL> {
  static constexpr int v = (!BATCH && DEFER) ? RMC_WAVES_F64 : RMC_WAVES_F64_WIDE;
};

// REGROUP: a line scattering whose rejection round fails stays pending and
// takes its next round at the next pass of the loop, where it runs in step
// with the other lanes' events (upar_round), instead of the wave looping
// until its last lane accepts.
// TAIL: the same kernel compiled for one wave per SIMD (registers to spare,
// no spills), for the launches over gathered slots at the end of a run,
// whose waves are no more than the SIMDs: each issues on its own, so its
// latency, not the chip's throughput, sets the pace.
template <class R, bool BATCH, bool DEFER, int NL, bool REGROUP = false, bool TAIL = false>
__global__ void __launch_bounds__(256)
    __attribute__((amdgpu_waves_per_eu(TAIL ? 1 : WavesPerEU<R, BATCH, DEFER, NL>::v,
                                       TAIL ? 1 : WavesPerEU<R, BATCH, DEFER, NL>::v)))
    k_transport(const ProblemK *__restrict__ probs,
                                                   const int64_t *__restrict__ starts, int n_probs,
                                                   unsigned long long *__restrict__ next,
                                                   int refill_min, int stack_levels,
                                                   SlotState *__restrict__ slots, int budget,
                                                   unsigned long long *__restrict__ slice) {
  extern __shared__ int lds[];
  const int stride = blockDim.x;
  int *stk = lds + threadIdx.x;
  int *pstk = lds + stack_levels * stride + threadIdx.x;
  const int64_t total = starts[n_probs];
  const int lane = __lane_id();
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  // this wave's region of the deferred peel-off queue; the wave ends its
  // slice early once one more iteration (an emission and an event, each
  // peeled toward every observer) could overflow it
  // (no queue when no problem of the launch has an observer)
  PeelQueue *const pq = DEFER ? probs[0].pq : nullptr;
  const bool queue = DEFER && pq != nullptr;
  const int64_t wave = gid >> 6;
  PeelSink<R> snk;
  snk.count = lds + 2 * stack_levels * stride + (threadIdx.x >> 6);
  snk.region = queue ? (PeelJob<R> *)pq->jobs + (size_t)wave * pq->cap : nullptr;
  snk.cap = queue ? (uint32_t)pq->cap : 0u;
  snk.lost = queue ? &pq->lost : nullptr;
  const int room = queue ? (int)pq->cap - 2 * 64 * MAX_OBS : 0x7fffffff;
  if (lane == 0) *snk.count = 0;

  Lane<R> s;
  Lane<R> z;            // counters when this slice took the packet over
  SliceCount acc{0, 0, 0, 0, 0};
  int prob = 0;
  bool active = false;
  bool drained = false;
  {
    const SlotState &q = slots[gid];
    if (q.active) {
      load_slot<R>(q, s, &prob);
      const ProblemK &pb = probs[BATCH ? prob : 0];
      const int X[3] = {s.c.ox, s.c.oy, s.c.oz};
      locate(pb, X, stk, stride, s.c);
      s.lf = load_leaf<R>(pb.leaves, s.c.leaf);
      active = true;
      z = s;
    }
  }
  for (int it = 0; it < budget; ++it) {
    if (DEFER && *snk.count > room) break;
    // ---- refill idle lanes: one atomic per wave, ranks from mbcnt
    if (!drained) {
      const unsigned long long idle = __ballot(!active);
      const int n_idle = __popcll(idle);
      const bool any_active = idle != ~0ull >> (64 - warpSize);
      if (n_idle > 0 && (n_idle >= refill_min || !any_active)) {
        unsigned long long base = 0;
        if (lane == __ffsll((long long)idle) - 1) base = atomicAdd(next, (unsigned long long)n_idle);
        base = __shfl(base, __ffsll((long long)idle) - 1);
        if (base >= (unsigned long long)total) drained = true;
        if (!active) {
          const unsigned long long below = idle & ((1ull << lane) - 1ull);
          const int64_t g = (int64_t)(base + __popcll(below));
          if (g < total) {
            if (BATCH) {
              int lo = 0, hi = n_probs - 1;
              while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (starts[mid] <= g) lo = mid; else hi = mid - 1;
              }
              prob = lo;
            }
            const ProblemK &pb = probs[BATCH ? prob : 0];
            const int64_t pid = pb.first + (g - starts[BATCH ? prob : 0]);
            emit<R, DEFER, NL>(pb, pid, s, stk, pstk, stride, snk);
            z = s;
            z.nscat = 0;
            z.cnt = LaneCount{0, 0, 0, 0, 0};
            int X[3];
            if (int_coords(pb.L, s.p, s.kd, X)) {
              locate(pb, X, stk, stride, s.c);
              s.lf = load_leaf<R>(pb.leaves, s.c.leaf);
              active = true;
            } else {
              add_delta(acc, s, z);
              finish<R, BATCH>(pb, s, ST_ESCAPED, slice);
            }
          }
        }
      }
    }
    if (__ballot(active) == 0ull) {
      if (drained) break;
      continue;
    }
    if (!active) continue;

    const ProblemK &pb = probs[BATCH ? prob : 0];
    const double kd[3] = {s.kd[0], s.kd[1], s.kd[2]};
    Opac<R, NL> o;
    opacity(pb, s.lf, (double)s.x, s.k, o);
    double face[3], lo[3], hi[3];
    int em = 0;
    double te = 0.0, td = 0.0, lmax = 0.0, tseg = 0.0;
    // a pending line scattering (REGROUP) is already at its event point
    const bool pend = REGROUP && s.rej != 0;
    // An event closer than the nearest face of a leaf inside the domain
    // happens in this leaf whatever the exit distance; only a packet that
    // may leave needs it (the decision is the one tau < tseg would take).
    bool here = pend || (s.lf.bnd == R(0) && s.tau < (double)o.ktot * inner_dist(s.c, pb.L, s.p));
    if (here) {
      cell_bounds(s.c, pb.L, lo, hi);
    } else {
      te = exit_dist(s.c, pb.L, s.p, kd, face, lo, hi, &em);
      td = domain_dist_leaf(s.lf, pb.domain, pb.dom, s.p, kd);
      lmax = te < td ? te : td;
      tseg = (double)o.ktot * lmax;
      here = s.tau < tseg;
    }
    int st = ST_NONE;
    if (here) {
      // the event happens inside this leaf (float path: kappa is a float
      // and tau_event came from a float logarithm, so a float reciprocal
      // of kappa loses nothing the path keeps)
      // (a pending event moves by 0: p stays, clamped into its own leaf)
      const double dist = pend ? 0.0
                               : (sizeof(R) == 4 ? s.tau * (double)__builtin_amdgcn_rcpf((float)o.ktot)
                                                 : s.tau / (double)o.ktot);
#pragma unroll
      for (int d = 0; d < 3; ++d) s.p[d] = fmin(fmax(fma(dist, kd[d], s.p[d]), lo[d]), hi[d]);
      s.path += dist;
      st = interact<R, DEFER, NL, REGROUP>(pb, s, o, pstk, stk, snk, stride);
    } else {
      s.tau -= tseg;
      s.path += lmax;
      ++s.cnt.cross;
      if (s.cnt.cross >= MAX_CROSS) {
        st = ST_STUCK;
      } else if (td <= te) {
#pragma unroll
        for (int d = 0; d < 3; ++d) s.p[d] = fma(td, kd[d], s.p[d]);
        st = ST_ESCAPED;
      } else {
        double pn[3];
        exit_point(te, em, s.p, kd, face, lo, hi, pn);
        s.p[0] = pn[0]; s.p[1] = pn[1]; s.p[2] = pn[2];
        wrap_slab(pb.domain, s.p, kd);
        int X[3];
        if (!int_coords(pb.L, s.p, kd, X)) {
          st = ST_ESCAPED;
        } else {
          relocate(pb, X, stk, stride, s.c);
          s.lf = load_leaf<R>(pb.leaves, s.c.leaf);
        }
      }
    }
    if (st != ST_NONE) {
      add_delta(acc, s, z);
      finish<R, BATCH>(pb, s, st, slice);
      active = false;
    }
  }
  // ---- park the packet (if any) for the next launch, publish the counts
  SlotState &q = slots[gid];
  if (active) {
    save_slot<R>(q, s, prob);
    add_delta(acc, s, z);
  } else {
    q.active = 0;
  }
  if (queue && lane == 0) {
    const int nq = *snk.count;
    pq->counts[wave] = (uint32_t)nq;
    if (nq) {
      atomicAdd(&pq->pushes, (unsigned long long)nq);
      atomicMax(&pq->max_region, (unsigned long long)nq);
    }
  }
  unsigned long long v[5] = {acc.scat, acc.dust, acc.cross, acc.peel_rays, acc.peel_cross};
  const int idx[5] = {S_SCAT, S_DUST_SCAT, S_CROSS, S_PEEL_RAYS, S_PEEL_CROSS};
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    unsigned long long x = v[j];
    for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off);
    if (lane == 0 && x) {
      atomicAdd(slice + idx[j], x);
      if (!BATCH) atomicAdd(probs[0].stats + idx[j], x);
    }
  }
}

// Number of slots (lanes) holding a packet after a launch.
__global__ void k_count_live(const SlotState *__restrict__ slots, int64_t n, unsigned long long *out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long v = (i < n && slots[i].active) ? 1ull : 0ull;
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
  if (__lane_id() == 0 && v) atomicAdd(out, v);
}

__global__ void k_clear_slots(SlotState *__restrict__ slots, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) slots[i].active = 0;
}

// Parked packets gathered to the front: every active slot of src[0, n) is
// copied to its own slot of dst (order not kept; a packet's walk does not
// depend on the lane that runs it), one atomic per wave; *n_live counts
// them.  Once every packet of a stream has started, the launches that
// follow run on the gathered slots with as many waves as the packets fill,
// so the last long walks share fewer SIMDs and each wave issues faster.
__global__ void k_compact_slots(const SlotState *__restrict__ src, int64_t n, SlotState *__restrict__ dst,
                                unsigned long long *n_live) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool act = i < n && src[i].active;
  const unsigned long long m = __ballot(act);
  if (m == 0ull) return;
  const int lane = __lane_id();
  const int leader = __ffsll((long long)m) - 1;
  unsigned long long base = 0;
  if (lane == leader) base = atomicAdd(n_live, (unsigned long long)__popcll(m));
  base = __shfl(base, leader);
  if (act) dst[base + (unsigned long long)__popcll(m & ((1ull << lane) - 1ull))] = src[i];
}

__global__ void k_fill_u32(uint32_t *p, int64_t n, uint32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Ray-cast pass over the peel-off rays queued by a transport launch.  A
// wave takes the queue regions one at a time; each lane walks one ray a
// leaf per iteration and takes the region's next ray as soon as its own is
// done, so the waves stay full while ray lengths vary.  The walk is the one
// of ray_walk from the queued state (a ray's start, or where it left its
// first leaf), and every deferred deposit is made here.
#ifndef RMC_DRAIN_WAVES_F32
#define RMC_DRAIN_WAVES_F32 4
#endif
#ifndef RMC_DRAIN_WAVES_F64
#define RMC_DRAIN_WAVES_F64 3
#endif
template <class R> struct DrainWaves;
template <> struct DrainWaves<float> { static constexpr int v = RMC_DRAIN_WAVES_F32; };
template <> struct DrainWaves<double> { static constexpr int v = RMC_DRAIN_WAVES_F64; };

template <class R, bool BATCH, int NL>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(DrainWaves<R>::v)))
    k_peel_drain(const ProblemK *__restrict__ probs, PeelQueue *pq,
                                                    unsigned long long *__restrict__ slice) {
  extern __shared__ int lds[];
  const int stride = blockDim.x;
  int *stk = lds + threadIdx.x;
  const int lane = __lane_id();
  const unsigned long long n_regions = pq->n_regions, cap = pq->cap;
  const PeelJob<R> *__restrict__ jobs = (const PeelJob<R> *)pq->jobs;
  const uint32_t *__restrict__ counts = pq->counts;
  const double cut = TauCut<R>::v;
  // wave-uniform: current region, next job in it, jobs in it
  unsigned long long reg = 0;
  uint32_t r_next = 0, r_n = 0;
  bool drained = false;
  bool active = false;
  int prob = 0, acc_prob = 0;
  double p[3], k[3], tau = 0.0, x = 0.0;
  R weight = R(0), kr[3];
  unsigned long long elem = 0;
  int oi = 0;
  uint32_t steps = 0;
  Cell c;
  unsigned long long nc_prob = 0, nc_all = 0;
  unsigned long long nd_prob = 0, nd_all = 0;   // float jobs outside the cube
  while (true) {
    unsigned long long idle = __ballot(!active);
    while (idle && !drained) {
      if (r_next >= r_n) {
        unsigned long long t = 0;
        if (lane == 0) t = atomicAdd(&pq->take, 1ull);
        reg = __shfl(t, 0);
        if (reg >= n_regions) {
          drained = true;
          break;
        }
        const uint32_t cnt = counts[reg];
        r_n = cnt < cap ? cnt : (uint32_t)cap;
        r_next = 0;
        continue;
      }
      const uint32_t avail = r_n - r_next;
      const uint32_t rank = (uint32_t)__popcll(idle & ((1ull << lane) - 1ull));
      const bool mine = ((idle >> lane) & 1ull) && rank < avail;
      if (mine) {
        const PeelJob<R> j = jobs[reg * cap + r_next + rank];
        const int jp = BATCH ? (int)(j.dst >> PQ_PROB_SHIFT) : 0;
        if (BATCH && jp != acc_prob) {
          if (nc_prob) atomicAdd(probs[acc_prob].stats + S_PEEL_CROSS, nc_prob);
          if (nd_prob) atomicAdd(probs[acc_prob].stats + S_PEEL_DROPPED, nd_prob);
          nc_prob = 0;
          nd_prob = 0;
          acc_prob = jp;
        }
        prob = jp;
        const ProblemK &pb = probs[prob];
        oi = (int)((j.dst >> PQ_OBS_SHIFT) & 15ull);
        const ObsK &ob = pb.obs[oi];
        k[0] = ob.k[0]; k[1] = ob.k[1]; k[2] = ob.k[2];
        kr[0] = (R)k[0]; kr[1] = (R)k[1]; kr[2] = (R)k[2];
        p[0] = j.p[0]; p[1] = j.p[1]; p[2] = j.p[2];
        x = (double)j.x;
        weight = (R)j.weight;
        bool binned = true;
        if constexpr (sizeof(R) == 8) {
          tau = j.tau;
          steps = j.steps;
          elem = j.dst & PQ_ELEM_MASK;
        } else {
          // float jobs come unbinned, from the ray's start
          tau = 0.0;
          steps = 0;
          const int pix = pixel_of<true>(ob, p);
          const int bin = bin_of<true>(ob, x);
          binned = pix >= 0 && bin >= 0;
          elem = binned ? (unsigned long long)pix * ob.nbins + bin : 0ull;
          if (!binned) {
            ++nd_prob;
            ++nd_all;
          }
        }
        int X[3];
        if (binned) {
          if (steps < MAX_CROSS && int_coords(pb.L, p, k, X)) {
            locate(pb, X, stk, stride, c);
            active = true;
          } else if (tau < cut) {
            atomic_add_real((R *)ob.cube + elem, weight * M<R>::exp((R)(-tau)));
          }
        }
      }
      const uint32_t n_idle = (uint32_t)__popcll(idle);
      r_next += avail < n_idle ? avail : n_idle;
      // lanes given a job that ended at once stay idle until the next pass
      idle &= ~__ballot(mine);
    }
    if (__ballot(active) == 0ull) {
      if (drained) break;
      continue;
    }
    if (!active) continue;
    const ProblemK &pb = probs[BATCH ? prob : 0];
    const LeafRec<R> lf = load_leaf<R>(pb.leaves, c.leaf);
    Opac<R, NL> o;
    opacity(pb, lf, x, kr, o);
    double face[3], lo[3], hi[3];
    int em;
    const double te = exit_dist(c, pb.L, p, k, face, lo, hi, &em, sizeof(R) == 4 ? pb.obs[oi].kinv : nullptr);
    const double td = domain_dist_leaf(lf, pb.domain, pb.dom, p, k);
    ++nc_prob;
    ++nc_all;
    bool done = false;
    if (td <= te) {
      tau += (double)o.ktot * td;
      done = true;
    } else {
      tau += (double)o.ktot * te;
      if (tau >= cut) {
        done = true;
      } else {
        double pn[3];
        exit_point(te, em, p, k, face, lo, hi, pn);
        p[0] = pn[0]; p[1] = pn[1]; p[2] = pn[2];
        wrap_slab(pb.domain, p, k);
        int X[3];
        if (!int_coords(pb.L, p, k, X)) {
          done = true;
        } else {
          relocate(pb, X, stk, stride, c);
          if (++steps >= MAX_CROSS) done = true;
        }
      }
    }
    if (done) {
      if (tau < cut) atomic_add_real((R *)pb.obs[oi].cube + elem, weight * M<R>::exp((R)(-tau)));
      active = false;
    }
  }
  // crossings and dropped deposits: per problem, and for the launch's
  // slice counters
  if (BATCH) {
    if (nc_prob) atomicAdd(probs[acc_prob].stats + S_PEEL_CROSS, nc_prob);
    if (nd_prob) atomicAdd(probs[acc_prob].stats + S_PEEL_DROPPED, nd_prob);
  } else {
    unsigned long long v = nc_prob, d = nd_prob;
    for (int off = 32; off > 0; off >>= 1) {
      v += __shfl_down(v, off);
      d += __shfl_down(d, off);
    }
    if (lane == 0 && v) atomicAdd(probs[0].stats + S_PEEL_CROSS, v);
    if (lane == 0 && d) atomicAdd(probs[0].stats + S_PEEL_DROPPED, d);
  }
  unsigned long long v = nc_all, d = nd_all;
  for (int off = 32; off > 0; off >>= 1) {
    v += __shfl_down(v, off);
    d += __shfl_down(d, off);
  }
  if (lane == 0 && v) atomicAdd(slice + S_PEEL_CROSS, v);
  if (lane == 0 && d) atomicAdd(slice + S_PEEL_DROPPED, d);
}

// After the ray-cast pass: report the launch's pushes, largest region and
// lost pushes (slice counters N_STATS .. N_STATS+2) and reset the totals.
__global__ void k_peel_reset(PeelQueue *pq, unsigned long long *slice) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    slice[N_STATS] = pq->pushes;
    slice[N_STATS + 1] = pq->max_region;
    slice[N_STATS + 2] = pq->lost;
    pq->lost = 0ull;
    pq->pushes = 0ull;
    pq->max_region = 0ull;
    pq->take = 0ull;
  }
}

// ------------------------------------------------------------------ probes
__global__ void k_trace(ProblemK pb, int64_t n, const double *__restrict__ orig,
                        const double *__restrict__ dir, int max_cells, int32_t *__restrict__ leaf_out,
                        double *__restrict__ seg_out, int32_t *__restrict__ n_out) {
  extern __shared__ int lds[];
  int *stk = lds + threadIdx.x;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  double p[3] = {orig[3 * r], orig[3 * r + 1], orig[3 * r + 2]};
  const double k[3] = {dir[3 * r], dir[3 * r + 1], dir[3 * r + 2]};
  int X[3];
  int cnt = 0;
  if (int_coords(pb.L, p, k, X)) {
    Cell c;
    locate(pb, X, stk, blockDim.x, c);
    while (cnt < max_cells) {
      double face[3], lo[3], hi[3];
      int em;
      const double te = exit_dist(c, pb.L, p, k, face, lo, hi, &em);
      const double td = domain_dist(pb.domain, pb.dom, p, k);
      leaf_out[r * max_cells + cnt] = c.leaf;
      if (td <= te) {
        seg_out[r * max_cells + cnt] = td;
        ++cnt;
        break;
      }
      seg_out[r * max_cells + cnt] = te;
      ++cnt;
      double pn[3];
      exit_point(te, em, p, k, face, lo, hi, pn);
      p[0] = pn[0]; p[1] = pn[1]; p[2] = pn[2];
      wrap_slab(pb.domain, p, k);
      if (!int_coords(pb.L, p, k, X)) break;
      relocate(pb, X, stk, blockDim.x, c);
    }
  }
  n_out[r] = cnt;
}

template <class R>
__global__ void k_tau(ProblemK pb, int64_t n, const double *__restrict__ orig,
                      const double *__restrict__ dir, const double *__restrict__ x_ext,
                      double *__restrict__ tau_out) {
  extern __shared__ int lds[];
  int *stk = lds + threadIdx.x;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const double p[3] = {orig[3 * r], orig[3 * r + 1], orig[3 * r + 2]};
  const double k[3] = {dir[3 * r], dir[3 * r + 1], dir[3 * r + 2]};
  uint32_t nc = 0;
  tau_out[r] = ray_tau<R>(pb, p, k, x_ext[r], __builtin_inf(), stk, blockDim.x, &nc, nullptr);
}

// ------------------------------------------------- peel-off image, adjoint
template <class R>
__global__ void k_image_fwd(ProblemK pb, int obs, int64_t n, const double *__restrict__ orig,
                            const double *__restrict__ x_ext, const double *__restrict__ w,
                            double *__restrict__ image, unsigned long long *__restrict__ ncross) {
  extern __shared__ int lds[];
  int *stk = lds + threadIdx.x;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t nc = 0;
  if (r < n) {
    const ObsK &ob = pb.obs[obs];
    const double p[3] = {orig[3 * r], orig[3 * r + 1], orig[3 * r + 2]};
    const int pix = pixel_of(ob, p);
    if (pix >= 0) {
      const double tau = ray_tau<R>(pb, p, ob.k, x_ext[r], TauCut<double>::v, stk, blockDim.x, &nc, nullptr,
                                    sizeof(R) == 4 ? ob.kinv : nullptr);
      if (tau < TauCut<double>::v) unsafeAtomicAdd(image + pix, w[r] * exp(-tau));
    }
  }
  // one atomic per wave for the crossing count
  unsigned long long v = nc;
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
  if (__lane_id() == 0 && v) atomicAdd(ncross, v);
}

// Adds each lane's (an, ak, av) to leaf `leaf` (< 0: nothing) of the
// gradients: one sum and one atomic per distinct leaf of the wave (a few
// when a wave holds rays of two sources); lanes with many distinct leaves
// fall back to their own atomics after four rounds.  Every lane of the
// wave must call it (shuffles).
__device__ __forceinline__ void wave_leaf_add(int leaf, double an, double ak, double av, double *g_n,
                                              double *g_k, double *g_v, int lane) {
  unsigned long long m = __ballot(leaf >= 0);
  for (int round = 0; m && round < 4; ++round) {
    const int lead = __ffsll((long long)m) - 1;
    const int l0 = __shfl(leaf, lead);
    const bool mine = leaf == l0;
    double sn = mine ? an : 0.0, sk = mine ? ak : 0.0, sv = mine ? av : 0.0;
    for (int off = 32; off > 0; off >>= 1) {
      sn += __shfl_xor(sn, off);
      sk += __shfl_xor(sk, off);
      sv += __shfl_xor(sv, off);
    }
    if (lane == lead) {
      unsafeAtomicAdd(g_n + l0, sn);
      unsafeAtomicAdd(g_k + l0, sk);
      unsafeAtomicAdd(g_v + l0, sv);
    }
    if (mine) leaf = -1;
    m = __ballot(leaf >= 0);
  }
  if (leaf >= 0) {
    unsafeAtomicAdd(g_n + leaf, an);
    unsafeAtomicAdd(g_k + leaf, ak);
    unsafeAtomicAdd(g_v + leaf, av);
  }
}

// Gradient terms of one crossing (segment seg of leaf record lf) of a ray
// at x_ext xr with weight g = -G_p w exp(-tau): d/dn_HI, d/dkappa_d and
// d/dv_los of g tau_c (formulas below).
template <class R>
__device__ __forceinline__ void crossing_grad(const ProblemK &pb, const LeafRec<R> &lf, double xr, const R kr[3],
                                              double seg, double g, double inv_vth_ref, double *an, double *ak,
                                              double *av) {
  Opac<R> o;
  opacity(pb, lf, xr, kr, o);
  const R b = R(pb.b_ref);
  const R den = R(1) + b * o.w;
  R sn = R(0), sv = R(0);
#pragma unroll
  for (int i = 0; i < MAX_LINES; ++i) {
    if (i < pb.n_lines) {
      const LineK &ln = pb.lines[i];
      const R a = R(ln.alpha) * lf.irho;
      sn += R(ln.kfac) * voigt_h<R>(a, o.x[i]);
      const R dxdw = M<R>::div(-lf.irho * R(ln.inv_mu) * R(ln.s) * (R(1) + b * (R)xr), den * den);
      sv += R(ln.kfac) * voigt_dhdx<R>(a, o.x[i]) * dxdw;
    }
  }
  *an = g * seg * pb.box_cm * (double)lf.irho * (double)sn;
  *ak = g * seg * pb.box_cm;
  *av = g * seg * (double)lf.nl * (double)sv * inv_vth_ref;
}

// dL/dtheta_c = -G_p w exp(-tau) sum over the ray's crossings of c of
// dtau/dtheta_c, with tau_c = (nl sum_i kfac_i H_i + kd) seg:
//   dtau/dn_HI   = seg box irho sum_i kfac_i H_i
//   dtau/dkappa_d = seg box
//   dtau/dv_los  = seg nl sum_i kfac_i H'_i dx_i/dw / v_th,ref,
//   dx_i/dw = -irho inv_mu_i s_i (1 + b x_ext) / (1 + b w)^2.
template <class R>
__global__ void __launch_bounds__(256) k_image_bwd(ProblemK pb, int obs, int64_t n, const double *__restrict__ orig,
                            const double *__restrict__ x_ext, const double *__restrict__ w,
                            const double *__restrict__ G, double inv_vth_ref,
                            double *__restrict__ g_n, double *__restrict__ g_k,
                            double *__restrict__ g_v, unsigned long long *__restrict__ ncross) {
  extern __shared__ int lds[];
  int *stk = lds + threadIdx.x;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = __lane_id();
  uint32_t nc = 0;
  const double *k = pb.obs[obs].k;
  const R kr[3] = {(R)k[0], (R)k[1], (R)k[2]};
  bool walking = false;
  double g = 0.0, xr = 0.0;
  double p[3] = {0.0, 0.0, 0.0};
  Cell c;
  uint32_t steps = 0;
  if (r < n) {
    const ObsK &ob = pb.obs[obs];
    const double p0[3] = {orig[3 * r], orig[3 * r + 1], orig[3 * r + 2]};
    const int pix = pixel_of(ob, p0);
    xr = x_ext[r];
    double tau = TauCut<double>::v;
    if (pix >= 0)
      tau = ray_tau<R>(pb, p0, ob.k, xr, TauCut<double>::v, stk, blockDim.x, &nc, nullptr,
                       sizeof(R) == 4 ? ob.kinv : nullptr);
    g = (pix >= 0 && tau < TauCut<double>::v) ? -G[pix] * w[r] * exp(-tau) : 0.0;
    if (g != 0.0) {
      // replay the ray (same traversal as the forward pass)
      p[0] = p0[0]; p[1] = p0[1]; p[2] = p0[2];
      int X[3];
      if (int_coords(pb.L, p, k, X)) {
        locate(pb, X, stk, blockDim.x, c);
        walking = true;
      }
    }
  }
  // The wave walks its rays in step (every lane runs every iteration) so
  // that the gradient contributions of lanes in the same leaf are summed
  // across the wave first: rays from one source share their cells, and
  // one atomic per leaf replaces up to 64.  Every lane reaches the
  // shuffles below (no lane has left the loop), so their sources are live.
  while (__ballot(walking)) {
    int leaf = -1;
    double an = 0.0, ak = 0.0, av = 0.0;
    if (walking) {
      const LeafRec<R> lf = load_leaf<R>(pb.leaves, c.leaf);
      double face[3], lo[3], hi[3];
      int em;
      const double te = exit_dist(c, pb.L, p, k, face, lo, hi, &em, sizeof(R) == 4 ? pb.obs[obs].kinv : nullptr);
      const double td = domain_dist_leaf(lf, pb.domain, pb.dom, p, k);
      const double seg = td <= te ? td : te;
      crossing_grad<R>(pb, lf, xr, kr, seg, g, inv_vth_ref, &an, &ak, &av);
      leaf = c.leaf;
      if (td <= te) {
        walking = false;
      } else {
        double pn[3];
        exit_point(te, em, p, k, face, lo, hi, pn);
        p[0] = pn[0]; p[1] = pn[1]; p[2] = pn[2];
        wrap_slab(pb.domain, p, k);
        int X[3];
        if (!int_coords(pb.L, p, k, X)) {
          walking = false;
        } else {
          relocate(pb, X, stk, blockDim.x, c);
          if (++steps >= MAX_CROSS) walking = false;
        }
      }
    }
    wave_leaf_add(leaf, an, ak, av, g_n, g_k, g_v, lane);
  }
  unsigned long long v = nc;
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
  if (lane == 0 && v) atomicAdd(ncross, v);
}

// Peel-off image of fixed rays that also records each ray's crossings (the
// tape read by k_image_bwd_tape).  The 64 rays of a wave walk in step, one
// leaf per iteration; every TAPE_CHUNK iterations the wave takes a new
// chunk (one atomic) and links it to its last one.  A wave that finds no
// chunk left goes on without recording (the host sees the count of chunks
// requested exceed the capacity and runs the pass again with more).  The
// walk and the optical depth are those of ray_tau, so the image equals the
// one k_image_fwd makes, up to the order of the additions.
template <class R>
__global__ void __launch_bounds__(256) k_image_fwd_tape(ProblemK pb, int obs, int64_t n,
                                                        const double *__restrict__ orig,
                                                        const double *__restrict__ x_ext,
                                                        const double *__restrict__ w, double *__restrict__ image,
                                                        unsigned long long *__restrict__ ncross, TapeK tp) {
  extern __shared__ int lds[];
  int *stk = lds + threadIdx.x;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t wave = r >> 6;
  const int lane = __lane_id();
  const ObsK &ob = pb.obs[obs];
  const double *k = ob.k;
  const R kr[3] = {(R)k[0], (R)k[1], (R)k[2]};
  const double *kinv = sizeof(R) == 4 ? ob.kinv : nullptr;
  const double cut = TauCut<double>::v;
  bool walking = false;
  int pix = -1;
  double xr = 0.0, tau = 0.0;
  double p[3] = {0.0, 0.0, 0.0};
  Cell c;
  uint32_t nc = 0;
  if (r < n) {
    p[0] = orig[3 * r]; p[1] = orig[3 * r + 1]; p[2] = orig[3 * r + 2];
    pix = pixel_of(ob, p);
    xr = x_ext[r];
    int X[3];
    if (pix >= 0 && int_coords(pb.L, p, k, X)) {
      locate(pb, X, stk, blockDim.x, c);
      walking = true;
    }
  }
  if (lane == 0) tp.first[wave] = -1;
  int64_t chunk = -1;   // wave-uniform
  for (uint32_t i = 0; __ballot(walking); ++i) {
    if (i % TAPE_CHUNK == 0) {
      unsigned long long q = 0;
      if (lane == 0) q = atomicAdd(tp.ctl, 1ull);
      q = __shfl(q, 0);
      const int64_t nxt = q < tp.cap ? (int64_t)q : -1;
      if (lane == 0) {
        if (i == 0) tp.first[wave] = nxt;
        else if (chunk >= 0) tp.next[chunk] = nxt;
        if (nxt >= 0) tp.next[nxt] = -1;
      }
      chunk = nxt;
    }
    if (walking) {
      const LeafRec<R> lf = load_leaf<R>(pb.leaves, c.leaf);
      Opac<R> o;
      opacity(pb, lf, xr, kr, o);
      double face[3], lo[3], hi[3];
      int em;
      const double te = exit_dist(c, pb.L, p, k, face, lo, hi, &em, kinv);
      const double td = domain_dist_leaf(lf, pb.domain, pb.dom, p, k);
      const double seg = td <= te ? td : te;
      ++nc;
      if (chunk >= 0) {
        const size_t e = (size_t)chunk * TAPE_ENTRIES + (size_t)(i % TAPE_CHUNK) * 64 + lane;
        tp.leaf[e] = c.leaf;
        ((R *)tp.seg)[e] = (R)seg;
      }
      tau += (double)o.ktot * seg;
      if (td <= te || tau >= cut) {
        walking = false;
      } else {
        double pn[3];
        exit_point(te, em, p, k, face, lo, hi, pn);
        p[0] = pn[0]; p[1] = pn[1]; p[2] = pn[2];
        wrap_slab(pb.domain, p, k);
        int X[3];
        if (!int_coords(pb.L, p, k, X) || nc >= MAX_CROSS) {
          walking = false;
        } else {
          relocate(pb, X, stk, blockDim.x, c);
        }
      }
    }
  }
  if (r < n) {
    const double wt = (pix >= 0 && tau < cut) ? w[r] * exp(-tau) : 0.0;
    if (wt != 0.0) unsafeAtomicAdd(image + pix, wt);
    tp.count[r] = (int32_t)nc;
    tp.pix[r] = pix;
    tp.wt[r] = wt;
    tp.x[r] = xr;
  }
  unsigned long long v = nc;
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
  if (lane == 0 && v) atomicAdd(ncross, v);
}

// Adjoint of the image from the tape of the last k_image_fwd_tape pass (same
// rays, same wave of 64 rays per 64 lanes): the crossings are read back in
// the order they were walked, so no geometry and no optical depth are
// computed again.  The gradient terms and their per-leaf wave sums are
// those of k_image_bwd.
template <class R>
__global__ void __launch_bounds__(256) k_image_bwd_tape(ProblemK pb, int obs, int64_t n, TapeK tp,
                                                        const double *__restrict__ G, double inv_vth_ref,
                                                        double *__restrict__ g_n, double *__restrict__ g_k,
                                                        double *__restrict__ g_v,
                                                        unsigned long long *__restrict__ ncross) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t wave = r >> 6;
  const int lane = __lane_id();
  const double *k = pb.obs[obs].k;
  const R kr[3] = {(R)k[0], (R)k[1], (R)k[2]};
  double g = 0.0, xr = 0.0;
  int cnt = 0;
  if (r < n) {
    const double wt = tp.wt[r];
    if (wt != 0.0) {
      g = -G[tp.pix[r]] * wt;
      if (g != 0.0) {
        cnt = tp.count[r];
        xr = tp.x[r];
      }
    }
  }
  // wave iterations needed: the longest crossing list among lanes with a
  // gradient (every lane's list starts at the wave's first iteration)
  int m = cnt;
  for (int off = 32; off > 0; off >>= 1) m = max(m, __shfl_xor(m, off));
  int64_t chunk = m > 0 ? tp.first[wave] : -1;
  for (int i = 0; i < m; ++i) {
    if (i > 0 && i % TAPE_CHUNK == 0) chunk = tp.next[chunk];
    if (chunk < 0) break;   // an incomplete tape (the host never passes one)
    int leaf = -1;
    double an = 0.0, ak = 0.0, av = 0.0;
    if (i < cnt) {
      const size_t e = (size_t)chunk * TAPE_ENTRIES + (size_t)(i % TAPE_CHUNK) * 64 + lane;
      leaf = tp.leaf[e];
      const double seg = (double)((const R *)tp.seg)[e];
      const LeafRec<R> lf = load_leaf<R>(pb.leaves, leaf);
      crossing_grad<R>(pb, lf, xr, kr, seg, g, inv_vth_ref, &an, &ak, &av);
    }
    wave_leaf_add(leaf, an, ak, av, g_n, g_k, g_v, lane);
  }
  unsigned long long v = (unsigned long long)cnt;
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
  if (lane == 0 && v) atomicAdd(ncross, v);
}

// ----------------------------------------------------- gas and sources in
// Gas fields as given (float or double; v is [3n]) checked and copied into
// the raw per-leaf array raw[8n] = {n_HI, T, vx, vy, vz, kappa_d, 0, 0} in
// double.  bad[0] receives the smallest leaf with a non-finite or negative
// value (or T <= 0), bad[1] the smallest with a velocity component of at
// least 0.1 c; both start at ~0 (set by the caller).
template <class T>
__global__ void k_stage_gas(int64_t n, const T *__restrict__ nh, const T *__restrict__ tk,
                            const T *__restrict__ v, const T *__restrict__ kd, double *__restrict__ raw,
                            unsigned long long *__restrict__ bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double a = (double)nh[i], t = (double)tk[i], k = (double)kd[i];
  const double vx = (double)v[3 * i], vy = (double)v[3 * i + 1], vz = (double)v[3 * i + 2];
  const bool ok = isfinite(a) && a >= 0.0 && isfinite(t) && t > 0.0 && isfinite(k) && k >= 0.0 && isfinite(vx) &&
                  isfinite(vy) && isfinite(vz);
  const double vmax = 0.1 * 2.99792458e10;
  if (!ok) atomicMin(bad, (unsigned long long)i);
  else if (fabs(vx) >= vmax || fabs(vy) >= vmax || fabs(vz) >= vmax) atomicMin(bad + 1, (unsigned long long)i);
  double *r = raw + 8 * i;
  r[0] = a; r[1] = t; r[2] = vx; r[3] = vy; r[4] = vz; r[5] = k; r[6] = 0.0; r[7] = 0.0;
}

// Leaf records (see rmc_device.h) from the raw gas: nl = n_HI box irho,
// irho = sqrt(T_ref / T), kd = kappa_d box, u = v / v_th,ref, and the
// domain-border flag of the leaf (level lv, integer coordinates ijk at its
// level): box -- touches a face of the cube; slab -- not strictly inside
// the slab; sphere -- some corner outside R (1 - 1e-9).  Plain IEEE double
// arithmetic, uncontracted, so the records are exact functions of the
// inputs; the float path rounds them once.
#pragma clang fp contract(off)
template <class R>
__global__ void k_leaf_records(int64_t n, const double *__restrict__ raw, const int8_t *__restrict__ lv,
                               const int32_t *__restrict__ ijk, double T_ref, double vth_ref, double box,
                               int domain, double d0, double d1, double d2, double d3, R *__restrict__ leaves) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double *g = raw + 8 * i;
  const double irho = sqrt(T_ref / g[1]);
  const int l = lv[i];
  const double h = ldexp(1.0, -l);
  double lo[3], hi[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    lo[d] = (double)ijk[3 * i + d] * h;
    hi[d] = (double)(ijk[3 * i + d] + 1) * h;
  }
  bool border;
  if (domain == DOM_BOX) {
    border = lo[0] <= 0.0 || hi[0] >= 1.0 || lo[1] <= 0.0 || hi[1] >= 1.0 || lo[2] <= 0.0 || hi[2] >= 1.0;
  } else if (domain == DOM_SLAB_Z) {
    border = !(lo[2] > d0 - d1 && hi[2] < d0 + d1);
  } else {
    const double Rr = d3 * (1.0 - 1e-9);
    const double c[3] = {d0, d1, d2};
    double far2 = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double a = fabs(lo[d] - c[d]), b = fabs(hi[d] - c[d]);
      const double m = a > b ? a : b;
      far2 += m * m;
    }
    border = !(far2 < Rr * Rr);
  }
  const double rec[8] = {g[0] * box * irho, irho, g[5] * box, g[2] / vth_ref, g[3] / vth_ref, g[4] / vth_ref,
                         border ? 1.0 : 0.0, log10(irho)};
  R *o = leaves + (size_t)i * LEAF_STRIDE;
#pragma unroll
  for (int q = 0; q < 8; ++q) o[q] = (R)rec[q];
}

// Device-resident sources checked as the host path checks them: positions
// in [0,1], finite x, unit directions (|k|^2 within 1e-6 of 1).  bad[0]
// receives the smallest failing source.
__global__ void k_check_sources(int64_t n, const double *__restrict__ pos, const double *__restrict__ dir,
                                const double *__restrict__ x, unsigned long long *__restrict__ bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  bool ok = isfinite(x[i]);
#pragma unroll
  for (int d = 0; d < 3; ++d) ok = ok && pos[3 * i + d] >= 0.0 && pos[3 * i + d] <= 1.0;
  if (dir) {
    const double nn = dir[3 * i] * dir[3 * i] + dir[3 * i + 1] * dir[3 * i + 1] + dir[3 * i + 2] * dir[3 * i + 2];
    ok = ok && fabs(nn - 1.0) < 1e-6;
  }
  if (!ok) atomicMin(bad, (unsigned long long)i);
}

// Gradient with respect to the cell velocity vector from the one with
// respect to v_los = k_obs . v (chain rule): g_v[3i + d] = g_vlos[i] k_d.
__global__ void k_vlos_to_v(int64_t n, const double *__restrict__ g_vlos, double k0, double k1, double k2,
                            double *__restrict__ g_v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double g = g_vlos[i];
  g_v[3 * i] = g * k0;
  g_v[3 * i + 1] = g * k1;
  g_v[3 * i + 2] = g * k2;
}
#pragma clang fp contract(fast)

// --------------------------------------------------------------- helpers
__global__ void k_hist(int64_t n, const int32_t *__restrict__ status, const double *__restrict__ x,
                       int nbins, double x_min, double span, unsigned long long *__restrict__ h) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || status[i] != ST_ESCAPED) return;
  const double fb = (x[i] - x_min) / span * nbins;
  if (!(fb >= 0.0 && fb < nbins)) return;
  const int b = (int)floor(fb);
  if (b < nbins) atomicAdd(h + b, 1ull);
}

// Zero the counters of every problem of a launch and the work queue (a
// kernel rather than a memset so that it can sit in a captured graph).
__global__ void k_batch_reset(const ProblemK *__restrict__ probs, int n, unsigned long long *next) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n * N_STATS) probs[i / N_STATS].stats[i % N_STATS] = 0ull;
  if (i == 0) *next = 0ull;
}

__global__ void k_fill_u64(unsigned long long *p, int64_t n, unsigned long long v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_u64_to_f64(const unsigned long long *a, double *b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (double)a[i];
}

__global__ void k_f32_to_f64(const float *a, double *b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (double)a[i];
}

__global__ void k_f64_to_f32(const double *a, float *b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}

// ------------------------------------------ fixed scratch (no allocation)
// Histogram counts of rmc_get_spectrum_noalloc: a file-scope device array
// of NOALLOC_MAX_BINS counters (each device the library runs on holds its
// own copy until the process ends).  Host code never uses the array's name
// as an address: scratch_address() asks the runtime for the current
// device's copy once and keeps it.
static __device__ __align__(256) unsigned long long scratch[NOALLOC_MAX_BINS];

hipError_t scratch_address(int device, unsigned long long **out) {
  static std::mutex mu;
  static unsigned long long *addr[256] = {};
  if (device < 0 || device >= 256) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(mu);
  if (!addr[device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[device] = (unsigned long long *)p;
  }
  *out = addr[device];
  return hipSuccess;
}

// ------------------------------------------------------------- launchers
static inline unsigned blocks_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

using TransportFn = void (*)(const ProblemK *, const int64_t *, int, unsigned long long *, int, int, SlotState *,
                            int, unsigned long long *);

// The one-round-per-pass form (regroup) is built for the deferred
// peel-off kernels only (the default); the one-wave tail form for the
// single-problem deferred kernels.
template <class R, int NL>
static TransportFn transport_fn(bool batch, bool defer, bool regroup, bool tail) {
  if (batch) {
    if (!defer) return k_transport<R, true, false, NL>;
    return regroup ? k_transport<R, true, true, NL, true> : k_transport<R, true, true, NL>;
  }
  if (!defer) return k_transport<R, false, false, NL>;
  if (tail) return regroup ? k_transport<R, false, true, NL, true, true> : k_transport<R, false, true, NL, false, true>;
  return regroup ? k_transport<R, false, true, NL, true> : k_transport<R, false, true, NL>;
}

static TransportFn transport_fn(bool fp32, bool batch, bool defer, bool one_line, bool regroup, bool tail = false) {
  if (fp32)
    return one_line ? transport_fn<float, 1>(batch, defer, regroup, tail)
                    : transport_fn<float, MAX_LINES>(batch, defer, regroup, tail);
  return one_line ? transport_fn<double, 1>(batch, defer, regroup, tail)
                  : transport_fn<double, MAX_LINES>(batch, defer, regroup, tail);
}

static size_t transport_lds(int stack_levels, int block) {
  return ((size_t)2 * stack_levels * block + block / 64) * sizeof(int);
}

hipError_t launch_transport(bool fp32, bool batch, bool defer, bool one_line, bool regroup, const ProblemK *d_probs,
                            const int64_t *d_starts, int n_probs, unsigned long long *d_next, int refill_min,
                            int stack_levels, int grid, int block, void *slots, int budget,
                            unsigned long long *slice, hipStream_t st, bool tail) {
  hipLaunchKernelGGL(transport_fn(fp32, batch, defer, one_line, regroup, tail), dim3(grid), dim3(block),
                     transport_lds(stack_levels, block), st,
                     d_probs, d_starts, n_probs, d_next, refill_min, stack_levels, (SlotState *)slots, budget, slice);
  return hipGetLastError();
}

using DrainFn = void (*)(const ProblemK *, PeelQueue *, unsigned long long *);

template <class R>
static DrainFn drain_fn(bool batch, bool one_line) {
  if (batch) return one_line ? k_peel_drain<R, true, 1> : k_peel_drain<R, true, MAX_LINES>;
  return one_line ? k_peel_drain<R, false, 1> : k_peel_drain<R, false, MAX_LINES>;
}

static DrainFn drain_fn(bool fp32, bool batch, bool one_line) {
  return fp32 ? drain_fn<float>(batch, one_line) : drain_fn<double>(batch, one_line);
}

hipError_t launch_peel_drain(bool fp32, bool batch, bool one_line, const ProblemK *d_probs, void *pq,
                             int stack_levels, int grid, unsigned long long *slice, hipStream_t st) {
  const int b = 256;
  const size_t lds = (size_t)stack_levels * b * sizeof(int);
  PeelQueue *q = (PeelQueue *)pq;
  hipLaunchKernelGGL(drain_fn(fp32, batch, one_line), dim3(grid), dim3(b), lds, st, d_probs, q, slice);
  if (hipError_t e = hipGetLastError()) return e;
  hipLaunchKernelGGL(k_peel_reset, dim3(1), dim3(64), 0, st, q, slice);
  return hipGetLastError();
}

int peel_drain_blocks_per_cu(bool fp32, bool batch, bool one_line, int stack_levels) {
  const size_t lds = (size_t)stack_levels * 256 * sizeof(int);
  int nb = 0;
  const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, drain_fn(fp32, batch, one_line), 256, lds);
  return (e == hipSuccess && nb > 0) ? nb : 1;
}

size_t peel_job_bytes(bool fp32) { return fp32 ? sizeof(PeelJob<float>) : sizeof(PeelJob<double>); }
size_t peel_queue_bytes() { return sizeof(PeelQueue); }

size_t slot_bytes() { return sizeof(SlotState); }

int transport_blocks_per_cu(bool fp32, bool batch, bool defer, bool one_line, bool regroup, int block,
                            int stack_levels) {
  int nb = 0;
  const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb,
                                                                    transport_fn(fp32, batch, defer, one_line, regroup),
                                                                    block,
                                                                    transport_lds(stack_levels, block));
  return (e == hipSuccess && nb > 0) ? nb : 1;
}

hipError_t launch_clear_slots(void *slots, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_clear_slots, dim3(blocks_for(n, 256)), dim3(256), 0, st, (SlotState *)slots, n);
  return hipGetLastError();
}

hipError_t launch_compact_slots(const void *src, int64_t n, void *dst, unsigned long long *n_live,
                                hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_compact_slots, dim3(blocks_for(n, 256)), dim3(256), 0, st, (const SlotState *)src, n,
                     (SlotState *)dst, n_live);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(n, 256)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

hipError_t launch_count_live(const void *slots, int64_t n, unsigned long long *out, hipStream_t st) {
  hipLaunchKernelGGL(k_count_live, dim3(blocks_for(n, 256)), dim3(256), 0, st, (const SlotState *)slots, n, out);
  return hipGetLastError();
}

hipError_t launch_trace(const ProblemK &pb, int64_t n, const double *orig, const double *dir,
                        int max_cells, int32_t *leaf, double *seg, int32_t *cnt, hipStream_t st) {
  const int b = 256;
  const size_t lds = (size_t)(pb.L > 0 ? pb.L : 1) * b * sizeof(int);
  hipLaunchKernelGGL(k_trace, dim3(blocks_for(n, b)), dim3(b), lds, st, pb, n, orig, dir, max_cells, leaf,
                     seg, cnt);
  return hipGetLastError();
}

hipError_t launch_tau(bool fp32, const ProblemK &pb, int64_t n, const double *orig, const double *dir,
                      const double *x, double *tau, hipStream_t st) {
  const int b = 256;
  const size_t lds = (size_t)(pb.L > 0 ? pb.L : 1) * b * sizeof(int);
  if (fp32)
    hipLaunchKernelGGL(k_tau<float>, dim3(blocks_for(n, b)), dim3(b), lds, st, pb, n, orig, dir, x, tau);
  else
    hipLaunchKernelGGL(k_tau<double>, dim3(blocks_for(n, b)), dim3(b), lds, st, pb, n, orig, dir, x, tau);
  return hipGetLastError();
}

hipError_t launch_image_fwd(bool fp32, const ProblemK &pb, int obs, int64_t n, const double *orig,
                            const double *x, const double *w, double *image, unsigned long long *ncross,
                            hipStream_t st) {
  const int b = 256;
  const size_t lds = (size_t)(pb.L > 0 ? pb.L : 1) * b * sizeof(int);
  if (fp32)
    hipLaunchKernelGGL(k_image_fwd<float>, dim3(blocks_for(n, b)), dim3(b), lds, st, pb, obs, n, orig, x, w,
                       image, ncross);
  else
    hipLaunchKernelGGL(k_image_fwd<double>, dim3(blocks_for(n, b)), dim3(b), lds, st, pb, obs, n, orig, x, w,
                       image, ncross);
  return hipGetLastError();
}

hipError_t launch_image_bwd(bool fp32, const ProblemK &pb, int obs, int64_t n, const double *orig,
                            const double *x, const double *w, const double *G, double inv_vth_ref,
                            double *gn, double *gk, double *gv, unsigned long long *ncross, hipStream_t st) {
  const int b = 256;
  const size_t lds = (size_t)(pb.L > 0 ? pb.L : 1) * b * sizeof(int);
  if (fp32)
    hipLaunchKernelGGL(k_image_bwd<float>, dim3(blocks_for(n, b)), dim3(b), lds, st, pb, obs, n, orig, x, w, G,
                       inv_vth_ref, gn, gk, gv, ncross);
  else
    hipLaunchKernelGGL(k_image_bwd<double>, dim3(blocks_for(n, b)), dim3(b), lds, st, pb, obs, n, orig, x, w, G,
                       inv_vth_ref, gn, gk, gv, ncross);
  return hipGetLastError();
}

int64_t tape_waves(int64_t n) { return (int64_t)blocks_for(n, 256) * 4; }

hipError_t launch_image_fwd_tape(bool fp32, const ProblemK &pb, int obs, int64_t n, const double *orig,
                                 const double *x, const double *w, double *image, unsigned long long *ncross,
                                 const TapeK &tp, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int b = 256;
  const size_t lds = (size_t)(pb.L > 0 ? pb.L : 1) * b * sizeof(int);
  if (fp32)
    hipLaunchKernelGGL(k_image_fwd_tape<float>, dim3(blocks_for(n, b)), dim3(b), lds, st, pb, obs, n, orig, x, w,
                       image, ncross, tp);
  else
    hipLaunchKernelGGL(k_image_fwd_tape<double>, dim3(blocks_for(n, b)), dim3(b), lds, st, pb, obs, n, orig, x, w,
                       image, ncross, tp);
  return hipGetLastError();
}

hipError_t launch_image_bwd_tape(bool fp32, const ProblemK &pb, int obs, int64_t n, const TapeK &tp,
                                 const double *G, double inv_vth_ref, double *gn, double *gk, double *gv,
                                 unsigned long long *ncross, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int b = 256;
  if (fp32)
    hipLaunchKernelGGL(k_image_bwd_tape<float>, dim3(blocks_for(n, b)), dim3(b), 0, st, pb, obs, n, tp, G,
                       inv_vth_ref, gn, gk, gv, ncross);
  else
    hipLaunchKernelGGL(k_image_bwd_tape<double>, dim3(blocks_for(n, b)), dim3(b), 0, st, pb, obs, n, tp, G,
                       inv_vth_ref, gn, gk, gv, ncross);
  return hipGetLastError();
}

hipError_t launch_stage_gas(bool f32_in, int64_t n, const void *nh, const void *tk, const void *v, const void *kd,
                           double *raw, unsigned long long *bad, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if (f32_in)
    hipLaunchKernelGGL(k_stage_gas<float>, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, (const float *)nh,
                       (const float *)tk, (const float *)v, (const float *)kd, raw, bad);
  else
    hipLaunchKernelGGL(k_stage_gas<double>, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, (const double *)nh,
                       (const double *)tk, (const double *)v, (const double *)kd, raw, bad);
  return hipGetLastError();
}

hipError_t launch_leaf_records(bool fp32, int64_t n, const double *raw, const int8_t *lv, const int32_t *ijk,
                               double T_ref, double vth_ref, double box, int domain, const double dom[4],
                               void *leaves, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if (fp32)
    hipLaunchKernelGGL(k_leaf_records<float>, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, raw, lv, ijk, T_ref,
                       vth_ref, box, domain, dom[0], dom[1], dom[2], dom[3], (float *)leaves);
  else
    hipLaunchKernelGGL(k_leaf_records<double>, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, raw, lv, ijk, T_ref,
                       vth_ref, box, domain, dom[0], dom[1], dom[2], dom[3], (double *)leaves);
  return hipGetLastError();
}

hipError_t launch_check_sources(int64_t n, const double *pos, const double *dir, const double *x,
                                unsigned long long *bad, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_check_sources, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, pos, dir, x, bad);
  return hipGetLastError();
}

hipError_t launch_vlos_to_v(int64_t n, const double *g_vlos, const double k[3], double *g_v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_vlos_to_v, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, g_vlos, k[0], k[1], k[2], g_v);
  return hipGetLastError();
}

hipError_t launch_hist(int64_t n, const int32_t *status, const double *x, int nbins, double x_min, double span,
                       unsigned long long *h, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_hist, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, status, x, nbins, x_min, span, h);
  return hipGetLastError();
}

hipError_t launch_batch_reset(const ProblemK *d_probs, int n, unsigned long long *d_next, hipStream_t st) {
  hipLaunchKernelGGL(k_batch_reset, dim3(blocks_for((int64_t)n * N_STATS, 256)), dim3(256), 0, st, d_probs, n,
                     d_next);
  return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long *p, int64_t n, unsigned long long v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u64, dim3(blocks_for(n, 256)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

hipError_t launch_u64_to_f64(const unsigned long long *a, double *b, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_u64_to_f64, dim3(blocks_for(n, 256)), dim3(256), 0, st, a, b, n);
  return hipGetLastError();
}

hipError_t launch_f32_to_f64(const float *a, double *b, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_f32_to_f64, dim3(blocks_for(n, 256)), dim3(256), 0, st, a, b, n);
  return hipGetLastError();
}

hipError_t launch_f64_to_f32(const double *a, float *b, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_f64_to_f32, dim3(blocks_for(n, 256)), dim3(256), 0, st, a, b, n);
  return hipGetLastError();
}

}  // namespace rmc
