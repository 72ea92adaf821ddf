// rmc_api.cpp -- host runtime behind include/rmc.h: contexts, mesh
// validation and breadth-first octree build, per-leaf records, launches.
#include "rmc.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "rmc_launch.h"

// observer bases and pixel spans must be the exact IEEE results of the
// written expressions
#pragma clang fp contract(off)

using namespace rmc;

namespace {

// CGS constants (CODATA 2018)
const double C_LIGHT = 2.99792458e10;
const double H_PLANCK = 6.62607015e-27;
const double K_BOLTZ = 1.380649e-16;
const double E_CHARGE = 4.80320471e-10;
const double M_ELECTRON = 9.1093837015e-28;
const double AMU_G = 1.66053906660e-24;

// Device allocation owned by a context; released explicitly (rmc_destroy
// lists every buffer of the context), since observer records holding one
// are copied when their vector grows.
struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  hipError_t ensure(size_t n) {
    if (n <= bytes && p) return hipSuccess;
    release();
    hipError_t e = hipMalloc(&p, n ? n : 1);
    if (e == hipSuccess) bytes = n;
    else p = nullptr;
    return e;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  template <class T> T *as() const { return (T *)p; }
};

struct ObsHost {
  ObsK k;
  size_t n_elems;
  DevBuf cube;
};

struct LineQ {
  double nu0, vth, dnu, a, sigma0;
};

// Sect. 3.1.1 line quantities at temperature T.
LineQ line_q(const rmc_line &ln, double T) {
  LineQ q;
  q.nu0 = C_LIGHT / (ln.lambda0_A * 1e-8);
  q.vth = std::sqrt(2.0 * K_BOLTZ * T / (ln.mass_amu * AMU_G));
  q.dnu = q.nu0 * q.vth / C_LIGHT;
  q.a = ln.A_ul / (4.0 * 3.14159265358979323846 * q.dnu);
  q.sigma0 = std::sqrt(3.14159265358979323846) * E_CHARGE * E_CHARGE * ln.f_lu / (M_ELECTRON * C_LIGHT * q.dnu);
  return q;
}

}  // namespace

struct rmc_ctx {
  int device = 0;
  int precision = RMC_FP64;
  hipStream_t stream = nullptr;
  std::string err;
  int forward_only = 0;
  int64_t max_events = 0;
  double skip_tau = 0.0, skip_frac = 0.0;
  int voigt_exact = 0;
  int spec_kind = 0;
  double spec_p[3] = {0.0, 0.0, 0.0};
  int block = 256;
  int waves_per_cu = 0;   // 0: as many as the transport kernel's occupancy allows
  int refill = 1;
  int peel_defer = 1;      // peel-off rays past their first leaf go to the ray-cast pass
  int slice_iters = 2048;
  int regroup = 0;         // one rejection round per pass of the transport loop
                           // (default 1 for RMC_FP64 contexts, set in rmc_create)
  int compact = 1;         // gather the last packets of a stream into fewer waves
  // mesh
  bool has_mesh = false;
  int64_t n_leaves = 0;
  int L = 0;
  double box_cm = 0.0;
  int64_t n_nodes = 0;
  DevBuf nodes;
  DevBuf top;              // level-top_level cell table (empty: none)
  int top_level = 0;
  // lines
  bool has_lines = false;
  int n_lines = 0;
  rmc_line lines[MAX_LINES];
  double T_ref = 0.0;
  // gas: raw per-leaf fields on the device (8 doubles per leaf: n_HI, T,
  // v(3), kappa_d, pad) and the leaf records built from them
  bool has_gas = false;
  bool leaves_dirty = false;
  DevBuf g_raw, g_stage, g_in, d_bad;
  DevBuf m_lv, m_ijk;     // leaf levels and integer coordinates (device)
  DevBuf leaves;
  double albedo = 0.32, g_hg = 0.73;
  int domain = RMC_DOM_BOX;
  double dom[4] = {0, 0, 0, 0};
  // sources
  int64_t n_src = 0;
  bool src_dir = false;
  DevBuf spos, sdir, sx;
  std::vector<ObsHost> obs;
  // outputs of the last run
  int64_t last_n = 0;
  DevBuf o_status, o_x, o_k, o_pos, o_nscat, o_path;
  DevBuf d_stats, d_next, d_prob, d_starts, tmp1, tmp2, tmp3, tmp4, tmp5, tmp6;
  DevBuf sx_eff;  // emitted x per source under a source spectrum
  DevBuf tab;     // tabulated continuum: lambda[n], beta[n-1], cum[n]
  int tab_n = 0;
  ProblemK pb_host;
  int64_t starts_host[2];
  int num_cus = 0;
  unsigned long long *scratch = nullptr;   // this device's fixed counters (no-allocation spectrum)
  hipEvent_t ev0 = nullptr, ev1 = nullptr, ev2 = nullptr;
  // batch launches
  DevBuf b_probs, b_starts;
  std::vector<ProblemK> b_host;
  std::vector<int64_t> b_starts_host;
  // streaming state (single problem or a batch led by this context)
  DevBuf slots, d_slice;
  DevBuf slots2, d_live;     // gathered slots (tail of a stream) and their count
  int s_tail_grid = 0;       // >0: blocks of the launches on gathered slots
  int64_t s_total = 0, s_done = 0;
  int s_grid = 0, s_levels = 1, s_nprobs = 0;
  bool s_open = false, s_batch = false;
  const ProblemK *s_probs = nullptr;
  const int64_t *s_starts = nullptr;
  std::vector<rmc_ctx *> s_members;
  rmc_run_stats s_acc;
  hipGraphExec_t s_graph = nullptr;   // slice counters + transport launch
  hipGraphExec_t s_graph2 = nullptr;  // ray-cast pass over the peel-off queue
  std::string s_key;
  PeelQueue *s_pq = nullptr;
  bool image_done = false;           // an image call has filled d_stats and ev0/ev1
  // model generation: bumped by every change of the mesh, lines, gas or domain
  uint64_t gen = 0;
  // tape of the last rmc_raycast_image_tape call (crossing lists for the adjoint)
  DevBuf tp_leaf, tp_seg, tp_next, tp_first, tp_count, tp_pix, tp_wt, tp_x, tp_ctl;
  unsigned long long tp_cap = 0;     // chunks of TAPE_ENTRIES crossings
  bool tp_valid = false;
  int tp_obs = -1;
  int64_t tp_n = 0;
  uint64_t tp_gen = 0;
  bool s_one_line = false;           // every problem of the stream has one line
  bool s_defer = true;               // transport kernel without the inline peel-off walker
                                     // (deferred peel-off, or no observer in the stream)
  // deferred peel-off rays: control block (PeelQueue) and job buffer
  DevBuf pq_ctl, pq_jobs, pq_counts;
  unsigned long long pq_cap = 0, pq_regions = 0;
};

namespace {

rmc_status fail(rmc_ctx *c, rmc_status s, const char *fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    c->err = buf;
  }
  return s;
}

#define HIPCHK(ctx, expr)                                                                   \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return fail(ctx, e_ == hipErrorOutOfMemory ? RMC_ENOMEM : RMC_EDEVICE, "%s: %s", #expr, \
                  hipGetErrorString(e_));                                                   \
  } while (0)

bool finite_nonneg(double v) { return std::isfinite(v) && v >= 0.0; }

uint64_t spread3(uint64_t v) {
  v &= 0xFFFFull;
  v = (v | (v << 16)) & 0x0000FF0000FFull;
  v = (v | (v << 8)) & 0x00F00F00F00F00Full;
  v = (v | (v << 4)) & 0x0C30C30C30C30C3ull;
  v = (v | (v << 2)) & 0x249249249249249ull;
  return v;
}
// Morton code with x in the lowest bit of each triple: the child octant
// index of the node array is x | y<<1 | z<<2.
uint64_t morton(uint32_t x, uint32_t y, uint32_t z) { return spread3(x) | (spread3(y) << 1) | (spread3(z) << 2); }

bool sorted_has(const std::vector<uint64_t> &v, uint64_t key) { return std::binary_search(v.begin(), v.end(), key); }

// Validate the leaves (Sect. 4.3 graded octree) and build the breadth-first
// node array: nodes of each level in Morton order, which is the order a
// breadth-first walk visiting children by octant produces.
rmc_status build_tree(int64_t n, const int8_t *level, const int32_t *ijk, std::vector<int32_t> &nodes, int &L,
                      std::string &msg) {
  char buf[256];
  if (n <= 0 || !level || !ijk) {
    msg = "empty mesh";
    return RMC_EINVAL;
  }
  if (n >= (int64_t)1 << 31) {
    msg = "too many leaves";
    return RMC_EINVAL;
  }
  L = 0;
  for (int64_t c = 0; c < n; ++c) {
    if (level[c] < 0 || level[c] > MAX_LEVEL) {
      snprintf(buf, sizeof buf, "leaf %lld: level %d outside [0,%d]", (long long)c, (int)level[c], MAX_LEVEL);
      msg = buf;
      return RMC_EMESH;
    }
    L = std::max(L, (int)level[c]);
  }
  std::vector<std::vector<std::pair<uint64_t, int32_t>>> lv(L + 1);
  for (int64_t c = 0; c < n; ++c) {
    const int l = level[c];
    const int64_t side = (int64_t)1 << l;
    const int64_t i = ijk[3 * c], j = ijk[3 * c + 1], k = ijk[3 * c + 2];
    if (i < 0 || j < 0 || k < 0 || i >= side || j >= side || k >= side) {
      snprintf(buf, sizeof buf, "leaf %lld: coordinates out of range for level %d", (long long)c, l);
      msg = buf;
      return RMC_EMESH;
    }
    lv[l].emplace_back(morton((uint32_t)i, (uint32_t)j, (uint32_t)k), (int32_t)c);
  }
  std::vector<std::vector<uint64_t>> leafkeys(L + 1), inner(L + 1);
  for (int l = 0; l <= L; ++l) {
    std::sort(lv[l].begin(), lv[l].end());
    leafkeys[l].resize(lv[l].size());
    for (size_t q = 0; q < lv[l].size(); ++q) {
      leafkeys[l][q] = lv[l][q].first;
      if (q && leafkeys[l][q] == leafkeys[l][q - 1]) {
        snprintf(buf, sizeof buf, "duplicate leaf at level %d (leaf %d)", l, lv[l][q].second);
        msg = buf;
        return RMC_EMESH;
      }
    }
  }
  for (int l = L; l >= 1; --l) {
    std::vector<uint64_t> &par = inner[l - 1];
    par.reserve(leafkeys[l].size() / 4 + inner[l].size() / 4 + 1);
    for (uint64_t m : leafkeys[l]) par.push_back(m >> 3);
    for (uint64_t m : inner[l]) par.push_back(m >> 3);
    std::sort(par.begin(), par.end());
    par.erase(std::unique(par.begin(), par.end()), par.end());
  }
  for (int l = 0; l <= L; ++l) {
    // a leaf that is also an ancestor of other leaves overlaps them
    std::vector<uint64_t> both;
    std::set_intersection(leafkeys[l].begin(), leafkeys[l].end(), inner[l].begin(), inner[l].end(),
                          std::back_inserter(both));
    if (!both.empty()) {
      snprintf(buf, sizeof buf, "overlapping leaves: a level-%d leaf contains finer leaves", l);
      msg = buf;
      return RMC_EMESH;
    }
  }
  nodes.clear();
  if (L == 0) {
    if (n != 1) {
      msg = "more than one level-0 leaf";
      return RMC_EMESH;
    }
    return RMC_OK;
  }
  std::vector<int64_t> off(L + 1, 0);
  for (int l = 1; l <= L; ++l) off[l] = off[l - 1] + (int64_t)inner[l - 1].size();
  const int64_t n_nodes = off[L];
  if (n_nodes >= (int64_t)1 << 31) {
    msg = "too many nodes";
    return RMC_EINVAL;
  }
  nodes.assign((size_t)n_nodes * 8, 0);
  for (int l = 0; l < L; ++l) {
    const auto &in_next = inner[l + 1];
    const auto &lf_next = leafkeys[l + 1];
    for (size_t r = 0; r < inner[l].size(); ++r) {
      const uint64_t m = inner[l][r];
      for (int oct = 0; oct < 8; ++oct) {
        const uint64_t cm = (m << 3) | (uint64_t)oct;
        int32_t v;
        auto it = std::lower_bound(in_next.begin(), in_next.end(), cm);
        if (it != in_next.end() && *it == cm) {
          v = (int32_t)(off[l + 1] + (it - in_next.begin()));
        } else {
          auto jt = std::lower_bound(lf_next.begin(), lf_next.end(), cm);
          if (jt == lf_next.end() || *jt != cm) {
            snprintf(buf, sizeof buf, "gap: level-%d cell under node %lld octant %d is not covered", l + 1,
                     (long long)(off[l] + (int64_t)r), oct);
            msg = buf;
            return RMC_EMESH;
          }
          v = -(lv[l + 1][jt - lf_next.begin()].second) - 1;
        }
        nodes[(size_t)(off[l] + (int64_t)r) * 8 + oct] = v;
      }
    }
  }
  // 2:1 grading across faces: the level-(l-2) ancestor of each same-size
  // face neighbour must be refined (an inner node)
  std::vector<int> bad_t;
  const int nt = std::max(1, std::min(16, (int)std::thread::hardware_concurrency()));
  std::vector<int64_t> bad(nt, -1);
  std::vector<std::thread> th;
  for (int t = 0; t < nt; ++t) {
    th.emplace_back([&, t]() {
      for (int64_t c = t; c < n; c += nt) {
        const int l = level[c];
        if (l < 2) continue;
        const int64_t side = (int64_t)1 << l;
        for (int d = 0; d < 3; ++d)
          for (int sg = -1; sg <= 1; sg += 2) {
            int64_t nb[3] = {ijk[3 * c], ijk[3 * c + 1], ijk[3 * c + 2]};
            nb[d] += sg;
            if (nb[d] < 0 || nb[d] >= side) continue;
            const uint64_t a = morton((uint32_t)(nb[0] >> 2), (uint32_t)(nb[1] >> 2), (uint32_t)(nb[2] >> 2));
            if (!sorted_has(inner[l - 2], a)) {
              bad[t] = c;
              return;
            }
          }
      }
    });
  }
  for (auto &x : th) x.join();
  for (int t = 0; t < nt; ++t)
    if (bad[t] >= 0) {
      snprintf(buf, sizeof buf, "not 2:1 graded: leaf %lld has a face neighbour two or more levels coarser",
               (long long)bad[t]);
      msg = buf;
      return RMC_EMESH;
    }
  return RMC_OK;
}

rmc_status enter(rmc_ctx *c) {
  if (!c) return RMC_EINVAL;
  c->err.clear();
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return fail(c, RMC_EDEVICE, "hipSetDevice: %s", hipGetErrorString(e));
  return RMC_OK;
}

rmc_status upload(rmc_ctx *c, DevBuf &dst, const void *src, size_t bytes, int mem) {
  HIPCHK(c, dst.ensure(bytes));
  if (bytes == 0) return RMC_OK;
  HIPCHK(c, hipMemcpyAsync(dst.p, src, bytes, mem == RMC_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                           c->stream));
  return RMC_OK;
}

rmc_status download(rmc_ctx *c, void *dst, const void *src, size_t bytes, int mem) {
  if (!dst || bytes == 0) return RMC_OK;
  HIPCHK(c, hipMemcpyAsync(dst, src, bytes, mem == RMC_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                           c->stream));
  return RMC_OK;
}

// Per-leaf records relative to T_ref (see rmc_device.h), built on the
// device from the raw gas, the leaves' levels and coordinates, the lines
// and the domain.
rmc_status build_leaves(rmc_ctx *c) {
  const LineQ q0 = line_q(c->lines[0], c->T_ref);
  const int64_t n = c->n_leaves;
  const bool f32 = c->precision == RMC_FP32_BULK;
  HIPCHK(c, c->leaves.ensure((size_t)n * LEAF_STRIDE * (f32 ? 4 : 8)));
  HIPCHK(c, launch_leaf_records(f32, n, c->g_raw.as<double>(), c->m_lv.as<int8_t>(), c->m_ijk.as<int32_t>(),
                                c->T_ref, q0.vth, c->box_cm, c->domain, c->dom, c->leaves.p, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->leaves_dirty = false;
  return RMC_OK;
}

void make_problem(rmc_ctx *c, int64_t first, int64_t n, uint64_t seed, ProblemK &pb) {
  std::memset(&pb, 0, sizeof pb);
  pb.nodes = c->nodes.as<int32_t>();
  pb.leaves = c->leaves.p;
  pb.L = c->L;
  pb.top = c->top_level > 0 ? c->top.as<int32_t>() : nullptr;
  pb.top_level = c->top_level;
  pb.n_lines = c->n_lines;
  const LineQ q0 = line_q(c->lines[0], c->T_ref);
  pb.b_ref = q0.vth / C_LIGHT;
  for (int i = 0; i < c->n_lines; ++i) {
    const rmc_line &ln = c->lines[i];
    const LineQ q = line_q(ln, c->T_ref);
    LineK &k = pb.lines[i];
    k.s = ln.lambda0_A / c->lines[0].lambda0_A;                    // nu_ref / nu_i
    k.delta = ((ln.lambda0_A - c->lines[0].lambda0_A) / c->lines[0].lambda0_A) / pb.b_ref;
    k.inv_s = c->lines[0].lambda0_A / ln.lambda0_A;
    k.mu = std::sqrt(c->lines[0].mass_amu / ln.mass_amu);
    k.inv_mu = std::sqrt(ln.mass_amu / c->lines[0].mass_amu);
    k.alpha = q.a;
    k.lalpha = std::log10(q.a);
    k.ibmu = 1.0 / (pb.b_ref * k.mu);
    k.kfac = ln.abundance * q.sigma0;
    k.rec = H_PLANCK * q.nu0 / (ln.mass_amu * AMU_G * C_LIGHT * C_LIGHT);
    k.phase = ln.phase;
    k.recoil = ln.recoil;
    k.n_fluor = ln.n_fluor;
    k.a_res = k.a_cum0 = 1.0;
    for (int j = 0; j < 2; ++j) k.xf0[j] = k.sf[j] = 0.0;
    if (ln.n_fluor > 0) {
      const double a_tot = ln.A_ul + ln.fluor_A_ul[0] + (ln.n_fluor > 1 ? ln.fluor_A_ul[1] : 0.0);
      k.a_res = ln.A_ul / a_tot;
      k.a_cum0 = (ln.A_ul + ln.fluor_A_ul[0]) / a_tot;
      for (int j = 0; j < ln.n_fluor; ++j) {
        const double lf = ln.fluor_lambda_A[j], l0 = c->lines[0].lambda0_A;
        k.xf0[j] = (l0 - lf) / (lf * pb.b_ref);
        k.sf[j] = l0 / lf;
      }
    }
    k.f.delta = (float)k.delta;
    k.f.s = (float)k.s;
    k.f.inv_s = (float)k.inv_s;
    k.f.inv_mu = (float)k.inv_mu;
    k.f.mu = (float)k.mu;
    k.f.alpha = (float)k.alpha;
    k.f.kfac = (float)k.kfac;
    k.f.ibmu = (float)k.ibmu;
    k.f.rec = (float)k.rec;
    k.f.a_res = (float)k.a_res;
    k.f.a_cum0 = (float)k.a_cum0;
    for (int j = 0; j < 2; ++j) {
      k.f.xf0[j] = (float)k.xf0[j];
      k.f.sf[j] = (float)k.sf[j];
    }
  }
  pb.b_ref_f = (float)pb.b_ref;
  pb.box_cm = c->box_cm;
  pb.domain = c->domain;
  for (int d = 0; d < 4; ++d) pb.dom[d] = c->dom[d];
  pb.albedo = c->albedo;
  pb.g_hg = c->g_hg;
  pb.albedo_f = (float)pb.albedo;
  pb.g_hg_f = (float)pb.g_hg;
  pb.forward_only = c->forward_only;
  pb.max_events = c->max_events;
  pb.skip_tau = c->skip_tau;
  pb.skip_frac = c->skip_frac;
  pb.voigt_exact = c->voigt_exact;
  pb.spec_kind = c->spec_kind;
  for (int q = 0; q < 3; ++q) pb.spec_p[q] = c->spec_p[q];
  pb.lambda_ref = c->lines[0].lambda0_A;
  pb.tab_n = c->tab_n;
  pb.tab_lam = c->tab_n ? c->tab.as<double>() : nullptr;
  pb.tab_beta = c->tab_n ? c->tab.as<double>() + c->tab_n : nullptr;
  pb.tab_cum = c->tab_n ? c->tab.as<double>() + 2 * c->tab_n - 1 : nullptr;
  pb.src_pos = c->spos.as<double>();
  pb.src_dir = c->src_dir ? c->sdir.as<double>() : nullptr;
  pb.src_x = c->sx.as<double>();
  pb.first = first;
  pb.n = n;
  pb.seed = seed;
  pb.status = c->o_status.as<int32_t>();
  pb.nscat = c->o_nscat.as<int32_t>();
  pb.x_out = c->o_x.as<double>();
  pb.k_out = c->o_k.as<double>();
  pb.pos_out = c->o_pos.as<double>();
  pb.path_out = c->o_path.as<double>();
  pb.n_obs = (int)c->obs.size();
  for (int o = 0; o < pb.n_obs; ++o) pb.obs[o] = c->obs[o].k;
  pb.stats = c->d_stats.as<unsigned long long>();
}

// The emitted x of packets [first, first+n) under the source spectrum,
// computed on stream st before the transport; pb.src_x then points at them.
// Monochromatic sources: nothing to do.
rmc_status apply_spectrum(rmc_ctx *c, ProblemK &pb, int64_t first, int64_t n, hipStream_t st) {
  if (!c->spec_kind || n <= 0) return RMC_OK;
  HIPCHK(c, c->sx_eff.ensure(sizeof(double) * (size_t)c->n_src));
  HIPCHK(c, launch_source_x(c->precision == RMC_FP32_BULK, pb, c->sx.as<double>(), c->sx_eff.as<double>(), first,
                            n, st));
  pb.src_x = c->sx_eff.as<double>();
  return RMC_OK;
}

rmc_status ready(rmc_ctx *c, bool need_sources) {
  if (!c->has_mesh) return fail(c, RMC_ESTATE, "no mesh (rmc_set_mesh)");
  if (!c->has_lines) return fail(c, RMC_ESTATE, "no lines (rmc_set_lines)");
  if (!c->has_gas) return fail(c, RMC_ESTATE, "no gas (rmc_set_gas)");
  if (c->leaves_dirty) {
    rmc_status r = build_leaves(c);
    if (r) return r;
  }
  if (need_sources && c->n_src <= 0) return fail(c, RMC_ESTATE, "no sources (rmc_set_sources)");
  if (c->domain == RMC_DOM_SLAB_Z)
    for (auto &o : c->obs)
      if (o.k.k[2] == 0.0) return fail(c, RMC_EINVAL, "slab domain: observers need k_z != 0");
  return RMC_OK;
}

// Output arrays for n packets; their statuses start at RMC_ST_NONE (set on
// stream st, the one the transport runs on), so packets not finished yet
// read as such.
rmc_status ensure_outputs(rmc_ctx *c, int64_t n, hipStream_t st) {
  const size_t m = (size_t)std::max<int64_t>(n, 1);
  HIPCHK(c, c->o_status.ensure(m * 4));
  HIPCHK(c, c->o_nscat.ensure(m * 4));
  HIPCHK(c, c->o_x.ensure(m * 8));
  HIPCHK(c, c->o_k.ensure(m * 24));
  HIPCHK(c, c->o_pos.ensure(m * 24));
  HIPCHK(c, c->o_path.ensure(m * 8));
  HIPCHK(c, c->d_stats.ensure(N_STATS * 8));
  HIPCHK(c, c->d_next.ensure(8));
  if (n > 0) HIPCHK(c, hipMemsetAsync(c->o_status.p, 0, (size_t)n * 4, st));
  return RMC_OK;
}

int grid_for(rmc_ctx *c, int64_t n, bool batch, int levels) {
  int64_t g;
  if (c->waves_per_cu > 0) {
    g = (int64_t)c->num_cus * c->waves_per_cu * 64 / c->block;
  } else {
    const int bpc = transport_blocks_per_cu(c->precision == RMC_FP32_BULK, batch, c->s_defer, c->s_one_line,
                                            c->regroup != 0,
                                            c->block,
                                            std::max(levels, 1));
    g = (int64_t)c->num_cus * bpc;
  }
  const int64_t need = (n + c->block - 1) / c->block;
  g = std::min(g, need);
  return (int)std::max<int64_t>(g, 1);
}

void fill_stats(rmc_run_stats *s, const unsigned long long *h, double ms) {
  s->emitted = h[S_EMITTED];
  s->escaped = h[S_ESCAPED];
  s->absorbed = h[S_ABSORBED];
  s->stuck = h[S_STUCK];
  s->scatterings = h[S_SCAT];
  s->dust_scatterings = h[S_DUST_SCAT];
  s->crossings = h[S_CROSS];
  s->peel_rays = h[S_PEEL_RAYS];
  s->peel_crossings = h[S_PEEL_CROSS];
  s->peel_dropped = h[S_PEEL_DROPPED];
  s->peel_deferred = 0;
  s->kernel_ms = ms;
  s->peel_pass_ms = 0.0;
  s->slices_cut = 0;
}

}  // namespace

extern "C" {

int rmc_abi_version(void) { return 9; }

rmc_status rmc_create(rmc_ctx **out, int device, int precision) {
  if (!out) return RMC_EINVAL;
  *out = nullptr;
  if (precision != RMC_FP64 && precision != RMC_FP32_BULK) return RMC_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return RMC_EDEVICE;
  rmc_ctx *c = new (std::nothrow) rmc_ctx();
  if (!c) return RMC_ENOMEM;
  c->device = device;
  c->precision = precision;
  // measured on the dusty sphere: the double kernel gains 2.6% with one
  // rejection round per pass, the float kernel loses 0.9%
  c->regroup = precision == RMC_FP64 ? 1 : 0;
  if (hipSetDevice(device) != hipSuccess ||
      hipDeviceGetAttribute(&c->num_cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
      scratch_address(device, &c->scratch) != hipSuccess ||
      hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess ||
      hipEventCreate(&c->ev2) != hipSuccess) {
    for (hipEvent_t e : {c->ev0, c->ev1, c->ev2})
      if (e) (void)hipEventDestroy(e);
    delete c;
    return RMC_EDEVICE;
  }
  *out = c;
  return RMC_OK;
}

void rmc_destroy(rmc_ctx *c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  if (c->s_graph) (void)hipGraphExecDestroy(c->s_graph);
  if (c->s_graph2) (void)hipGraphExecDestroy(c->s_graph2);
  DevBuf *bufs[] = {&c->nodes, &c->top, &c->leaves, &c->spos, &c->sdir, &c->sx, &c->o_status, &c->o_x, &c->o_k,
                    &c->o_pos, &c->o_nscat, &c->o_path, &c->d_stats, &c->d_next, &c->d_prob, &c->d_starts,
                    &c->tmp1, &c->tmp2, &c->tmp3, &c->tmp4, &c->tmp5, &c->tmp6, &c->b_probs, &c->b_starts,
                    &c->slots, &c->d_slice, &c->pq_ctl, &c->pq_jobs, &c->pq_counts, &c->tp_leaf,
                    &c->tp_seg, &c->tp_next, &c->tp_first, &c->tp_count, &c->tp_pix, &c->tp_wt, &c->tp_x,
                    &c->tp_ctl, &c->sx_eff, &c->tab, &c->g_raw, &c->g_stage, &c->g_in, &c->d_bad,
                    &c->m_lv, &c->m_ijk, &c->slots2, &c->d_live};
  for (DevBuf *b : bufs) b->release();
  for (auto &o : c->obs) o.cube.release();
  if (c->ev0) (void)hipEventDestroy(c->ev0);
  if (c->ev1) (void)hipEventDestroy(c->ev1);
  if (c->ev2) (void)hipEventDestroy(c->ev2);
  delete c;
}

const char *rmc_last_error(const rmc_ctx *c) { return c ? c->err.c_str() : "null context"; }

rmc_status rmc_set_stream(rmc_ctx *c, void *s) {
  rmc_status r = enter(c);
  if (r) return r;
  c->stream = (hipStream_t)s;
  return RMC_OK;
}

rmc_status rmc_set_option(rmc_ctx *c, int opt, int64_t v) {
  rmc_status r = enter(c);
  if (r) return r;
  switch (opt) {
    case RMC_OPT_FORWARD_ONLY: c->forward_only = v ? 1 : 0; break;
    case RMC_OPT_MAX_EVENTS:
      if (v < 0) return fail(c, RMC_EINVAL, "max_events < 0");
      c->max_events = v;
      break;
    case RMC_OPT_BLOCK:
      if (v != 64 && v != 128 && v != 256) return fail(c, RMC_EINVAL, "block must be 64, 128 or 256");
      c->block = (int)v;
      break;
    case RMC_OPT_WAVES_PER_CU:
      if (v < 0 || v > 32) return fail(c, RMC_EINVAL, "waves per CU in [0,32] (0: occupancy limit)");
      c->waves_per_cu = (int)v;
      break;
    case RMC_OPT_REFILL:
      if (v < 1 || v > 64) return fail(c, RMC_EINVAL, "refill in [1,64]");
      c->refill = (int)v;
      break;
    case RMC_OPT_PEEL_DEFER:
      if (v != 0 && v != 1) return fail(c, RMC_EINVAL, "peel defer is 0 or 1");
      c->peel_defer = (int)v;
      break;
    case RMC_OPT_SLICE_ITERS:
      if (v < 1 || v > (1 << 30)) return fail(c, RMC_EINVAL, "slice iterations in [1, 2^30]");
      c->slice_iters = (int)v;
      break;
    case RMC_OPT_REGROUP:
      if (v != 0 && v != 1) return fail(c, RMC_EINVAL, "regroup is 0 or 1");
      c->regroup = (int)v;
      break;
    case RMC_OPT_COMPACT:
      if (v != 0 && v != 1) return fail(c, RMC_EINVAL, "compact is 0 or 1");
      c->compact = (int)v;
      break;
    case RMC_OPT_VOIGT:
      if (v != 0 && v != 1) return fail(c, RMC_EINVAL, "voigt is 0 (Tasitsiomi) or 1 (accurate)");
      if (v == 1 && c->precision != RMC_FP64)
        return fail(c, RMC_EUNSUPPORTED, "the accurate Voigt function is an RMC_FP64 option");
      c->voigt_exact = (int)v;
      break;
    default: return fail(c, RMC_EINVAL, "unknown option %d", opt);
  }
  return RMC_OK;
}

rmc_status rmc_set_source_spectrum(rmc_ctx *c, int kind, const double *params) {
  rmc_status r = enter(c);
  if (r) return r;
  if (kind == RMC_SPEC_MONO) {
    c->spec_kind = 0;
    return RMC_OK;
  }
  if (!params) return fail(c, RMC_EINVAL, "null spectrum parameters");
  if (kind == RMC_SPEC_GAUSS) {
    if (!finite_nonneg(params[0])) return fail(c, RMC_EINVAL, "Gaussian sigma must be finite and >= 0");
  } else if (kind == RMC_SPEC_POWER_LAW) {
    if (!(std::isfinite(params[0]) && std::isfinite(params[1]) && std::isfinite(params[2])) ||
        !(params[0] > 0.0) || !(params[1] > params[0]))
      return fail(c, RMC_EINVAL, "power law needs 0 < lambda_min < lambda_max and a finite beta");
  } else {
    return fail(c, RMC_EINVAL, "unknown spectrum kind %d", kind);
  }
  c->spec_kind = kind;
  for (int q = 0; q < 3; ++q) c->spec_p[q] = kind == RMC_SPEC_GAUSS && q > 0 ? 0.0 : params[q];
  return RMC_OK;
}

rmc_status rmc_set_source_table(rmc_ctx *c, int n, const double *lambda_A, const double *f_lambda) {
  rmc_status r = enter(c);
  if (r) return r;
  if (n < 2 || !lambda_A || !f_lambda) return fail(c, RMC_EINVAL, "a table needs at least 2 points");
  for (int i = 0; i < n; ++i) {
    if (!(lambda_A[i] > 0.0) || !std::isfinite(lambda_A[i]) || !(f_lambda[i] > 0.0) || !std::isfinite(f_lambda[i]))
      return fail(c, RMC_EINVAL, "table point %d: wavelength and F_lambda must be positive and finite", i);
    if (i > 0 && !(lambda_A[i] > lambda_A[i - 1])) return fail(c, RMC_EINVAL, "table wavelengths must increase");
  }
  // per bin: the slope of the power law through its ends and the integral
  // of lambda F_lambda over it (ratio form), accumulated
  std::vector<double> h(3 * (size_t)n - 1);
  double *lam = h.data(), *beta = lam + n, *cum = beta + (n - 1);
  cum[0] = 0.0;
  for (int i = 0; i < n; ++i) lam[i] = lambda_A[i];
  for (int i = 0; i + 1 < n; ++i) {
    const double l0 = lambda_A[i], l1 = lambda_A[i + 1], q = l1 / l0;
    const double b = std::log(f_lambda[i + 1] / f_lambda[i]) / std::log(q);
    beta[i] = b;
    const double cnt = b == -2.0 ? f_lambda[i] * l0 * l0 * std::log(q)
                                 : f_lambda[i] * l0 * l0 * (std::pow(q, b + 2.0) - 1.0) / (b + 2.0);
    if (!std::isfinite(cnt)) return fail(c, RMC_EINVAL, "table bin %d: photon count overflows", i);
    cum[i + 1] = cum[i] + cnt;
  }
  // work already queued on the context's stream may still read the old table
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, c->tab.ensure(h.size() * sizeof(double)));
  HIPCHK(c, hipMemcpyAsync(c->tab.p, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->tab_n = n;
  c->spec_kind = RMC_SPEC_TABLE;
  return RMC_OK;
}

rmc_status rmc_set_core_skip(rmc_ctx *c, double tau_skip, double frac) {
  rmc_status r = enter(c);
  if (r) return r;
  if (!std::isfinite(tau_skip)) return fail(c, RMC_EINVAL, "core-skip tau_skip not finite");
  if (!std::isfinite(frac) || frac < 0) return fail(c, RMC_EINVAL, "core-skip frac must be finite and >= 0");
  c->skip_tau = tau_skip > 0 ? tau_skip : 0.0;
  c->skip_frac = tau_skip > 0 ? frac : 0.0;
  return RMC_OK;
}

// Table of the level-T cells, T = min(L, TOP_LEVEL), from which point
// location starts: each entry is the node at level T above the cell, or the
// leaf (of level <= T) covering it, as -(leaf | level << TOP_LEVEL_SHIFT) - 1.
// None (T = 0) for a single-leaf mesh or when leaf indices do not fit below
// the level bits.
static void build_top(const std::vector<int32_t> &nodes, int L, int64_t n_leaves, std::vector<int32_t> &top, int &T) {
  top.clear();
  T = 0;
  if (L == 0 || n_leaves >= ((int64_t)1 << TOP_LEVEL_SHIFT)) return;
  T = std::min(L, TOP_LEVEL);
  const int side = 1 << T;
  top.assign((size_t)side * side * side, 0);
  for (int k = 0; k < side; ++k)
    for (int j = 0; j < side; ++j)
      for (int i = 0; i < side; ++i) {
        int node = 0, e = 0;
        bool leaf = false;
        for (int lev = 0; lev < T; ++lev) {
          const int sh = T - lev - 1;
          const int oct = ((i >> sh) & 1) | (((j >> sh) & 1) << 1) | (((k >> sh) & 1) << 2);
          const int32_t ch = nodes[(size_t)node * 8 + oct];
          if (ch < 0) {
            e = -((((-ch) - 1) | ((lev + 1) << TOP_LEVEL_SHIFT)) + 1);
            leaf = true;
            break;
          }
          node = ch;
        }
        top[((size_t)k * side + j) * side + i] = leaf ? e : node;
      }
}

rmc_status rmc_set_mesh(rmc_ctx *c, int64_t n, const int8_t *level, const int32_t *ijk, double box_cm) {
  rmc_status r = enter(c);
  if (r) return r;
  if (!(box_cm > 0.0) || !std::isfinite(box_cm)) return fail(c, RMC_EINVAL, "box_cm must be > 0");
  std::vector<int32_t> nodes;
  int L = 0;
  std::string msg;
  r = build_tree(n, level, ijk, nodes, L, msg);
  if (r) return fail(c, r, "%s", msg.c_str());
  HIPCHK(c, c->nodes.ensure(std::max<size_t>(nodes.size() * 4, 32)));
  if (!nodes.empty()) HIPCHK(c, hipMemcpy(c->nodes.p, nodes.data(), nodes.size() * 4, hipMemcpyHostToDevice));
  std::vector<int32_t> top;
  int T = 0;
  build_top(nodes, L, n, top, T);
  if (!top.empty()) {
    HIPCHK(c, c->top.ensure(top.size() * 4));
    HIPCHK(c, hipMemcpy(c->top.p, top.data(), top.size() * 4, hipMemcpyHostToDevice));
  }
  c->top_level = T;
  HIPCHK(c, c->m_lv.ensure((size_t)n));
  HIPCHK(c, c->m_ijk.ensure((size_t)n * 12));
  HIPCHK(c, hipMemcpy(c->m_lv.p, level, (size_t)n, hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(c->m_ijk.p, ijk, (size_t)n * 12, hipMemcpyHostToDevice));
  c->n_leaves = n;
  c->n_nodes = (int64_t)nodes.size() / 8;
  c->L = L;
  c->box_cm = box_cm;
  c->has_mesh = true;
  c->has_gas = false;
  ++c->gen;
  return RMC_OK;
}

rmc_status rmc_set_lines(rmc_ctx *c, int n, const rmc_line *lines, double T_ref) {
  rmc_status r = enter(c);
  if (r) return r;
  if (n < 1 || n > MAX_LINES || !lines) return fail(c, RMC_EINVAL, "1..%d lines", MAX_LINES);
  if (!(T_ref > 0.0) || !std::isfinite(T_ref)) return fail(c, RMC_EINVAL, "T_ref must be > 0");
  for (int i = 0; i < n; ++i) {
    const rmc_line &l = lines[i];
    if (!(l.lambda0_A > 0) || !(l.A_ul > 0) || !(l.f_lu >= 0) || !(l.mass_amu > 0) || !finite_nonneg(l.abundance) ||
        (l.phase != RMC_PHASE_LYA_DIPOLE && l.phase != RMC_PHASE_ISOTROPIC))
      return fail(c, RMC_EINVAL, "line %d: bad parameters", i);
    if (l.n_fluor < 0 || l.n_fluor > 2) return fail(c, RMC_EINVAL, "line %d: 0..2 fluorescent channels", i);
    for (int j = 0; j < l.n_fluor; ++j)
      if (!(l.fluor_lambda_A[j] > 0) || !std::isfinite(l.fluor_lambda_A[j]) || !(l.fluor_A_ul[j] > 0) ||
          !std::isfinite(l.fluor_A_ul[j]))
        return fail(c, RMC_EINVAL, "line %d: bad fluorescent channel %d", i, j);
    c->lines[i] = l;
  }
  c->n_lines = n;
  c->T_ref = T_ref;
  c->has_lines = true;
  ++c->gen;
  if (c->has_gas) return build_leaves(c);
  return RMC_OK;
}

rmc_status rmc_set_gas(rmc_ctx *c, const void *n_hi, const void *T, const void *v, const void *kd, int dtype,
                       int mem) {
  rmc_status r = enter(c);
  if (r) return r;
  if (!c->has_mesh) return fail(c, RMC_ESTATE, "rmc_set_mesh first");
  if (!c->has_lines) return fail(c, RMC_ESTATE, "rmc_set_lines first");
  if (!n_hi || !T || !v || !kd) return fail(c, RMC_EINVAL, "null gas array");
  if (dtype != RMC_F32 && dtype != RMC_F64) return fail(c, RMC_EINVAL, "dtype must be RMC_F32 or RMC_F64");
  if (mem != RMC_HOST && mem != RMC_DEVICE) return fail(c, RMC_EINVAL, "mem must be RMC_HOST or RMC_DEVICE");
  const int64_t n = c->n_leaves;
  const size_t esz = dtype == RMC_F32 ? 4 : 8;
  const void *src[4] = {n_hi, T, v, kd};
  if (mem == RMC_HOST) {
    // one staging allocation for the four host arrays (6 values per leaf)
    HIPCHK(c, c->g_in.ensure((size_t)n * 6 * esz));
    const size_t off[4] = {0, (size_t)n, (size_t)2 * n, (size_t)5 * n};
    const size_t cnt[4] = {(size_t)n, (size_t)n, (size_t)3 * n, (size_t)n};
    for (int j = 0; j < 4; ++j) {
      void *dst = (char *)c->g_in.p + off[j] * esz;
      HIPCHK(c, hipMemcpyAsync(dst, src[j], cnt[j] * esz, hipMemcpyHostToDevice, c->stream));
      src[j] = dst;
    }
  }
  HIPCHK(c, c->g_stage.ensure((size_t)n * 64));
  HIPCHK(c, c->d_bad.ensure(16));
  HIPCHK(c, launch_fill_u64(c->d_bad.as<unsigned long long>(), 2, ~0ull, c->stream));
  HIPCHK(c, launch_stage_gas(dtype == RMC_F32, n, src[0], src[1], src[2], src[3], c->g_stage.as<double>(),
                             c->d_bad.as<unsigned long long>(), c->stream));
  unsigned long long bad[2] = {0, 0};
  HIPCHK(c, hipMemcpyAsync(bad, c->d_bad.p, sizeof bad, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (mem == RMC_HOST) c->g_in.release();
  if (bad[0] != ~0ull) return fail(c, RMC_EINVAL, "leaf %llu: non-finite or negative gas value", bad[0]);
  if (bad[1] != ~0ull) return fail(c, RMC_EINVAL, "leaf %llu: |v| >= 0.1 c", bad[1]);
  std::swap(c->g_raw, c->g_stage);
  r = build_leaves(c);
  if (r) return r;
  c->has_gas = true;
  ++c->gen;
  return RMC_OK;
}

rmc_status rmc_set_dust(rmc_ctx *c, double albedo, double g) {
  rmc_status r = enter(c);
  if (r) return r;
  if (!(albedo >= 0.0 && albedo <= 1.0) || !(g > -1.0 && g < 1.0)) return fail(c, RMC_EINVAL, "albedo in [0,1], |g| < 1");
  c->albedo = albedo;
  c->g_hg = g;
  return RMC_OK;
}

rmc_status rmc_set_domain(rmc_ctx *c, int kind, const double p[4]) {
  rmc_status r = enter(c);
  if (r) return r;
  double q[4] = {0, 0, 0, 0};
  if (kind != RMC_DOM_BOX) {
    if (!p) return fail(c, RMC_EINVAL, "domain parameters needed");
    for (int d = 0; d < 4; ++d) q[d] = p[d];
  }
  if (kind == RMC_DOM_SLAB_Z) {
    if (!(q[1] > 0) || q[0] - q[1] < 0.0 || q[0] + q[1] > 1.0) return fail(c, RMC_EINVAL, "slab must lie in [0,1]");
  } else if (kind == RMC_DOM_SPHERE) {
    if (!(q[3] > 0) || q[0] - q[3] < 0 || q[0] + q[3] > 1 || q[1] - q[3] < 0 || q[1] + q[3] > 1 || q[2] - q[3] < 0 ||
        q[2] + q[3] > 1)
      return fail(c, RMC_EINVAL, "sphere must lie inside the unit cube");
  } else if (kind != RMC_DOM_BOX) {
    return fail(c, RMC_EINVAL, "unknown domain kind %d", kind);
  }
  c->domain = kind;
  for (int d = 0; d < 4; ++d) c->dom[d] = q[d];
  if (c->has_gas) c->leaves_dirty = true;
  ++c->gen;
  return RMC_OK;
}

rmc_status rmc_set_sources(rmc_ctx *c, int64_t n, const double *pos, const double *dir, const double *x, int mem) {
  rmc_status r = enter(c);
  if (r) return r;
  if (n <= 0 || !pos || !x) return fail(c, RMC_EINVAL, "need n > 0, positions and frequencies");
  if (mem == RMC_HOST) {
    for (int64_t i = 0; i < n; ++i) {
      for (int d = 0; d < 3; ++d)
        if (!(pos[3 * i + d] >= 0.0 && pos[3 * i + d] <= 1.0)) return fail(c, RMC_EINVAL, "source %lld outside the box", (long long)i);
      if (!std::isfinite(x[i])) return fail(c, RMC_EINVAL, "source %lld: non-finite x", (long long)i);
      if (dir) {
        const double nn = dir[3 * i] * dir[3 * i] + dir[3 * i + 1] * dir[3 * i + 1] + dir[3 * i + 2] * dir[3 * i + 2];
        if (!(std::fabs(nn - 1.0) < 1e-6)) return fail(c, RMC_EINVAL, "source %lld: direction not unit", (long long)i);
      }
    }
  }
  if (mem == RMC_DEVICE) {
    HIPCHK(c, c->d_bad.ensure(16));
    HIPCHK(c, launch_fill_u64(c->d_bad.as<unsigned long long>(), 1, ~0ull, c->stream));
    HIPCHK(c, launch_check_sources(n, pos, dir, x, c->d_bad.as<unsigned long long>(), c->stream));
    unsigned long long bad = 0;
    HIPCHK(c, hipMemcpyAsync(&bad, c->d_bad.p, 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (bad != ~0ull)
      return fail(c, RMC_EINVAL, "source %llu outside the box, with non-finite x or a non-unit direction", bad);
  } else if (mem != RMC_HOST) {
    return fail(c, RMC_EINVAL, "mem must be RMC_HOST or RMC_DEVICE");
  }
  r = upload(c, c->spos, pos, (size_t)n * 24, mem);
  if (r) return r;
  r = upload(c, c->sx, x, (size_t)n * 8, mem);
  if (r) return r;
  c->src_dir = dir != nullptr;
  if (dir) {
    r = upload(c, c->sdir, dir, (size_t)n * 24, mem);
    if (r) return r;
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->n_src = n;
  return RMC_OK;
}

rmc_status rmc_add_observer(rmc_ctx *c, const double k[3], int nx, int ny, int nbins, const double fov[4], double x_min,
                            double x_max, int *id) {
  rmc_status r = enter(c);
  if (r) return r;
  if ((int)c->obs.size() >= MAX_OBS) return fail(c, RMC_EUNSUPPORTED, "at most %d observers", MAX_OBS);
  if (!k || !fov || nx <= 0 || ny <= 0 || nbins <= 0 || !(x_max > x_min) || !(fov[1] > fov[0]) || !(fov[3] > fov[2]))
    return fail(c, RMC_EINVAL, "bad observer");
  const double nn = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
  if (!(std::fabs(nn - 1.0) < 1e-12)) return fail(c, RMC_EINVAL, "observer direction must be a unit vector");
  ObsHost o;
  std::memset(&o.k, 0, sizeof o.k);
  for (int d = 0; d < 3; ++d) o.k.k[d] = k[d];
  // image basis: e1 = normalize(z x k) (x when k is along z), e2 = k x e1
  double e1[3];
  if (k[0] == 0.0 && k[1] == 0.0) {
    e1[0] = 1.0; e1[1] = 0.0; e1[2] = 0.0;
  } else {
    const double nrm = std::sqrt(k[1] * k[1] + k[0] * k[0]);
    e1[0] = -k[1] / nrm; e1[1] = k[0] / nrm; e1[2] = 0.0;
  }
  const double e2[3] = {k[1] * e1[2] - k[2] * e1[1], k[2] * e1[0] - k[0] * e1[2], k[0] * e1[1] - k[1] * e1[0]};
  for (int d = 0; d < 3; ++d) {
    o.k.e1[d] = e1[d];
    o.k.e2[d] = e2[d];
  }
  o.k.u0 = fov[0];
  o.k.uspan = fov[1] - fov[0];
  o.k.v0 = fov[2];
  o.k.vspan = fov[3] - fov[2];
  o.k.x_min = x_min;
  o.k.xspan = x_max - x_min;
  o.k.nx = nx;
  o.k.ny = ny;
  o.k.nbins = nbins;
  for (int d = 0; d < 3; ++d) o.k.kinv[d] = k[d] != 0.0 ? 1.0 / k[d] : 0.0;
  for (int d = 0; d < 3; ++d) o.k.kf[d] = (float)o.k.k[d];
  o.k.su = nx / o.k.uspan;
  o.k.sv = ny / o.k.vspan;
  o.k.sx = nbins / o.k.xspan;
  o.n_elems = (size_t)nx * ny * nbins;
  const size_t esz = c->precision == RMC_FP32_BULK ? 4 : 8;
  HIPCHK(c, o.cube.ensure(o.n_elems * esz));
  HIPCHK(c, hipMemsetAsync(o.cube.p, 0, o.n_elems * esz, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  o.k.cube = o.cube.p;
  c->obs.push_back(o);
  if (id) *id = (int)c->obs.size() - 1;
  return RMC_OK;
}

rmc_status rmc_reset_cubes(rmc_ctx *c) {
  rmc_status r = enter(c);
  if (r) return r;
  const size_t esz = c->precision == RMC_FP32_BULK ? 4 : 8;
  for (auto &o : c->obs) HIPCHK(c, hipMemsetAsync(o.cube.p, 0, o.n_elems * esz, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return RMC_OK;
}

// ------------------------------------------------------------ streaming
namespace {

void add_run_stats(rmc_run_stats &a, const rmc_run_stats &b) {
  a.emitted += b.emitted; a.escaped += b.escaped; a.absorbed += b.absorbed; a.stuck += b.stuck;
  a.scatterings += b.scatterings; a.dust_scatterings += b.dust_scatterings; a.crossings += b.crossings;
  a.peel_rays += b.peel_rays; a.peel_crossings += b.peel_crossings; a.peel_dropped += b.peel_dropped;
  a.peel_deferred += b.peel_deferred;
  a.slices_cut += b.slices_cut;
  a.peel_pass_ms += b.peel_pass_ms;
  a.kernel_ms += b.kernel_ms;
}

constexpr unsigned long long PQ_FIRST_CAP = 1024;          // jobs per region (one region per wave)
constexpr unsigned long long PQ_MAX_BYTES = 32ull << 30;    // job buffer limit
static_assert(PQ_FIRST_CAP > 2 * 64 * MAX_OBS, "a region must hold one wave iteration of pushes");

// Control block of the deferred peel-off queue, or null when peel-off rays
// are walked inline (option off).  Its regions are laid out per transport
// wave by stream_open.
rmc_status peel_queue(rmc_ctx *c, PeelQueue **out) {
  *out = nullptr;
  if (!c->peel_defer) return RMC_OK;
  HIPCHK(c, c->pq_ctl.ensure(peel_queue_bytes()));
  if (!c->pq_cap) {
    // first guess: a sixteenth of a wave's peel-off rays in one launch
    const unsigned long long rays = 64ull * (unsigned long long)c->slice_iters * std::max<size_t>(c->obs.size(), 1);
    c->pq_cap = PQ_FIRST_CAP;
    while (c->pq_cap < rays / 16 && c->pq_cap < (1ull << 16)) c->pq_cap <<= 1;
  }
  *out = c->pq_ctl.as<PeelQueue>();
  return RMC_OK;
}

// Lay out n_regions regions of c->pq_cap jobs and upload the control
// block (totals zero).
rmc_status layout_queue(rmc_ctx *c, unsigned long long n_regions) {
  // at least PQ_FIRST_CAP, so that a region always has room for a wave
  // iteration's pushes
  const unsigned long long max_cap =
      std::max<unsigned long long>(PQ_MAX_BYTES / peel_job_bytes(c->precision == RMC_FP32_BULK) / n_regions, PQ_FIRST_CAP);
  c->pq_cap = std::min(c->pq_cap, max_cap);
  HIPCHK(c, c->pq_counts.ensure(n_regions * 4));
  HIPCHK(c, c->pq_jobs.ensure(n_regions * c->pq_cap * peel_job_bytes(c->precision == RMC_FP32_BULK)));
  PeelQueue q;
  q.jobs = c->pq_jobs.p;
  q.counts = c->pq_counts.as<uint32_t>();
  q.cap = c->pq_cap;
  q.n_regions = n_regions;
  q.pushes = 0;
  q.max_region = 0;
  q.take = 0;
  q.lost = 0;
  HIPCHK(c, hipMemcpyAsync(c->pq_ctl.p, &q, sizeof q, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->pq_regions = n_regions;
  return RMC_OK;
}

// Whether a wave may have ended its slice early for room: its region held
// more than the capacity less one wave iteration's pushes.
bool slice_cut(const rmc_ctx *c, unsigned long long max_region) {
  const unsigned long long per_iter = 2ull * 64 * MAX_OBS;   // pushes one wave iteration can make
  return max_region + per_iter > c->pq_cap;
}

// After a launch in which a wave ended its slice early because its region
// was nearly full, enlarge the regions eightfold (up to PQ_MAX_BYTES) for
// the next launches.
rmc_status grow_queue(rmc_ctx *c, unsigned long long max_region) {
  if (!slice_cut(c, max_region)) return RMC_OK;
  const unsigned long long max_cap =
      std::max<unsigned long long>(PQ_MAX_BYTES / peel_job_bytes(c->precision == RMC_FP32_BULK) / c->pq_regions, PQ_FIRST_CAP);
  if (c->pq_cap >= max_cap) return RMC_OK;
  const unsigned long long cap = c->pq_cap * 8;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const unsigned long long old = c->pq_cap;
  c->pq_cap = std::min(cap, max_cap);
  if (c->pq_jobs.ensure(c->pq_regions * c->pq_cap * peel_job_bytes(c->precision == RMC_FP32_BULK)) != hipSuccess) {
    (void)hipGetLastError();
    c->pq_cap = old;    // keep the old size (waves go on ending slices early)
  }
  return layout_queue(c, c->pq_regions);
}

// Prepare slots and counters for a stream over the problems already
// uploaded at s_probs / s_starts.
rmc_status stream_open(rmc_ctx *c, int64_t total, int n_probs, int levels, bool batch) {
  c->image_done = false;
  c->s_total = total;
  c->s_done = 0;
  c->s_nprobs = n_probs;
  c->s_levels = std::max(levels, 1);
  c->s_batch = batch;
  c->s_grid = grid_for(c, total, batch, levels);
  c->s_tail_grid = 0;
  const int64_t n_slots = (int64_t)c->s_grid * c->block;
  HIPCHK(c, c->slots.ensure((size_t)n_slots * slot_bytes()));
  HIPCHK(c, c->d_slice.ensure((N_STATS + 3) * 8));
  HIPCHK(c, c->d_next.ensure(8));
  HIPCHK(c, launch_clear_slots(c->slots.p, n_slots, c->stream));
  if (c->s_pq) {
    rmc_status r = layout_queue(c, (unsigned long long)n_slots / 64);
    if (r) return r;
  }
  HIPCHK(c, launch_batch_reset(c->s_probs, n_probs, c->d_next.as<unsigned long long>(), c->stream));
  std::memset(&c->s_acc, 0, sizeof c->s_acc);
  c->s_open = true;
  // one slice = zero the slice counters, one transport launch; captured
  // once per shape and replayed
  char key[256];
  PeelQueue *pq = c->s_pq;
  snprintf(key, sizeof key, "%p/%p/%p/%p/%p/%d/%d/%d/%d/%d/%d/%d/%d/%d", (void *)c->s_probs, (void *)c->s_starts,
           c->slots.p, c->d_slice.p, (void *)pq, n_probs, c->s_grid, c->block, c->refill, c->s_levels,
           c->precision, c->slice_iters, (int)batch,
           (int)c->regroup * 4 + (int)c->s_one_line * 2 + (int)c->s_defer);
  if (c->s_key != key || !c->s_graph) {
    for (hipGraphExec_t *ge : {&c->s_graph, &c->s_graph2})
      if (*ge) {
        (void)hipGraphExecDestroy(*ge);
        *ge = nullptr;
      }
    const bool f32 = c->precision == RMC_FP32_BULK;
    hipStream_t cap = nullptr;
    HIPCHK(c, hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    hipError_t e = hipSuccess;
    for (int part = 0; part < (pq ? 2 : 1) && e == hipSuccess; ++part) {
      hipGraph_t g = nullptr;
      e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
      if (part == 0) {
        if (e == hipSuccess) e = launch_fill_u64(c->d_slice.as<unsigned long long>(), N_STATS + 3, 0ull, cap);
        if (e == hipSuccess)
          e = launch_transport(f32, batch, c->s_defer, c->s_one_line, c->regroup != 0, c->s_probs, c->s_starts,
                               n_probs,
                               c->d_next.as<unsigned long long>(), c->refill, c->s_levels, c->s_grid, c->block,
                               c->slots.p, c->slice_iters, c->d_slice.as<unsigned long long>(), cap);
      } else {
        const int grid = c->num_cus * peel_drain_blocks_per_cu(f32, batch, c->s_one_line, c->s_levels);
        if (e == hipSuccess)
          e = launch_peel_drain(f32, batch, c->s_one_line, c->s_probs, pq, c->s_levels, grid,
                                c->d_slice.as<unsigned long long>(),
                                cap);
      }
      hipError_t e2 = hipStreamEndCapture(cap, &g);
      if (e == hipSuccess) e = e2;
      if (e == hipSuccess) e = hipGraphInstantiate(part == 0 ? &c->s_graph : &c->s_graph2, g, nullptr, nullptr, 0);
      if (g) (void)hipGraphDestroy(g);
    }
    (void)hipStreamDestroy(cap);
    if (e != hipSuccess) {
      c->s_open = false;
      return fail(c, RMC_EDEVICE, "graph capture: %s", hipGetErrorString(e));
    }
    c->s_key = key;
  }
  return RMC_OK;
}

// Once every packet of the stream has started (the queue is drained), the
// live packets are total - done, all parked in slots.  When they fill at
// most three quarters of the lanes launched, gather them to the front
// (through slots2) and run the next launches with the blocks they fill:
// the last, longest walks then share the SIMDs with fewer waves, and each
// wave issues its instructions faster.  Which lane runs a packet does not
// change its walk, so results are those of the full grid (cube additions
// aside, whose order differs).
rmc_status gather_tail(rmc_ctx *c) {
  const int64_t live = c->s_total - c->s_done;
  const int grid = c->s_tail_grid > 0 ? c->s_tail_grid : c->s_grid;
  const int64_t lanes = (int64_t)grid * c->block;
  if (live > lanes * 3 / 4) return RMC_OK;
  const int new_grid = (int)((live + c->block - 1) / c->block);
  const int64_t n_new = (int64_t)new_grid * c->block;
  HIPCHK(c, c->slots2.ensure((size_t)n_new * slot_bytes()));
  HIPCHK(c, c->d_live.ensure(8));
  HIPCHK(c, launch_clear_slots(c->slots2.p, n_new, c->stream));
  HIPCHK(c, launch_fill_u64(c->d_live.as<unsigned long long>(), 1, 0ull, c->stream));
  HIPCHK(c, launch_compact_slots(c->slots.p, lanes, c->slots2.p, c->d_live.as<unsigned long long>(), c->stream));
  HIPCHK(c, hipMemcpyAsync(c->slots.p, c->slots2.p, (size_t)n_new * slot_bytes(), hipMemcpyDeviceToDevice,
                           c->stream));
  unsigned long long got = 0;
  HIPCHK(c, hipMemcpyAsync(&got, c->d_live.p, 8, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if ((int64_t)got != live) {
    c->s_open = false;
    return fail(c, RMC_EDEVICE, "gathering the last packets: %llu parked, %lld expected", got, (long long)live);
  }
  c->s_tail_grid = new_grid;
  return RMC_OK;
}

rmc_status stream_step(rmc_ctx *c, rmc_run_stats *slice, int64_t *remaining) {
  if (!c->s_open) return fail(c, RMC_ESTATE, "no open stream (rmc_stream_begin)");
  rmc_run_stats z;
  std::memset(&z, 0, sizeof z);
  if (c->s_done >= c->s_total) {
    if (slice) *slice = z;
    if (remaining) *remaining = 0;
    return RMC_OK;
  }
  HIPCHK(c, hipEventRecord(c->ev0, c->stream));
  if (c->s_tail_grid > 0) {
    // the captured launches with the grid of the gathered slots
    const bool f32 = c->precision == RMC_FP32_BULK;
    HIPCHK(c, launch_fill_u64(c->d_slice.as<unsigned long long>(), N_STATS + 3, 0ull, c->stream));
    // regions of waves not launched must read empty in the pass
    if (c->s_pq) HIPCHK(c, launch_fill_u32(c->pq_counts.as<uint32_t>(), (int64_t)c->pq_regions, 0u, c->stream));
    // at most one wave per SIMD: the kernel compiled for one (no spills)
    const bool lone = (int64_t)c->s_tail_grid * (c->block / 64) <= (int64_t)c->num_cus * 4;
    HIPCHK(c, launch_transport(f32, c->s_batch, c->s_defer, c->s_one_line, c->regroup != 0, c->s_probs,
                               c->s_starts, c->s_nprobs, c->d_next.as<unsigned long long>(), c->refill,
                               c->s_levels, c->s_tail_grid, c->block, c->slots.p, c->slice_iters,
                               c->d_slice.as<unsigned long long>(), c->stream, lone));
    HIPCHK(c, hipEventRecord(c->ev1, c->stream));
    if (c->s_pq) {
      const int grid = c->num_cus * peel_drain_blocks_per_cu(f32, c->s_batch, c->s_one_line, c->s_levels);
      HIPCHK(c, launch_peel_drain(f32, c->s_batch, c->s_one_line, c->s_probs, c->s_pq, c->s_levels, grid,
                                  c->d_slice.as<unsigned long long>(), c->stream));
    }
  } else {
    HIPCHK(c, hipGraphLaunch(c->s_graph, c->stream));
    HIPCHK(c, hipEventRecord(c->ev1, c->stream));
    if (c->s_pq) HIPCHK(c, hipGraphLaunch(c->s_graph2, c->stream));
  }
  HIPCHK(c, hipEventRecord(c->ev2, c->stream));
  unsigned long long h[N_STATS + 3], next = 0;
  HIPCHK(c, hipMemcpyAsync(h, c->d_slice.p, sizeof h, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(&next, c->d_next.p, 8, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  float ms = 0.f, ms2 = 0.f;
  HIPCHK(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
  HIPCHK(c, hipEventElapsedTime(&ms2, c->ev1, c->ev2));
  fill_stats(&z, h, ms);
  z.peel_deferred = h[N_STATS];
  z.peel_pass_ms = c->s_pq ? ms2 : 0.0;
  if (c->s_pq) {
    if (h[N_STATS + 2]) {
      c->s_open = false;
      return fail(c, RMC_EDEVICE, "peel-off queue: %llu rays found their region full", h[N_STATS + 2]);
    }
    z.slices_cut = slice_cut(c, h[N_STATS + 1]) ? 1 : 0;
    rmc_status r = grow_queue(c, h[N_STATS + 1]);
    if (r) return r;
  }
  c->s_done += (int64_t)h[S_EMITTED];
  add_run_stats(c->s_acc, z);
  if (slice) *slice = z;
  if (remaining) *remaining = c->s_total - c->s_done;
  if (c->compact && (int64_t)next >= c->s_total && c->s_done < c->s_total) {
    rmc_status r = gather_tail(c);
    if (r) return r;
  }
  return RMC_OK;
}

rmc_status stream_begin_single(rmc_ctx *c, uint64_t seed, int64_t first, int64_t n) {
  rmc_status r = ready(c, true);
  if (r) return r;
  if (first < 0 || n < 0 || first + n > c->n_src) return fail(c, RMC_EINVAL, "packet range outside the sources");
  r = ensure_outputs(c, n, c->stream);
  if (r) return r;
  c->last_n = n;
  make_problem(c, first, n, seed, c->pb_host);
  r = apply_spectrum(c, c->pb_host, first, n, c->stream);
  if (r) return r;
  r = peel_queue(c, &c->s_pq);
  if (r) return r;
  if (c->obs.empty()) c->s_pq = nullptr;
  c->s_defer = c->s_pq != nullptr || c->obs.empty();
  c->pb_host.pq = c->s_pq;
  c->pb_host.index = 0;
  c->s_one_line = c->n_lines == 1 && c->lines[0].n_fluor == 0;
  c->starts_host[0] = 0;
  c->starts_host[1] = n;
  HIPCHK(c, c->d_prob.ensure(sizeof(ProblemK)));
  HIPCHK(c, c->d_starts.ensure(16));
  HIPCHK(c, hipMemcpyAsync(c->d_prob.p, &c->pb_host, sizeof(ProblemK), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->d_starts.p, c->starts_host, 16, hipMemcpyHostToDevice, c->stream));
  c->s_probs = c->d_prob.as<ProblemK>();
  c->s_starts = c->d_starts.as<int64_t>();
  c->s_members.assign(1, c);
  return stream_open(c, n, 1, c->L, false);
}

// Totals of a finished stream: per-problem counters and the summed
// launch times.
rmc_status stream_finish(rmc_ctx *c, rmc_run_stats *per, rmc_run_stats *total) {
  while (c->s_done < c->s_total) {
    rmc_status r = stream_step(c, nullptr, nullptr);
    if (r) return r;
  }
  c->s_open = false;
  const int np = (int)c->s_members.size();
  std::vector<unsigned long long> h((size_t)np * N_STATS);
  for (int i = 0; i < np; ++i)
    HIPCHK(c, hipMemcpyAsync(h.data() + (size_t)i * N_STATS, c->s_members[i]->d_stats.p, N_STATS * 8,
                             hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  unsigned long long t[N_STATS] = {0};
  for (int i = 0; i < np; ++i) {
    if (per) {
      fill_stats(per + i, h.data() + (size_t)i * N_STATS, c->s_acc.kernel_ms);
      per[i].peel_pass_ms = c->s_acc.peel_pass_ms;
    }
    for (int q = 0; q < N_STATS; ++q) t[q] += h[(size_t)i * N_STATS + q];
  }
  if (total) {
    fill_stats(total, t, c->s_acc.kernel_ms);
    total->peel_deferred = c->s_acc.peel_deferred;
    total->peel_pass_ms = c->s_acc.peel_pass_ms;
    total->slices_cut = c->s_acc.slices_cut;
  }
  if ((int64_t)t[S_EMITTED] != c->s_total)
    return fail(c, RMC_EDEVICE, "transport finished %llu of %lld packets", t[S_EMITTED], (long long)c->s_total);
  return RMC_OK;
}

}  // namespace

rmc_status rmc_stream_begin(rmc_ctx *c, uint64_t seed, int64_t first, int64_t n) {
  rmc_status r = enter(c);
  if (r) return r;
  return stream_begin_single(c, seed, first, n);
}

rmc_status rmc_stream_step(rmc_ctx *c, rmc_run_stats *slice, int64_t *remaining) {
  rmc_status r = enter(c);
  if (r) return r;
  return stream_step(c, slice, remaining);
}

rmc_status rmc_stream_end(rmc_ctx *c, rmc_run_stats *total) {
  rmc_status r = enter(c);
  if (r) return r;
  if (!c->s_open) return fail(c, RMC_ESTATE, "no open stream (rmc_stream_begin)");
  return stream_finish(c, nullptr, total);
}

rmc_status rmc_run(rmc_ctx *c, uint64_t seed, int64_t first, int64_t n, rmc_run_stats *stats) {
  rmc_status r = enter(c);
  if (r) return r;
  r = stream_begin_single(c, seed, first, n);
  if (r) return r;
  return stream_finish(c, nullptr, stats);
}

rmc_status rmc_get_packets(rmc_ctx *c, int32_t *status, double *x, double *k, double *pos, int32_t *nscat,
                           double *path, int mem) {
  rmc_status r = enter(c);
  if (r) return r;
  const int64_t n = c->last_n;
  if (n <= 0) return fail(c, RMC_ESTATE, "no run yet");
  if ((r = download(c, status, c->o_status.p, n * 4, mem))) return r;
  if ((r = download(c, x, c->o_x.p, n * 8, mem))) return r;
  if ((r = download(c, k, c->o_k.p, n * 24, mem))) return r;
  if ((r = download(c, pos, c->o_pos.p, n * 24, mem))) return r;
  if ((r = download(c, nscat, c->o_nscat.p, n * 4, mem))) return r;
  if ((r = download(c, path, c->o_path.p, n * 8, mem))) return r;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return RMC_OK;
}

rmc_status rmc_get_spectrum(rmc_ctx *c, int nbins, double x_min, double x_max, double *hist, int mem) {
  rmc_status r = enter(c);
  if (r) return r;
  if (nbins <= 0 || !(x_max > x_min) || !hist) return fail(c, RMC_EINVAL, "bad histogram");
  if (c->last_n <= 0) return fail(c, RMC_ESTATE, "no run yet");
  HIPCHK(c, c->tmp1.ensure((size_t)nbins * 8));
  HIPCHK(c, c->tmp2.ensure((size_t)nbins * 8));
  HIPCHK(c, launch_fill_u64(c->tmp1.as<unsigned long long>(), nbins, 0ull, c->stream));
  HIPCHK(c, launch_hist(c->last_n, c->o_status.as<int32_t>(), c->o_x.as<double>(), nbins, x_min, x_max - x_min,
                        c->tmp1.as<unsigned long long>(), c->stream));
  double *dst = mem == RMC_DEVICE ? hist : c->tmp2.as<double>();
  HIPCHK(c, launch_u64_to_f64(c->tmp1.as<unsigned long long>(), dst, nbins, c->stream));
  if (mem != RMC_DEVICE)
    HIPCHK(c, hipMemcpyAsync(hist, c->tmp2.p, (size_t)nbins * 8, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return RMC_OK;
}

rmc_status rmc_get_spectrum_noalloc(rmc_ctx *c, int nbins, double x_min, double x_max, double *hist) {
  rmc_status r = enter(c);
  if (r) return r;
  if (nbins <= 0 || nbins > NOALLOC_MAX_BINS)
    return fail(c, RMC_EINVAL, "nbins %d outside [1, %d], the fixed counter array of this call", nbins,
                NOALLOC_MAX_BINS);
  if (!(x_max > x_min) || !hist) return fail(c, RMC_EINVAL, "bad histogram");
  if (c->last_n <= 0) return fail(c, RMC_ESTATE, "no run yet");
  // the counters keep the last call's values: cleared by a fill kernel
  HIPCHK(c, launch_fill_u64(c->scratch, nbins, 0ull, c->stream));
  HIPCHK(c, launch_hist(c->last_n, c->o_status.as<int32_t>(), c->o_x.as<double>(), nbins, x_min, x_max - x_min,
                        c->scratch, c->stream));
  HIPCHK(c, launch_u64_to_f64(c->scratch, hist, nbins, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return RMC_OK;
}

rmc_status rmc_get_cube(rmc_ctx *c, int id, void *out, int dtype, int mem) {
  rmc_status r = enter(c);
  if (r) return r;
  if (id < 0 || id >= (int)c->obs.size() || !out) return fail(c, RMC_EINVAL, "bad observer id");
  ObsHost &o = c->obs[id];
  const bool f32 = c->precision == RMC_FP32_BULK;
  const int64_t n = (int64_t)o.n_elems;
  if ((dtype == RMC_F64) == !f32) {
    const size_t bytes = n * (f32 ? 4 : 8);
    HIPCHK(c, hipMemcpyAsync(out, o.cube.p, bytes, mem == RMC_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                             c->stream));
  } else {
    const size_t bytes = n * (dtype == RMC_F64 ? 8 : 4);
    void *dst = out;
    if (mem != RMC_DEVICE) {
      HIPCHK(c, c->tmp3.ensure(bytes));
      dst = c->tmp3.p;
    }
    if (dtype == RMC_F64) HIPCHK(c, launch_f32_to_f64(o.cube.as<float>(), (double *)dst, n, c->stream));
    else HIPCHK(c, launch_f64_to_f32(o.cube.as<double>(), (float *)dst, n, c->stream));
    if (mem != RMC_DEVICE) HIPCHK(c, hipMemcpyAsync(out, dst, bytes, hipMemcpyDeviceToHost, c->stream));
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return RMC_OK;
}

rmc_status rmc_trace_cells(rmc_ctx *c, int64_t n, const double *orig, const double *dir, int32_t max_cells,
                           int32_t *leaf_out, double *seg_out, int32_t *n_out, int mem) {
  rmc_status r = enter(c);
  if (r) return r;
  if (!c->has_mesh) return fail(c, RMC_ESTATE, "no mesh");
  if (n <= 0 || max_cells <= 0 || !orig || !dir || !leaf_out || !seg_out || !n_out) return fail(c, RMC_EINVAL, "bad trace arguments");
  ProblemK pb;
  std::memset(&pb, 0, sizeof pb);
  pb.nodes = c->nodes.as<int32_t>();
  pb.L = c->L;
  pb.top = c->top_level > 0 ? c->top.as<int32_t>() : nullptr;
  pb.top_level = c->top_level;
  pb.domain = c->domain;
  for (int d = 0; d < 4; ++d) pb.dom[d] = c->dom[d];
  const double *o = orig, *k = dir;
  int32_t *lo = leaf_out, *no = n_out;
  double *so = seg_out;
  const size_t cells = (size_t)n * max_cells;
  if (mem != RMC_DEVICE) {
    if ((r = upload(c, c->tmp1, orig, n * 24, RMC_HOST))) return r;
    if ((r = upload(c, c->tmp2, dir, n * 24, RMC_HOST))) return r;
    HIPCHK(c, c->tmp3.ensure(cells * 4));
    HIPCHK(c, c->tmp4.ensure(cells * 8));
    HIPCHK(c, c->tmp5.ensure(n * 4));
    o = c->tmp1.as<double>();
    k = c->tmp2.as<double>();
    lo = c->tmp3.as<int32_t>();
    so = c->tmp4.as<double>();
    no = c->tmp5.as<int32_t>();
  }
  HIPCHK(c, launch_trace(pb, n, o, k, max_cells, lo, so, no, c->stream));
  if (mem != RMC_DEVICE) {
    HIPCHK(c, hipMemcpyAsync(leaf_out, lo, cells * 4, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(seg_out, so, cells * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(n_out, no, n * 4, hipMemcpyDeviceToHost, c->stream));
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return RMC_OK;
}

rmc_status rmc_tau(rmc_ctx *c, int64_t n, const double *orig, const double *dir, const double *x_ext, double *tau_out,
                   int mem) {
  rmc_status r = enter(c);
  if (r) return r;
  r = ready(c, false);
  if (r) return r;
  if (n <= 0 || !orig || !dir || !x_ext || !tau_out) return fail(c, RMC_EINVAL, "bad tau arguments");
  ProblemK pb;
  make_problem(c, 0, 0, 0, pb);
  const double *o = orig, *k = dir, *x = x_ext;
  double *t = tau_out;
  if (mem != RMC_DEVICE) {
    if ((r = upload(c, c->tmp1, orig, n * 24, RMC_HOST))) return r;
    if ((r = upload(c, c->tmp2, dir, n * 24, RMC_HOST))) return r;
    if ((r = upload(c, c->tmp3, x_ext, n * 8, RMC_HOST))) return r;
    HIPCHK(c, c->tmp4.ensure(n * 8));
    o = c->tmp1.as<double>();
    k = c->tmp2.as<double>();
    x = c->tmp3.as<double>();
    t = c->tmp4.as<double>();
  }
  HIPCHK(c, launch_tau(c->precision == RMC_FP32_BULK, pb, n, o, k, x, t, c->stream));
  if (mem != RMC_DEVICE) HIPCHK(c, hipMemcpyAsync(tau_out, t, n * 8, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return RMC_OK;
}

static rmc_status image_common(rmc_ctx *c, int id, int64_t n, const double *orig, const double *x_ext, const double *w,
                               int mem, const double **o, const double **x, const double **ww) {
  rmc_status r = ready(c, false);
  if (r) return r;
  if (id < 0 || id >= (int)c->obs.size()) return fail(c, RMC_EINVAL, "bad observer id");
  if (n <= 0 || !orig || !x_ext || !w) return fail(c, RMC_EINVAL, "bad ray arguments");
  *o = orig;
  *x = x_ext;
  *ww = w;
  if (mem != RMC_DEVICE) {
    if ((r = upload(c, c->tmp1, orig, n * 24, RMC_HOST))) return r;
    if ((r = upload(c, c->tmp2, x_ext, n * 8, RMC_HOST))) return r;
    if ((r = upload(c, c->tmp3, w, n * 8, RMC_HOST))) return r;
    *o = c->tmp1.as<double>();
    *x = c->tmp2.as<double>();
    *ww = c->tmp3.as<double>();
  }
  HIPCHK(c, c->d_stats.ensure(N_STATS * 8));
  HIPCHK(c, launch_fill_u64(c->d_stats.as<unsigned long long>(), N_STATS, 0ull, c->stream));
  return RMC_OK;
}

rmc_status rmc_raycast_image(rmc_ctx *c, int id, int64_t n, const double *orig, const double *x_ext, const double *w,
                             double *image, int mem) {
  rmc_status r = enter(c);
  if (r) return r;
  const double *o, *x, *ww;
  if ((r = image_common(c, id, n, orig, x_ext, w, mem, &o, &x, &ww))) return r;
  if (!image) return fail(c, RMC_EINVAL, "null image");
  ProblemK pb;
  make_problem(c, 0, 0, 0, pb);
  const size_t npix = (size_t)c->obs[id].k.nx * c->obs[id].k.ny;
  double *img = image;
  if (mem != RMC_DEVICE) {
    HIPCHK(c, c->tmp4.ensure(npix * 8));
    img = c->tmp4.as<double>();
  }
  HIPCHK(c, hipMemsetAsync(img, 0, npix * 8, c->stream));
  HIPCHK(c, hipEventRecord(c->ev0, c->stream));
  HIPCHK(c, launch_image_fwd(c->precision == RMC_FP32_BULK, pb, id, n, o, x, ww, img,
                             c->d_stats.as<unsigned long long>() + S_PEEL_CROSS, c->stream));
  HIPCHK(c, hipEventRecord(c->ev1, c->stream));
  c->image_done = true;
  if (mem != RMC_DEVICE) HIPCHK(c, hipMemcpyAsync(image, img, npix * 8, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return RMC_OK;
}

rmc_status rmc_image_stats(rmc_ctx *c, uint64_t *crossings, double *kernel_ms) {
  rmc_status r = enter(c);
  if (r) return r;
  if (!c->image_done) return fail(c, RMC_ESTATE, "no image call yet");
  unsigned long long h = 0;
  HIPCHK(c, hipMemcpyAsync(&h, c->d_stats.as<unsigned long long>() + S_PEEL_CROSS, 8, hipMemcpyDeviceToHost,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  float ms = 0.f;
  HIPCHK(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
  if (crossings) *crossings = h;
  if (kernel_ms) *kernel_ms = ms;
  return RMC_OK;
}

// After an image gradient: the velocity-vector gradient g_v[3n] = g_vlos
// k_obs from the line-of-sight one at dv (device), into gvv (mem).
static rmc_status vlos_to_v(rmc_ctx *c, int id, const double *dv, double *gvv, int mem) {
  if (!gvv) return RMC_OK;
  const size_t nl = (size_t)c->n_leaves;
  double *dst = gvv;
  if (mem != RMC_DEVICE) {
    HIPCHK(c, c->tmp6.ensure(nl * 24));
    dst = c->tmp6.as<double>();
  }
  HIPCHK(c, launch_vlos_to_v((int64_t)nl, dv, c->obs[id].k.k, dst, c->stream));
  if (mem != RMC_DEVICE) HIPCHK(c, hipMemcpyAsync(gvv, dst, nl * 24, hipMemcpyDeviceToHost, c->stream));
  return RMC_OK;
}

rmc_status rmc_raycast_image_backward(rmc_ctx *c, int id, int64_t n, const double *orig, const double *x_ext,
                                      const double *w, const double *G, double *gn, double *gk, double *gv,
                                      double *gvv, int mem) {
  rmc_status r = enter(c);
  if (r) return r;
  if (c->voigt_exact) return fail(c, RMC_EUNSUPPORTED, "the image gradient needs RMC_OPT_VOIGT 0 (Tasitsiomi dH/dx)");
  const double *o, *x, *ww;
  if ((r = image_common(c, id, n, orig, x_ext, w, mem, &o, &x, &ww))) return r;
  if (!G || !gn || !gk || !gv) return fail(c, RMC_EINVAL, "null gradient buffer");
  ProblemK pb;
  make_problem(c, 0, 0, 0, pb);
  const size_t npix = (size_t)c->obs[id].k.nx * c->obs[id].k.ny;
  const size_t nl = (size_t)c->n_leaves;
  const double *Gd = G;
  double *a = gn, *b = gk, *d = gv;
  if (mem != RMC_DEVICE) {
    if ((r = upload(c, c->tmp4, G, npix * 8, RMC_HOST))) return r;
    Gd = c->tmp4.as<double>();
    HIPCHK(c, c->tmp5.ensure(nl * 24));
    a = c->tmp5.as<double>();
    b = a + nl;
    d = b + nl;
  }
  HIPCHK(c, hipMemsetAsync(a, 0, nl * 8, c->stream));
  HIPCHK(c, hipMemsetAsync(b, 0, nl * 8, c->stream));
  HIPCHK(c, hipMemsetAsync(d, 0, nl * 8, c->stream));
  const double inv_vth_ref = 1.0 / line_q(c->lines[0], c->T_ref).vth;
  HIPCHK(c, hipEventRecord(c->ev0, c->stream));
  HIPCHK(c, launch_image_bwd(c->precision == RMC_FP32_BULK, pb, id, n, o, x, ww, Gd, inv_vth_ref, a, b, d,
                             c->d_stats.as<unsigned long long>() + S_PEEL_CROSS, c->stream));
  HIPCHK(c, hipEventRecord(c->ev1, c->stream));
  c->image_done = true;
  if ((r = vlos_to_v(c, id, d, gvv, mem))) return r;
  if (mem != RMC_DEVICE) {
    HIPCHK(c, hipMemcpyAsync(gn, a, nl * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(gk, b, nl * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(gv, d, nl * 8, hipMemcpyDeviceToHost, c->stream));
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return RMC_OK;
}

constexpr unsigned long long TAPE_MAX_BYTES = 32ull << 30;   // crossing-list limit

// Device view of the context's tape buffers.
static TapeK tape_view(rmc_ctx *c) {
  TapeK t;
  t.leaf = c->tp_leaf.as<int32_t>();
  t.seg = c->tp_seg.p;
  t.next = c->tp_next.as<int64_t>();
  t.first = c->tp_first.as<int64_t>();
  t.count = c->tp_count.as<int32_t>();
  t.pix = c->tp_pix.as<int32_t>();
  t.wt = c->tp_wt.as<double>();
  t.x = c->tp_x.as<double>();
  t.ctl = c->tp_ctl.as<unsigned long long>();
  t.cap = c->tp_cap;
  return t;
}

rmc_status rmc_raycast_image_tape(rmc_ctx *c, int id, int64_t n, const double *orig, const double *x_ext,
                                  const double *w, double *image, int mem) {
  rmc_status r = enter(c);
  if (r) return r;
  const double *o, *x, *ww;
  if ((r = image_common(c, id, n, orig, x_ext, w, mem, &o, &x, &ww))) return r;
  if (!image) return fail(c, RMC_EINVAL, "null image");
  c->tp_valid = false;
  ProblemK pb;
  make_problem(c, 0, 0, 0, pb);
  const bool f32 = c->precision == RMC_FP32_BULK;
  const size_t seg_bytes = f32 ? 4 : 8;
  const size_t chunk_bytes = (size_t)TAPE_ENTRIES * (4 + seg_bytes) + 8;
  const int64_t waves = tape_waves(n);
  HIPCHK(c, c->tp_first.ensure((size_t)waves * 8));
  HIPCHK(c, c->tp_count.ensure((size_t)n * 4));
  HIPCHK(c, c->tp_pix.ensure((size_t)n * 4));
  HIPCHK(c, c->tp_wt.ensure((size_t)n * 8));
  HIPCHK(c, c->tp_x.ensure((size_t)n * 8));
  HIPCHK(c, c->tp_ctl.ensure(8));
  // first guess: four chunks (128 crossings per ray) per wave, or what the
  // context used before; a pass that runs out is repeated with the exact
  // number of chunks it asked for (the walks do not change)
  if (c->tp_cap < (unsigned long long)waves * 4) c->tp_cap = (unsigned long long)waves * 4;
  const size_t npix = (size_t)c->obs[id].k.nx * c->obs[id].k.ny;
  double *img = image;
  if (mem != RMC_DEVICE) {
    HIPCHK(c, c->tmp4.ensure(npix * 8));
    img = c->tmp4.as<double>();
  }
  for (int attempt = 0;; ++attempt) {
    if ((double)c->tp_cap * (double)chunk_bytes > (double)TAPE_MAX_BYTES)
      return fail(c, RMC_ENOMEM, "tape of %llu chunks exceeds %llu bytes (use rmc_raycast_image_backward)",
                  c->tp_cap, TAPE_MAX_BYTES);
    HIPCHK(c, c->tp_leaf.ensure((size_t)c->tp_cap * TAPE_ENTRIES * 4));
    HIPCHK(c, c->tp_seg.ensure((size_t)c->tp_cap * TAPE_ENTRIES * seg_bytes));
    HIPCHK(c, c->tp_next.ensure((size_t)c->tp_cap * 8));
    HIPCHK(c, launch_fill_u64(c->tp_ctl.as<unsigned long long>(), 1, 0ull, c->stream));
    HIPCHK(c, launch_fill_u64(c->d_stats.as<unsigned long long>(), N_STATS, 0ull, c->stream));
    HIPCHK(c, hipMemsetAsync(img, 0, npix * 8, c->stream));
    HIPCHK(c, hipEventRecord(c->ev0, c->stream));
    HIPCHK(c, launch_image_fwd_tape(f32, pb, id, n, o, x, ww, img, c->d_stats.as<unsigned long long>() + S_PEEL_CROSS,
                                    tape_view(c), c->stream));
    HIPCHK(c, hipEventRecord(c->ev1, c->stream));
    unsigned long long asked = 0;
    HIPCHK(c, hipMemcpyAsync(&asked, c->tp_ctl.p, 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (asked <= c->tp_cap) break;
    if (attempt >= 2) return fail(c, RMC_EDEVICE, "tape pass asked for %llu chunks again", asked);
    c->tp_cap = asked;
  }
  c->image_done = true;
  c->tp_valid = true;
  c->tp_obs = id;
  c->tp_n = n;
  c->tp_gen = c->gen;
  if (mem != RMC_DEVICE) HIPCHK(c, hipMemcpyAsync(image, img, npix * 8, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return RMC_OK;
}

rmc_status rmc_raycast_image_backward_tape(rmc_ctx *c, const double *G, double *gn, double *gk, double *gv,
                                           double *gvv, int mem) {
  rmc_status r = enter(c);
  if (r) return r;
  if (c->voigt_exact) return fail(c, RMC_EUNSUPPORTED, "the image gradient needs RMC_OPT_VOIGT 0 (Tasitsiomi dH/dx)");
  if ((r = ready(c, false))) return r;
  if (!c->tp_valid || c->tp_gen != c->gen || c->tp_obs >= (int)c->obs.size())
    return fail(c, RMC_ESTATE, "no tape for the current model (rmc_raycast_image_tape)");
  if (!G || !gn || !gk || !gv) return fail(c, RMC_EINVAL, "null gradient buffer");
  ProblemK pb;
  make_problem(c, 0, 0, 0, pb);
  const int id = c->tp_obs;
  const size_t npix = (size_t)c->obs[id].k.nx * c->obs[id].k.ny;
  const size_t nl = (size_t)c->n_leaves;
  const double *Gd = G;
  double *a = gn, *b = gk, *d = gv;
  if (mem != RMC_DEVICE) {
    if ((r = upload(c, c->tmp4, G, npix * 8, RMC_HOST))) return r;
    Gd = c->tmp4.as<double>();
    HIPCHK(c, c->tmp5.ensure(nl * 24));
    a = c->tmp5.as<double>();
    b = a + nl;
    d = b + nl;
  }
  HIPCHK(c, hipMemsetAsync(a, 0, nl * 8, c->stream));
  HIPCHK(c, hipMemsetAsync(b, 0, nl * 8, c->stream));
  HIPCHK(c, hipMemsetAsync(d, 0, nl * 8, c->stream));
  HIPCHK(c, c->d_stats.ensure(N_STATS * 8));
  HIPCHK(c, launch_fill_u64(c->d_stats.as<unsigned long long>(), N_STATS, 0ull, c->stream));
  const double inv_vth_ref = 1.0 / line_q(c->lines[0], c->T_ref).vth;
  HIPCHK(c, hipEventRecord(c->ev0, c->stream));
  HIPCHK(c, launch_image_bwd_tape(c->precision == RMC_FP32_BULK, pb, id, c->tp_n, tape_view(c), Gd, inv_vth_ref, a, b,
                                  d, c->d_stats.as<unsigned long long>() + S_PEEL_CROSS, c->stream));
  HIPCHK(c, hipEventRecord(c->ev1, c->stream));
  c->image_done = true;
  if ((r = vlos_to_v(c, id, d, gvv, mem))) return r;
  if (mem != RMC_DEVICE) {
    HIPCHK(c, hipMemcpyAsync(gn, a, nl * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(gk, b, nl * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(gv, d, nl * 8, hipMemcpyDeviceToHost, c->stream));
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return RMC_OK;
}

namespace {

// Upload the problem descriptors of a batch and open a stream over them.
rmc_status batch_open(rmc_ctx *const *P, int np, const uint64_t *seeds, const int64_t *npk) {
  rmc_ctx *c0 = P[0];
  rmc_status r;
  int maxL = 1;
  for (int i = 0; i < np; ++i) {
    rmc_ctx *c = P[i];
    if (!c || c->device != c0->device || c->precision != c0->precision)
      return fail(c0, RMC_EINVAL, "problem %d: contexts must share device and precision", i);
    r = ready(c, true);
    if (r) return fail(c0, r, "problem %d: %s", i, c->err.c_str());
    if (npk[i] < 0 || npk[i] > c->n_src) return fail(c0, RMC_EINVAL, "problem %d: packet count outside the sources", i);
    r = ensure_outputs(c, npk[i], c0->stream);
    if (r) return fail(c0, r, "problem %d: %s", i, c->err.c_str());
    maxL = std::max(maxL, c->L);
  }
  if (np > (1 << 19)) return fail(c0, RMC_EINVAL, "at most 2^19 problems per batch");
  bool any_obs = false;
  for (int i = 0; i < np; ++i) any_obs = any_obs || !P[i]->obs.empty();
  r = peel_queue(c0, &c0->s_pq);
  if (r) return r;
  if (!any_obs) c0->s_pq = nullptr;
  c0->s_defer = c0->s_pq != nullptr || !any_obs;
  c0->s_one_line = true;
  for (int i = 0; i < np; ++i)
    c0->s_one_line = c0->s_one_line && P[i]->n_lines == 1 && P[i]->lines[0].n_fluor == 0;
  c0->b_host.resize(np);
  c0->b_starts_host.assign(np + 1, 0);
  for (int i = 0; i < np; ++i) {
    P[i]->last_n = npk[i];
    make_problem(P[i], 0, npk[i], seeds[i], c0->b_host[i]);
    r = apply_spectrum(P[i], c0->b_host[i], 0, npk[i], c0->stream);
    if (r) return fail(c0, r, "problem %d: %s", i, P[i]->err.c_str());
    c0->b_host[i].pq = c0->s_pq;
    c0->b_host[i].index = i;
    c0->b_starts_host[i + 1] = c0->b_starts_host[i] + npk[i];
  }
  const int64_t tot = c0->b_starts_host[np];
  HIPCHK(c0, c0->b_probs.ensure(sizeof(ProblemK) * np));
  HIPCHK(c0, c0->b_starts.ensure(8 * (np + 1)));
  HIPCHK(c0, hipMemcpyAsync(c0->b_probs.p, c0->b_host.data(), sizeof(ProblemK) * np, hipMemcpyHostToDevice, c0->stream));
  HIPCHK(c0, hipMemcpyAsync(c0->b_starts.p, c0->b_starts_host.data(), 8 * (np + 1), hipMemcpyHostToDevice, c0->stream));
  c0->s_probs = c0->b_probs.as<ProblemK>();
  c0->s_starts = c0->b_starts.as<int64_t>();
  c0->s_members.assign(P, P + np);
  return stream_open(c0, tot, np, maxL, true);
}

}  // namespace

rmc_status rmc_batch_begin(rmc_ctx *const *P, int np, const uint64_t *seeds, const int64_t *npk) {
  if (!P || np <= 0 || !P[0] || !seeds || !npk) return RMC_EINVAL;
  rmc_status r = enter(P[0]);
  if (r) return r;
  return batch_open(P, np, seeds, npk);
}

rmc_status rmc_batch_run(rmc_ctx *const *P, int np, const uint64_t *seeds, const int64_t *npk,
                         rmc_run_stats *per, rmc_run_stats *total) {
  if (!P || np <= 0 || !seeds || !npk) return RMC_EINVAL;
  rmc_ctx *c0 = P[0];
  rmc_status r = enter(c0);
  if (r) return r;
  r = batch_open(P, np, seeds, npk);
  if (r) return r;
  return stream_finish(c0, per, total);
}

namespace {

// Copy every observer cube of the members into one buffer (save) or back
// from it (restore), on c0's stream.
rmc_status cube_snapshot(rmc_ctx *const *P, int np, DevBuf &snap, bool save) {
  rmc_ctx *c0 = P[0];
  size_t total = 0;
  for (int i = 0; i < np; ++i)
    for (auto &o : P[i]->obs) total += o.n_elems * (P[i]->precision == RMC_FP32_BULK ? 4 : 8);
  if (save) HIPCHK(c0, snap.ensure(total));
  size_t off = 0;
  for (int i = 0; i < np; ++i)
    for (auto &o : P[i]->obs) {
      const size_t b = o.n_elems * (P[i]->precision == RMC_FP32_BULK ? 4 : 8);
      char *s = (char *)snap.p + off;
      HIPCHK(c0, hipMemcpyAsync(save ? (void *)s : o.cube.p, save ? o.cube.p : (const void *)s, b,
                                hipMemcpyDeviceToDevice, c0->stream));
      off += b;
    }
  HIPCHK(c0, hipStreamSynchronize(c0->stream));
  return RMC_OK;
}

rmc_status autotune_trials(rmc_ctx *const *P, int np, const uint64_t *seeds, const int64_t *npk, int trials,
                           int best[3]);

}  // namespace

rmc_status rmc_batch_autotune(rmc_ctx *const *P, int np, const uint64_t *seeds, const int64_t *npk, int trials,
                              int best[3]) {
  if (!P || np <= 0 || !seeds || !npk || trials <= 0) return RMC_EINVAL;
  rmc_status r = enter(P[0]);
  if (r) return r;
  // the trial launches deposit peel-off rays into the members' cubes: they
  // are put back as they were afterwards
  DevBuf snap;
  r = cube_snapshot(P, np, snap, true);
  if (r == RMC_OK) {
    r = autotune_trials(P, np, seeds, npk, trials, best);
    const rmc_status r2 = cube_snapshot(P, np, snap, false);
    if (r == RMC_OK) r = r2;
  }
  snap.release();
  return r;
}

namespace {

rmc_status autotune_trials(rmc_ctx *const *P, int np, const uint64_t *seeds, const int64_t *npk, int trials,
                           int best[3]) {
  rmc_ctx *c0 = P[0];
  rmc_status r;
  const int blocks[] = {64, 128, 256};
  const int refills[] = {1, 8, 32};
  const int slices[] = {256, 2048, 8192};
  double best_rate = -1.0;
  int bb = c0->block, br = c0->refill, bs = c0->slice_iters;
  for (int b : blocks)
    for (int f : refills)
      for (int sl : slices) {
        c0->block = b;
        c0->refill = f;
        c0->slice_iters = sl;
        r = batch_open(P, np, seeds, npk);
        if (r) return r;
        // every shape runs the same loop iterations per lane: an untimed
        // start (lanes starting their first packets), then `trials` windows
        // of 8192 iterations, each step timed whole (launches,
        // synchronisation and counters), so that shapes are ranked on the
        // same stretch of the run with what a shorter slice costs per unit
        // of work beyond its kernel times
        constexpr int64_t WINDOW = 8192;
        double work = 0.0, ms = 0.0;
        int64_t done = 0;
        const int64_t start = WINDOW, end = WINDOW * (1 + (int64_t)trials);
        while (done < end) {
          rmc_run_stats st;
          int64_t rem = 0;
          const auto t0 = std::chrono::steady_clock::now();
          r = stream_step(c0, &st, &rem);
          if (r) return r;
          const double wall = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
          if (done >= start || rem == 0) {
            work += (double)st.scatterings + (double)st.crossings + (double)st.peel_crossings;
            ms += wall;
          }
          done += sl;
          if (rem == 0) break;
        }
        c0->s_open = false;
        const double rate = ms > 0.0 ? work / ms : 0.0;
        if (rate > best_rate) {
          best_rate = rate;
          bb = b;
          br = f;
          bs = sl;
        }
      }
  c0->block = bb;
  c0->refill = br;
  c0->slice_iters = bs;
  if (best) {
    best[0] = bb;
    best[1] = br;
    best[2] = bs;
  }
  return RMC_OK;
}

}  // namespace

rmc_status rmc_mesh_check(int64_t n, const int8_t *level, const int32_t *ijk, char *msg, int msg_len) {
  std::vector<int32_t> nodes;
  int L = 0;
  std::string m;
  rmc_status r = build_tree(n, level, ijk, nodes, L, m);
  if (msg && msg_len > 0) {
    std::strncpy(msg, m.c_str(), (size_t)msg_len - 1);
    msg[msg_len - 1] = 0;
  }
  return r;
}

rmc_status rmc_line_quantities(const rmc_line *ln, double T, double out[5]) {
  if (!ln || !out || !(T > 0) || !(ln->lambda0_A > 0) || !(ln->mass_amu > 0)) return RMC_EINVAL;
  const LineQ q = line_q(*ln, T);
  out[0] = q.nu0;
  out[1] = q.vth;
  out[2] = q.dnu;
  out[3] = q.a;
  out[4] = q.sigma0;
  return RMC_OK;
}

}  // extern "C"
