// Drives the oracle's entry points on small inputs, for a build with the
// address and undefined-behaviour sanitizers (tests/test_sanitizers.py).
// Exits 0 when every call returned what it should; a sanitizer report
// aborts the program.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "rmc_oracle.h"

namespace {

struct Mesh {
  std::vector<int8_t> level;
  std::vector<int32_t> ijk;
  int64_t n() const { return (int64_t)level.size(); }
};

Mesh uniform(int l) {
  Mesh m;
  const int s = 1 << l;
  for (int k = 0; k < s; ++k)
    for (int j = 0; j < s; ++j)
      for (int i = 0; i < s; ++i) {
        m.level.push_back((int8_t)l);
        m.ijk.insert(m.ijk.end(), {i, j, k});
      }
  return m;
}

// uniform level 2 with the eight cells nearest the centre split once
Mesh refined() {
  Mesh m;
  for (int k = 0; k < 4; ++k)
    for (int j = 0; j < 4; ++j)
      for (int i = 0; i < 4; ++i) {
        const bool inner = i >= 1 && i <= 2 && j >= 1 && j <= 2 && k >= 1 && k <= 2;
        if (!inner) {
          m.level.push_back(2);
          m.ijk.insert(m.ijk.end(), {i, j, k});
          continue;
        }
        for (int c = 0; c < 8; ++c) {
          m.level.push_back(3);
          m.ijk.insert(m.ijk.end(), {2 * i + (c & 1), 2 * j + ((c >> 1) & 1), 2 * k + ((c >> 2) & 1)});
        }
      }
  return m;
}

int failures = 0;
void check(bool ok, const char *what) {
  if (!ok) {
    std::fprintf(stderr, "FAIL: %s\n", what);
    ++failures;
  }
}

}  // namespace

int main() {
  Mesh u = uniform(3), r = refined();
  check(orc_mesh_validate(u.n(), u.level.data(), u.ijk.data()) == 0, "uniform mesh valid");
  check(orc_mesh_validate(r.n(), r.level.data(), r.ijk.data()) == 0, "refined mesh valid");
  check(orc_mesh_validate(u.n() - 1, u.level.data() + 1, u.ijk.data() + 3) == -3, "gap");
  Mesh bad = u;
  bad.ijk[0] = 8;
  check(orc_mesh_validate(bad.n(), bad.level.data(), bad.ijk.data()) == -1, "out of range");
  Mesh dup = u;
  dup.level.push_back(3);
  dup.ijk.insert(dup.ijk.end(), {0, 0, 0});
  check(orc_mesh_validate(dup.n(), dup.level.data(), dup.ijk.data()) == -2, "duplicate");

  // a dusty, moving sphere on the refined mesh with two observers
  const int64_t n = r.n();
  std::vector<double> nh(n, 1e-4), T(n, 1e4), v(3 * n), kd(n, 3e-22);
  for (int64_t i = 0; i < 3 * n; ++i) v[i] = 1e6 * std::sin(0.7 * (double)i);
  orc_problem pb{};
  pb.n_leaves = n;
  pb.level = r.level.data();
  pb.ijk = r.ijk.data();
  pb.box_cm = 3.0857e21;
  pb.n_hi = nh.data();
  pb.T = T.data();
  pb.v = v.data();
  pb.kappa_d = kd.data();
  pb.domain_kind = ORC_DOM_SPHERE;
  pb.domain[0] = pb.domain[1] = pb.domain[2] = 0.5;
  pb.domain[3] = 0.5;
  pb.n_lines = 1;
  pb.lines[0] = orc_line{1215.67, 6.265e8, 0.416, 1.00794, 1.0, ORC_PHASE_LYA, 1, 0, {0, 0}, {0, 0}};
  pb.T_ref = 1e4;
  pb.albedo = 0.32;
  pb.g_hg = 0.73;
  const int np = 200;
  std::vector<double> pos(3 * np, 0.5), xs(np, 0.0);
  orc_observer ob[2] = {};
  const double ks[2][3] = {{0, 0, 1}, {0.6, 0, 0.8}};
  for (int o = 0; o < 2; ++o) {
    for (int d = 0; d < 3; ++d) ob[o].k[d] = ks[o][d];
    ob[o].nx = 8;
    ob[o].ny = 8;
    ob[o].nbins = 10;
    ob[o].fov[0] = ob[o].fov[2] = -0.5;
    ob[o].fov[1] = ob[o].fov[3] = 0.5;
    ob[o].x_min = -30;
    ob[o].x_max = 30;
  }
  std::vector<double> c0(8 * 8 * 10), c1(8 * 8 * 10);
  double *cubes[2] = {c0.data(), c1.data()};
  std::vector<int32_t> st(np), ns(np);
  std::vector<double> xo(np), ko(3 * np), po(3 * np), path(np);
  orc_stats s{};
  for (double cut : {0.0, 746.0}) {
    pb.peel_tau_cut = cut;
    check(orc_run(&pb, np, pos.data(), nullptr, xs.data(), 7, 0, np, 2, ob, cubes, st.data(), xo.data(),
                  ko.data(), po.data(), ns.data(), path.data(), 2, &s) == 0, "orc_run");
    check(s.emitted == np && s.escaped + s.absorbed + s.stuck == np, "conservation");
  }
  pb.peel_tau_cut = 0.0;
  pb.core_skip_tau = 1.0;
  pb.core_skip_frac = 0.2;
  check(orc_run(&pb, np, pos.data(), nullptr, xs.data(), 8, 0, np, 1, ob, cubes, st.data(), xo.data(), ko.data(),
                po.data(), ns.data(), path.data(), 2, &s) == 0, "orc_run core skip");
  pb.core_skip_tau = 0.0;

  // probes and the image adjoint
  const int nr = 50;
  std::vector<double> orig(3 * nr), dir(3 * nr), xr(nr), w(nr, 1.0 / (4 * M_PI)), tau(nr);
  for (int i = 0; i < nr; ++i) {
    const double a = 0.37 * i, b = 0.11 * i;
    dir[3 * i] = std::sin(a) * std::cos(b);
    dir[3 * i + 1] = std::sin(a) * std::sin(b);
    dir[3 * i + 2] = std::cos(a);
    for (int d = 0; d < 3; ++d) orig[3 * i + d] = 0.3 + 0.008 * ((i * (d + 3)) % 50);
    xr[i] = -5.0 + 0.2 * i;
  }
  const int mc = 64;
  std::vector<int32_t> leaf(nr * mc), cnt(nr);
  std::vector<double> seg(nr * mc);
  check(orc_trace(&pb, nr, orig.data(), dir.data(), mc, leaf.data(), seg.data(), cnt.data()) == 0, "trace");
  check(orc_tau(&pb, nr, orig.data(), dir.data(), xr.data(), tau.data()) == 0, "tau");
  std::vector<double> img(64), G(64), gn(n), gk(n), gv(n);
  for (int p = 0; p < 64; ++p) G[p] = std::cos(0.3 * p);
  int64_t ncr = 0;
  check(orc_raycast_image(&pb, &ob[0], nr, orig.data(), xr.data(), w.data(), img.data(), G.data(), gn.data(),
                          gk.data(), gv.data(), 2, &ncr) == 0 && ncr > 0, "raycast image");

  // samplers and line quantities
  std::vector<double> smp(2000);
  orc_sample_upar(1000, 2.5, 4.7e-4, 3, smp.data());
  orc_sample_upar(1000, 9.0, 4.7e-4, 3, smp.data());
  for (int kind = 0; kind < 4; ++kind) orc_sample_mu(1000, kind, 0.73, 4, smp.data());
  orc_sample_uperp(1000, 1.5, 5, smp.data());
  orc_single_scatter(1000, &pb.lines[0], 1e4, 1.0, 6, smp.data());
  double q[5];
  orc_line_quantities(&pb.lines[0], 1e4, q);
  check(q[4] > 5.8e-14 && q[4] < 6.0e-14, "sigma0");
  check(std::fabs(orc_voigt_h_exact(1e-3, 0.5) / orc_voigt_h(1e-3, 0.5) - 1) < 0.02, "voigt");
  std::printf("oracle driver: %d failures\n", failures);
  return failures ? 1 : 0;
}
