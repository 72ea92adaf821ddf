// Drives the library's host-only entry points (mesh validation and the
// breadth-first tree build, line quantities, the interface version) on
// valid and invalid meshes, for a build with the address and
// undefined-behaviour sanitizers on the host code (tests/test_sanitizers.py).
// No device is touched.  Exits 0 when every call returned what it should.
#include <cstdio>
#include <cstring>
#include <vector>

#include "rmc.h"

namespace {
int failures = 0;
void check(bool ok, const char *what) {
  if (!ok) {
    std::fprintf(stderr, "FAIL: %s\n", what);
    ++failures;
  }
}

void uniform(int l, std::vector<int8_t> &lv, std::vector<int32_t> &ijk) {
  const int s = 1 << l;
  for (int k = 0; k < s; ++k)
    for (int j = 0; j < s; ++j)
      for (int i = 0; i < s; ++i) {
        lv.push_back((int8_t)l);
        ijk.insert(ijk.end(), {i, j, k});
      }
}
}  // namespace

int main() {
  char msg[256];
  std::vector<int8_t> lv;
  std::vector<int32_t> ijk;
  uniform(3, lv, ijk);
  check(rmc_mesh_check((int64_t)lv.size(), lv.data(), ijk.data(), msg, sizeof msg) == RMC_OK, "uniform");
  // one leaf split into its eight children: still valid (and 2:1 graded)
  std::vector<int8_t> l2(lv.begin() + 1, lv.end());
  std::vector<int32_t> i2(ijk.begin() + 3, ijk.end());
  for (int c = 0; c < 8; ++c) {
    l2.push_back(4);
    i2.insert(i2.end(), {c & 1, (c >> 1) & 1, (c >> 2) & 1});
  }
  check(rmc_mesh_check((int64_t)l2.size(), l2.data(), i2.data(), msg, sizeof msg) == RMC_OK, "split leaf");
  // gap, overlap, out of range, a short message buffer
  check(rmc_mesh_check((int64_t)lv.size() - 1, lv.data() + 1, ijk.data() + 3, msg, sizeof msg) == RMC_EMESH, "gap");
  std::vector<int8_t> l3 = lv;
  std::vector<int32_t> i3 = ijk;
  l3.push_back(2);
  i3.insert(i3.end(), {0, 0, 0});
  check(rmc_mesh_check((int64_t)l3.size(), l3.data(), i3.data(), msg, 4) == RMC_EMESH && std::strlen(msg) < 4,
        "overlap");
  std::vector<int32_t> i4 = ijk;
  i4[0] = 99;
  check(rmc_mesh_check((int64_t)lv.size(), lv.data(), i4.data(), nullptr, 0) != RMC_OK, "out of range");
  std::vector<int8_t> l5 = lv;
  l5[0] = 20;
  check(rmc_mesh_check((int64_t)l5.size(), l5.data(), ijk.data(), msg, sizeof msg) != RMC_OK, "bad level");
  check(rmc_mesh_check(0, nullptr, nullptr, msg, sizeof msg) != RMC_OK, "empty");
  // not graded: level 1 beside level 3
  std::vector<int8_t> l6;
  std::vector<int32_t> i6;
  for (int c = 1; c < 8; ++c) {
    l6.push_back(1);
    i6.insert(i6.end(), {c & 1, (c >> 1) & 1, (c >> 2) & 1});
  }
  for (int c = 0; c < 7; ++c) {
    l6.push_back(2);
    i6.insert(i6.end(), {(c & 1), ((c >> 1) & 1), ((c >> 2) & 1)});
  }
  for (int c = 0; c < 8; ++c) {
    l6.push_back(3);
    i6.insert(i6.end(), {2 + (c & 1), 2 + ((c >> 1) & 1), 2 + ((c >> 2) & 1)});
  }
  check(rmc_mesh_check((int64_t)l6.size(), l6.data(), i6.data(), msg, sizeof msg) == RMC_EMESH, "not graded");
  rmc_line ly{};
  ly.lambda0_A = 1215.67;
  ly.A_ul = 6.265e8;
  ly.f_lu = 0.416;
  ly.mass_amu = 1.00794;
  ly.abundance = 1.0;
  double q[5];
  check(rmc_line_quantities(&ly, 1e4, q) == RMC_OK && q[4] > 5.8e-14 && q[4] < 6.0e-14, "line quantities");
  check(rmc_line_quantities(&ly, -1.0, q) == RMC_EINVAL, "negative T");
  check(rmc_line_quantities(nullptr, 1e4, q) == RMC_EINVAL, "null line");
  check(rmc_abi_version() > 0, "abi version");
  std::printf("host driver: %d failures\n", failures);
  return failures ? 1 : 0;
}
