// Host-only calls of libgb under the address / undefined-behaviour or thread sanitizer (CPU; no
// device is touched): the multilevel partitioner and its worker pool on a 3D lattice graph, the
// on-the-fly update, the pre-determined SP2 sequence and gap estimate, the Chebyshev
// coefficients and chemical potential, and the argument checks of the device entry points.
// Prints "ok" and exits 0 when every call returned what is expected.
#include <cmath>
#include <cstdio>
#include <algorithm>
#include <cstdlib>
#include <vector>

#include "../../include/gb.h"

#define CHECK(c)                                                         \
  do {                                                                   \
    if (!(c)) {                                                          \
      std::fprintf(stderr, "check failed: %s (line %d): %s\n", #c,      \
                   __LINE__, gb_last_error());                           \
      return 1;                                                          \
    }                                                                    \
  } while (0)

// symmetric CSR of an L^3 periodic lattice with the 26 nearest cells (self loops included)
static void lattice(int L, std::vector<int32_t>& rp, std::vector<int32_t>& col) {
  const int n = L * L * L;
  rp.assign(n + 1, 0);
  col.clear();
  for (int v = 0; v < n; ++v) {
    const int x = v % L, y = (v / L) % L, z = v / (L * L);
    std::vector<int32_t> nb;
    for (int dz = -1; dz <= 1; ++dz)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          const int u = ((x + dx + L) % L) + L * (((y + dy + L) % L) + L * ((z + dz + L) % L));
          nb.push_back(u);
        }
    std::sort(nb.begin(), nb.end());
    nb.erase(std::unique(nb.begin(), nb.end()), nb.end());
    col.insert(col.end(), nb.begin(), nb.end());
    rp[v + 1] = (int32_t)col.size();
  }
}

int main() {
  // multilevel communities (worker pool) twice, then carried to the same graph
  std::vector<int32_t> rp, col;
  lattice(24, rp, col);
  const int n = (int)rp.size() - 1;
  std::vector<int32_t> cp(n + 1), cv(n), cp2(n + 1), cv2(n);
  int32_t nc = 0, nc2 = 0;
  int64_t cost = 0, cost2 = 0;
  for (int rep = 0; rep < 2; ++rep) {
    CHECK(gb_partition_host(n, rp.data(), col.data(), 32, &nc, cp.data(), cv.data(), &cost) ==
          GB_OK);
    CHECK(nc > n / 32 - 1 && cp[nc] == n && cost > 0);
  }
  std::vector<int> seen(n, 0);
  for (int i = 0; i < n; ++i) seen[cv[i]]++;
  for (int i = 0; i < n; ++i) CHECK(seen[i] == 1);
  CHECK(gb_partition_update_host(n, rp.data(), col.data(), nc, cp.data(), cv.data(), &nc2,
                                 cp2.data(), cv2.data(), &cost2) == GB_OK);
  CHECK(nc2 == nc && cost2 == cost);
  CHECK(gb_partition_host(0, rp.data(), col.data(), 32, &nc, cp.data(), cv.data(), &cost) ==
        GB_EINVAL);
  CHECK(gb_partition_host(n, nullptr, col.data(), 32, &nc, cp.data(), cv.data(), &cost) ==
        GB_EINVAL);

  // pre-determined sequence and the gap estimate from its own traces (scalar model spectrum)
  uint8_t seq[127];
  int32_t len = 0;
  CHECK(gb_sp2_sequence(-3.0, 3.0, -0.2, 0.4, 1e-12, 127, seq, &len) == GB_OK && len > 10);
  CHECK(gb_sp2_sequence(-3.0, 3.0, 0.4, -0.2, 1e-12, 127, seq, &len) == GB_EINVAL);
  {
    // eigenvalues: 40 occupied at -1..-0.2 and 40 empty at 0.4..2 (X0 images), traces per step
    std::vector<double> x;
    for (int i = 0; i < 40; ++i) x.push_back((3.0 - (-1.0 + 0.8 * i / 39.0)) / 6.0);
    for (int i = 0; i < 40; ++i) x.push_back((3.0 - (0.4 + 1.6 * i / 39.0)) / 6.0);
    std::vector<double> t1, t2;
    for (int k = 0; k <= len; ++k) {
      double a = 0, b = 0;
      for (double v : x) {
        a += v;
        b += v * v;
      }
      t1.push_back(a);
      t2.push_back(b);
      if (k < len)
        for (double& v : x) v = seq[k] ? 2 * v - v * v : v * v;
    }
    gb_gap_estimate g;
    const gb_status st = gb_sp2_estimate_gap(t1.data(), t2.data(), seq, len, 40.0, -3.0, 3.0,
                                             0.0, &g);
    CHECK(st == GB_OK || st == GB_EINVAL);
    if (st == GB_OK) CHECK(g.homo_bound >= -0.2 - 1e-9 && g.lumo_bound <= 0.4 + 1e-9);
  }

  // Chebyshev coefficients of the Fermi function and the chemical potential from traces
  std::vector<double> c(201), tr(201);
  CHECK(gb_chebyshev_fermi(-3.0, 3.0, 5.0, 0.1, 200, 0, c.data()) == GB_OK);
  for (int k = 0; k <= 200; ++k) tr[k] = (k % 2 == 0) ? 100.0 / (1.0 + k) : 0.0;
  double mu = 0;
  const gb_status ms = gb_foe_solve_mu(tr.data(), 200, -3.0, 3.0, 5.0, 50.0, 0, &mu);
  CHECK(ms == GB_OK || ms == GB_EINVAL);
  CHECK(gb_chebyshev_fermi(3.0, -3.0, 5.0, 0.1, 200, 0, c.data()) == GB_EINVAL);

  // argument checks of device entry points fail before any device work
  gb_ell H{8, 3, (int32_t*)0x1000, (double*)0x1000}, D{8, 3, (int32_t*)0x1000, (double*)0x1000};
  CHECK(gb_density(nullptr, 4, 1e-5, nullptr, &D, nullptr, nullptr) == GB_EINVAL);
  CHECK(gb_density(&H, 9, 1e-5, nullptr, &D, nullptr, nullptr) == GB_EINVAL);
  CHECK(gb_density(&H, 4, -1.0, nullptr, &D, nullptr, nullptr) == GB_EINVAL);
  gb_sp2_opts o{};
  o.launch_mode = 9;
  CHECK(gb_density(&H, 4, 1e-5, &o, &D, nullptr, nullptr) == GB_EINVAL);
  size_t bytes = 1;
  CHECK(gb_density_workspace(&H, nullptr, &bytes) == GB_EINVAL && bytes == 0);
  CHECK(gb_spectral_bounds_noalloc(nullptr, nullptr, nullptr, nullptr) == GB_EINVAL);
  // the partitioner's host buffers are kept between calls until gb_trim releases them
  CHECK(gb_trim() == GB_OK);
  std::printf("ok\n");
  return 0;
}
