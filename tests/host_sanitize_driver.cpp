// Driver for the sanitizer test of the host C++ (tests/test_host_sanitizers.py):
// built with g++ -fsanitize=address,undefined together with host_setup.cpp
// and api_host.cpp, it runs the host-only API on a mesh read from a binary
// file, writes the results for comparison with the regular build, and feeds
// the validation a set of invalid descriptions.  Exit status 0 when every
// call returned what it should.
//
// Input file (native endianness): int32 n, m, n_groups, n_pins, n_modes,
// weight_mode, has_bone; float64 rest[n*3]; int32 tets[m*4]; float64
// youngs[m], poisson[m], fiber[m*3]; int32 group[m], pins[n_pins]; int32
// bone[m] if has_bone; float64 b[n*3] (right-hand side of the test solve).
// Output file: float64 x[n*3] (L_ff^-1 b), y[n*3] (L_w b), nu[k1],
// phi[k1*n], vol[m], w[m].
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../include/emu_host.h"

namespace emu {
const std::string& last_error_str();
}

template <typename T>
static bool rd(FILE* f, std::vector<T>& v, size_t n) {
  v.resize(n);
  return n == 0 || fread(v.data(), sizeof(T), n, f) == n;
}

int main(int argc, char** argv) {
  if (argc != 3) {
    fprintf(stderr, "usage: %s mesh.bin out.bin\n", argv[0]);
    return 2;
  }
  FILE* f = fopen(argv[1], "rb");
  if (!f) return 2;
  int32_t hdr[7];
  if (fread(hdr, 4, 7, f) != 7) return 2;
  const int n = hdr[0], m = hdr[1], ng = hdr[2], np = hdr[3], nm = hdr[4], wm = hdr[5], hb = hdr[6];
  std::vector<double> rest, youngs, poisson, fiber, b;
  std::vector<int32_t> tets, group, pins, bone;
  bool ok = rd(f, rest, 3 * (size_t)n) && rd(f, tets, 4 * (size_t)m) && rd(f, youngs, m) && rd(f, poisson, m) &&
            rd(f, fiber, 3 * (size_t)m) && rd(f, group, m) && rd(f, pins, np) && (!hb || rd(f, bone, m)) &&
            rd(f, b, 3 * (size_t)n);
  fclose(f);
  if (!ok) return 2;

  emu_mesh_desc d{};
  d.n_vertices = n;
  d.n_tets = m;
  d.n_groups = ng;
  d.n_pins = np;
  d.rest_xyz = rest.data();
  d.tets = tets.data();
  d.youngs = youngs.data();
  d.poisson = poisson.data();
  d.fiber = fiber.data();
  d.group = group.data();
  d.pins = pins.data();
  d.pin_xyz = nullptr;
  d.weight_mode = wm;
  d.n_modes = nm;
  d.bone = hb ? bone.data() : nullptr;

  int fails = 0;
  emu_host_setup* s = nullptr;
  if (emu_host_setup_create(&d, &s) != EMU_OK) {
    fprintf(stderr, "create failed: %s\n", emu::last_error_str().c_str());
    return 1;
  }
  emu_mesh_info info{};
  if (emu_host_setup_info(s, &info) != EMU_OK) ++fails;
  const int k1 = info.n_modes / 3;
  std::vector<double> x(3 * (size_t)n), y(3 * (size_t)n), nu(k1), phi((size_t)k1 * n), vol(m), w(m);
  std::vector<int32_t> ot(4 * (size_t)m);
  if (emu_host_setup_solve(s, b.data(), x.data()) != EMU_OK) ++fails;
  if (emu_host_setup_apply(s, b.data(), y.data()) != EMU_OK) ++fails;
  if (k1 > 0 && emu_host_setup_modes(s, nu.data(), phi.data()) != EMU_OK) ++fails;
  if (emu_host_setup_geometry(s, ot.data(), vol.data(), w.data()) != EMU_OK) ++fails;
  if (emu_host_setup_destroy(s) != EMU_OK) ++fails;

  // invalid descriptions: each must be rejected with EMU_E_INVALID
  auto expect_invalid = [&](emu_mesh_desc bad, const char* what) {
    emu_host_setup* t = nullptr;
    const emu_status c = emu_host_setup_create(&bad, &t);
    if (c != EMU_E_INVALID) {
      fprintf(stderr, "%s: status %d\n", what, (int)c);
      ++fails;
      if (t) emu_host_setup_destroy(t);
    }
  };
  {
    std::vector<int32_t> t2 = tets;
    t2[5] = n + 7;
    emu_mesh_desc e = d;
    e.tets = t2.data();
    expect_invalid(e, "vertex id out of range");
  }
  {
    std::vector<double> y2 = youngs;
    y2[m / 2] = std::nan("");
    emu_mesh_desc e = d;
    e.youngs = y2.data();
    expect_invalid(e, "NaN Young's modulus");
  }
  {
    std::vector<int32_t> g2 = group;
    g2[0] = ng + 3;
    emu_mesh_desc e = d;
    e.group = g2.data();
    expect_invalid(e, "group out of range");
  }
  {
    emu_mesh_desc e = d;
    e.n_modes = 4;
    expect_invalid(e, "n_modes not a multiple of 3");
  }
  {
    emu_mesh_desc e = d;
    e.n_pins = 0;
    expect_invalid(e, "no pins");
  }
  {
    std::vector<double> r2 = rest;
    for (int c = 0; c < 3; ++c) r2[3 * tets[4 * 3 + 1] + c] = r2[3 * tets[4 * 3] + c];  // a zero-volume tet
    emu_mesh_desc e = d;
    e.rest_xyz = r2.data();
    expect_invalid(e, "zero-volume tet");
  }

  FILE* o = fopen(argv[2], "wb");
  if (!o) return 2;
  fwrite(x.data(), 8, x.size(), o);
  fwrite(y.data(), 8, y.size(), o);
  fwrite(nu.data(), 8, nu.size(), o);
  fwrite(phi.data(), 8, phi.size(), o);
  fwrite(vol.data(), 8, vol.size(), o);
  fwrite(w.data(), 8, w.size(), o);
  fclose(o);
  printf("k1 %d fails %d\n", k1, fails);
  return fails == 0 ? 0 : 1;
}
