// Host-only C API (emu_host.h): the mesh setup without a device.
#include <cstring>
#include <new>

#include "../../include/emu_host.h"
#include "host_setup.hpp"

namespace emu {
const std::string& last_error_str();
}

struct emu_host_setup {
  emu::HostMesh hm;
};

extern "C" {

emu_status emu_host_setup_create(const emu_mesh_desc* desc, emu_host_setup** out) {
  if (!desc || !out) {
    emu::set_error("NULL argument");
    return EMU_E_INVALID;
  }
  *out = nullptr;
  try {
    auto* s = new emu_host_setup();
    try {
      emu::host_setup(*desc, s->hm, true);
    } catch (...) {
      delete s;
      throw;
    }
    *out = s;
    return EMU_OK;
  } catch (const emu::Error& e) {
    emu::set_error(e.msg);
    return e.code;
  } catch (const std::bad_alloc&) {
    emu::set_error("host allocation failed");
    return EMU_E_OOM;
  }
}

emu_status emu_host_setup_destroy(emu_host_setup* s) {
  delete s;
  return EMU_OK;
}

emu_status emu_host_setup_info(const emu_host_setup* s, emu_mesh_info* info) {
  if (!s || !info) return EMU_E_INVALID;
  const auto& hm = s->hm;
  std::memset(info, 0, sizeof(*info));
  info->n_vertices = hm.n;
  info->n_tets = hm.m;
  info->n_free = hm.nf;
  info->n_modes = 3 * hm.k1;
  info->n_supernodes = hm.fac.ns;
  info->n_levels = hm.fac.nlevels;
  info->factor_nnz = hm.fac.nnz();
  info->mu_ref = hm.mu_ref;
  info->alpha = hm.alpha;
  info->fiber_k = hm.kf;
  info->setup_ms = hm.setup_ms;
  info->mode_captured = hm.mode_captured;
  return EMU_OK;
}

emu_status emu_host_setup_solve(const emu_host_setup* s, const double* b, double* x) {
  if (!s || !b || !x) return EMU_E_INVALID;
  const auto& hm = s->hm;
  std::vector<double> bi(3 * (size_t)hm.nf), xi(3 * (size_t)hm.nf);
  for (int32_t f = 0; f < hm.nf; ++f)
    for (int c = 0; c < 3; ++c) bi[3 * f + c] = b[3 * (size_t)hm.vold[f] + c];
  emu::host_factor_solve(hm.fac, 3, bi.data(), xi.data());
  std::memset(x, 0, sizeof(double) * 3 * (size_t)hm.n);
  for (int32_t f = 0; f < hm.nf; ++f)
    for (int c = 0; c < 3; ++c) x[3 * (size_t)hm.vold[f] + c] = xi[3 * f + c];
  return EMU_OK;
}

emu_status emu_host_setup_apply(const emu_host_setup* s, const double* x, double* y) {
  if (!s || !x || !y) return EMU_E_INVALID;
  const auto& hm = s->hm;
  for (int32_t u = 0; u < hm.n; ++u) {
    double acc[3] = {0, 0, 0};
    for (int32_t k = hm.lap_ptr[u]; k < hm.lap_ptr[u + 1]; ++k)
      for (int c = 0; c < 3; ++c) acc[c] += hm.lap_val[k] * x[3 * (size_t)hm.lap_idx[k] + c];
    for (int c = 0; c < 3; ++c) y[3 * (size_t)u + c] = acc[c];
  }
  return EMU_OK;
}

emu_status emu_host_setup_modes(const emu_host_setup* s, double* nu, double* phi) {
  if (!s) return EMU_E_INVALID;
  const auto& hm = s->hm;
  if (nu)
    for (int j = 0; j < hm.k1; ++j) nu[j] = hm.nu[j];
  if (phi) {
    std::memset(phi, 0, sizeof(double) * (size_t)hm.k1 * hm.n);
    for (int j = 0; j < hm.k1; ++j)
      for (int32_t f = 0; f < hm.nf; ++f) phi[(size_t)j * hm.n + hm.vold[f]] = hm.phi[(size_t)j * hm.nf + f];
  }
  return EMU_OK;
}

emu_status emu_host_setup_geometry(const emu_host_setup* s, int32_t* tets, double* vol, double* w) {
  if (!s) return EMU_E_INVALID;
  const auto& hm = s->hm;
  if (tets) std::memcpy(tets, hm.tets.data(), sizeof(int32_t) * 4 * (size_t)hm.m);
  if (vol) std::memcpy(vol, hm.vol.data(), sizeof(double) * hm.m);
  if (w) std::memcpy(w, hm.w.data(), sizeof(double) * hm.m);
  return EMU_OK;
}

}  // extern "C"
