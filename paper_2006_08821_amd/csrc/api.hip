// C ABI of the device library (include/emu.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <random>
#include <string>
#include <thread>
#include <vector>

#include "mesh_impl.hpp"

namespace {

__global__ void k_to_user_q(const double* q, const int32_t* vold, int n, double* out) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int u = vold[v];
  out[3 * u] = q[3 * v];
  out[3 * u + 1] = q[3 * v + 1];
  out[3 * u + 2] = q[3 * v + 2];
}
__global__ void k_from_user_q(const double* in, const int32_t* vold, int n, double* q) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int u = vold[v];
  q[3 * v] = in[3 * u];
  q[3 * v + 1] = in[3 * u + 1];
  q[3 * v + 2] = in[3 * u + 2];
}

}  // namespace

namespace {

emu_status fail_with(const emu::Error& e) {
  emu::set_error(e.msg);
  return e.code;
}

void modes_layout(const emu::HostMesh& hm, std::vector<double>& phi, std::vector<double>& nu) {
  phi.assign((size_t)emu::kMaxK1 * hm.n, 0.0);
  nu.assign(emu::kMaxK1, 1.0);
  if ((int)hm.nu.size() < hm.k1) return;  // modes not computed yet (device eigenpairs follow)
  for (int j = 0; j < hm.k1; ++j) {
    nu[j] = hm.nu[j];
    for (int32_t f = 0; f < hm.nf; ++f) phi[(size_t)emu::kMaxK1 * f + j] = hm.phi[(size_t)j * hm.nf + f];
  }
}

void upload_modes(emu_mesh* M) {
  std::vector<double> phi, nu;
  modes_layout(M->hm, phi, nu);
  HIPCHK(hipMemcpy((void*)M->d.phi, phi.data(), phi.size() * 8, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy((void*)M->d.nu, nu.data(), nu.size() * 8, hipMemcpyHostToDevice));
}

// Device memory for the duration of one call (the caller's allocator when
// it has one), released after the mesh's stream has drained.
struct TmpDev {
  emu_mesh* M;
  double* p = nullptr;
  TmpDev(emu_mesh* m, size_t count) : M(m) {
    const size_t nb = std::max<size_t>(1, count) * sizeof(double);
    if (M->dev_alloc) p = (double*)M->dev_alloc(nb, M->alloc_ctx);
    else if (hipMalloc((void**)&p, nb) != hipSuccess) p = nullptr;
    if (!p) throw emu::Error{EMU_E_OOM, "device allocation of the eigen work arrays failed"};
  }
  ~TmpDev() {
    (void)hipStreamSynchronize(M->st);
    if (M->dev_free) M->dev_free(p, M->alloc_ctx);
    else (void)hipFree(p);
  }
  TmpDev(const TmpDev&) = delete;
  TmpDev& operator=(const TmpDev&) = delete;
};

// Upper-triangular R with R^T R = G (kEigCols square, row-major) and its
// inverse; false if G is not numerically positive definite.
bool chol_upper_inverse(const std::vector<double>& G, std::vector<double>& Rinv) {
  constexpr int B = emu::kEigCols;
  std::vector<double> R((size_t)B * B, 0.0);
  double dmax = 0;
  for (int i = 0; i < B; ++i) dmax = std::max(dmax, G[(size_t)i * B + i]);
  for (int i = 0; i < B; ++i) {
    double s = G[(size_t)i * B + i];
    for (int k = 0; k < i; ++k) s -= R[(size_t)k * B + i] * R[(size_t)k * B + i];
    if (!(s > 1e-13 * dmax)) return false;
    const double rii = std::sqrt(s);
    R[(size_t)i * B + i] = rii;
    for (int j = i + 1; j < B; ++j) {
      double t = 0.5 * (G[(size_t)i * B + j] + G[(size_t)j * B + i]);
      for (int k = 0; k < i; ++k) t -= R[(size_t)k * B + i] * R[(size_t)k * B + j];
      R[(size_t)i * B + j] = t / rii;
    }
  }
  Rinv.assign((size_t)B * B, 0.0);
  for (int j = 0; j < B; ++j) {  // column j of R^{-1}: back substitution
    for (int i = j; i >= 0; --i) {
      double t = i == j ? 1.0 : 0.0;
      for (int k = i + 1; k <= j; ++k) t -= R[(size_t)i * B + k] * Rinv[(size_t)k * B + j];
      Rinv[(size_t)i * B + j] = t / R[(size_t)i * B + i];
    }
  }
  return true;
}

// The lowest k1 eigenpairs of L_ff (eq. low-rank) on the device: block
// inverse subspace iteration on kEigCols vectors (CholQR2 after each solve
// with the factor), Rayleigh-Ritz with L_ff each step, stopped at the host
// solver's test (relative residual <= 1e-8 for the k1 lowest pairs); then the
// host's sign and normalization, and the captured fraction of trace(L_ff^-1)
// from nine probes.  false (nothing written) if the mesh is too small for the
// block or the iteration does not reach the test.
bool device_modes(emu_mesh* M) {
  emu::Range range("emu device eigenpairs");
  auto& hm = M->hm;
  const emu::DevMesh& d = M->d;
  constexpr int B = emu::kEigCols, NP = B / 3;
  const int k1 = hm.k1, nf = hm.nf;
  if (k1 == 0) return true;
  if (nf < 4 * B) return false;
  hipStream_t st = M->st;
  const int64_t ps = 3 * (int64_t)hm.n;
  const int nblk = std::max(emu::eig_gram_blocks(nf), (nf + 255) / 256);
  const size_t nd = 3 * (size_t)NP * ps + 9 * (size_t)hm.m + (size_t)nblk * B * B + 2 * (size_t)B * B + B;
  TmpDev tmp(M, nd);
  double* X = tmp.p;
  double* Y = X + NP * ps;
  double* LX = Y + NP * ps;
  double* V = LX + NP * ps;
  double* part = V + 9 * (size_t)hm.m;
  double* W = part + (size_t)nblk * B * B;
  double* out = W + (size_t)B * B;
  double* lam = out + (size_t)B * B;
  HIPCHK(hipMemsetAsync(X, 0, 8 * 3 * (size_t)NP * ps, st));
  {
    std::vector<double> h((size_t)NP * ps, 0.0);
    std::mt19937_64 rng(20200615ULL);
    std::normal_distribution<double> nd01(0.0, 1.0);
    for (int c = 0; c < B; ++c)
      for (int i = 0; i < nf; ++i) h[(c / 3) * ps + 3 * (int64_t)i + c % 3] = nd01(rng);
    HIPCHK(hipMemcpyAsync(X, h.data(), 8 * h.size(), hipMemcpyHostToDevice, st));
  }
  std::vector<double> G, Rinv, T((size_t)B * B), Wv((size_t)B * B), ev(B), r(B);
  auto fetch = [&](size_t count, double* dst) {
    HIPCHK(hipMemcpyAsync(dst, out, 8 * count, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
  };
  auto cholqr = [&](const double* src, double* dst) {
    G.resize((size_t)B * B);
    emu::launch_eig_gram(nf, ps, src, src, part, out, st);
    fetch(G.size(), G.data());
    if (!chol_upper_inverse(G, Rinv)) return false;
    HIPCHK(hipMemcpyAsync(W, Rinv.data(), 8 * Rinv.size(), hipMemcpyHostToDevice, st));
    emu::launch_eig_mul(nf, ps, src, W, dst, st);
    return true;
  };
  if (!cholqr(X, Y) || !cholqr(Y, X)) return false;
  bool conv = false;
  for (int it = 0; it < 300 && !conv; ++it) {
    for (int p = 0; p < NP; ++p) {  // Y = L_ff^{-1} X
      HIPCHK(hipMemcpyAsync(d.rhs, X + p * ps, 24 * (size_t)nf, hipMemcpyDeviceToDevice, st));
      emu::launch_sweeps(d, M->plan, Y + p * ps, st);
    }
    if (!cholqr(Y, X) || !cholqr(X, Y)) return false;  // orthonormal basis in Y
    for (int p = 0; p < NP; ++p) {                       // LX = L_ff Y
      emu::launch_lff_apply(d, Y + p * ps, V, st);
      HIPCHK(hipMemcpyAsync(LX + p * ps, d.rhs, 24 * (size_t)nf, hipMemcpyDeviceToDevice, st));
    }
    emu::launch_eig_gram(nf, ps, Y, LX, part, out, st);  // Rayleigh-Ritz
    fetch(T.size(), T.data());
    for (int a = 0; a < B; ++a)
      for (int c = 0; c < a; ++c) T[(size_t)a * B + c] = T[(size_t)c * B + a] = 0.5 * (T[(size_t)a * B + c] + T[(size_t)c * B + a]);
    emu::jacobi_eigh(B, T.data(), ev.data(), Wv.data());
    HIPCHK(hipMemcpyAsync(W, Wv.data(), 8 * Wv.size(), hipMemcpyHostToDevice, st));
    emu::launch_eig_mul(nf, ps, Y, W, X, st);  // Ritz vectors
    emu::launch_eig_mul(nf, ps, LX, W, Y, st);  // and L_ff times them
    HIPCHK(hipMemcpyAsync(lam, ev.data(), 8 * (size_t)B, hipMemcpyHostToDevice, st));
    emu::launch_eig_resid(nf, ps, X, Y, lam, k1, part, out, st);
    fetch((size_t)k1, r.data());
    double worst = 0;
    for (int j = 0; j < k1; ++j) worst = std::max(worst, std::sqrt(std::max(0.0, r[j])) / std::fabs(ev[j]));
    conv = worst < 1e-8;
  }
  if (!conv) return false;
  std::vector<double> h((size_t)NP * ps);
  HIPCHK(hipMemcpyAsync(h.data(), X, 8 * h.size(), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  hm.nu.assign(ev.begin(), ev.begin() + k1);
  hm.phi.assign((size_t)k1 * nf, 0.0);
  for (int j = 0; j < k1; ++j) {
    auto at = [&](int i) { return h[(j / 3) * ps + 3 * (int64_t)i + j % 3]; };
    int im = 0;
    double nn = 0;
    for (int i = 0; i < nf; ++i) {
      if (std::fabs(at(i)) > std::fabs(at(im))) im = i;
      nn += at(i) * at(i);
    }
    const double sg = (at(im) < 0 ? -1.0 : 1.0) / std::sqrt(nn);
    for (int i = 0; i < nf; ++i) hm.phi[(size_t)j * nf + i] = sg * at(i);
  }
  {
    // trace(L_ff^{-1}) from nine +-1 probes (three packs) for the captured fraction
    std::vector<double> z(3 * (size_t)ps, 0.0), zi(3 * (size_t)ps);
    std::mt19937_64 r2(7);
    for (int p = 0; p < 3; ++p)
      for (int64_t k = 0; k < 3 * (int64_t)nf; ++k) z[p * ps + k] = (r2() & 1) ? 1.0 : -1.0;
    HIPCHK(hipMemcpyAsync(X, z.data(), 8 * z.size(), hipMemcpyHostToDevice, st));
    for (int p = 0; p < 3; ++p) {
      HIPCHK(hipMemcpyAsync(d.rhs, X + p * ps, 24 * (size_t)nf, hipMemcpyDeviceToDevice, st));
      emu::launch_sweeps(d, M->plan, Y + p * ps, st);
    }
    HIPCHK(hipMemcpyAsync(zi.data(), Y, 8 * zi.size(), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    double tr = 0;
    for (size_t k = 0; k < z.size(); ++k) tr += z[k] * zi[k];
    tr /= 9.0;
    double capd = 0;
    for (int j = 0; j < k1; ++j) capd += 1.0 / hm.nu[j];
    hm.mode_captured = tr > 0 ? capd / tr : 0;
  }
  upload_modes(M);
  return true;
}

// Modes of a mesh whose image was uploaded without them: on the device, or
// by the host solver where the device iteration declines.
void ensure_modes(emu_mesh* M) {
  if ((int)M->hm.nu.size() == M->hm.k1) {
    upload_modes(M);
    return;
  }
  if (!device_modes(M)) {
    emu::host_modes(M->hm, M->hm.k1);
    upload_modes(M);
  }
}

void upload_pins(emu_mesh* M) {
  const auto& hm = M->hm;
  HIPCHK(hipMemcpy((void*)M->d.pin_rhs, hm.pin_rhs.data(), hm.pin_rhs.size() * 8, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy((void*)M->d.pin_xyz, hm.pin_xyz.data(), hm.pin_xyz.size() * 8, hipMemcpyHostToDevice));
}

// Collects the pieces of a DevImage (256-byte aligned offsets).
struct ImageBuilder {
  emu::DevImage& im;
  template <typename T>
  void put(size_t slot, const std::vector<T>& v) {
    add(slot, v.size() * sizeof(T), v.data());
  }
  void reserve(size_t slot, size_t bytes) { add(slot, bytes, nullptr); }
  void add(size_t slot, size_t bytes, const void* src) {
    emu::DevImage::Piece p;
    p.slot = slot;
    p.offset = im.total;
    p.bytes = std::max<size_t>(1, bytes);
    if (src && bytes) p.data.assign((const char*)src, (const char*)src + bytes);
    im.total += (p.bytes + 255) & ~(size_t)255;
    im.pieces.push_back(std::move(p));
  }
};
#define SLOT(f) offsetof(emu::DevMesh, f)

}  // namespace

std::shared_ptr<const emu::DevImage> emu::prepare_image(const emu::HostMesh& hm) {
  auto imp = std::make_shared<emu::DevImage>();
  emu::DevImage& im = *imp;
  ImageBuilder B{im};
  auto& d = im.d;
  const int32_t n = hm.n, m = hm.m, nf = hm.nf;
  const auto& fac = hm.fac;
  d.n = n;
  d.nf = nf;
  d.m = m;
  d.k1 = hm.k1;
  d.npins = hm.npins;
  d.ngroups = hm.ngroups;
  d.nb = std::max(1, std::min((m + emu::kBlock - 1) / emu::kBlock, 1024));
  // Gram workgroups: one round at two workgroups per compute unit (fewer
  // partial sums for the reduction that follows)
  d.nbg = std::max(1, std::min((m + 63) / 64, 512));
  d.mixed = hm.precision == EMU_PRECISION_MIXED;
  d.coupled = hm.hessian_blocks == EMU_BLOCKS_COUPLED;
  d.alpha = hm.alpha;
  d.kf = hm.kf;

  // element arrays in internal order (structure of arrays)
  std::vector<int32_t> vid(4 * (size_t)m);
  {
    std::vector<double> dminv(9 * (size_t)m), vol(m), mu(m), lhat(m), w(m), fib(3 * (size_t)m);
    std::vector<int32_t> grp(m);
    for (int32_t e = 0; e < m; ++e) {
      const int32_t o = hm.eold[e];
      for (int k = 0; k < 4; ++k) vid[(size_t)k * m + e] = hm.vnew[hm.tets[4 * (size_t)o + k]];
      for (int k = 0; k < 9; ++k) dminv[(size_t)k * m + e] = hm.dminv[9 * (size_t)o + k];
      vol[e] = hm.vol[o];
      mu[e] = hm.mu[o];
      lhat[e] = hm.lhat[o];
      w[e] = hm.w[o];
      for (int c = 0; c < 3; ++c) fib[(size_t)c * m + e] = hm.fiber[3 * (size_t)o + c];
      grp[e] = hm.group[o];
    }
    B.put(SLOT(vid), vid);
    B.put(SLOT(dminv), dminv);
    B.put(SLOT(vol), vol);
    B.put(SLOT(mu), mu);
    B.put(SLOT(lhat), lhat);
    B.put(SLOT(w), w);
    B.put(SLOT(fib), fib);
    B.put(SLOT(grp), grp);
  }
  const size_t tsz = d.mixed ? 4 : 8;
  B.reserve(SLOT(R), 72 * (size_t)m);
  B.reserve(SLOT(S), 48 * (size_t)m);
  B.reserve(SLOT(gbar), 9 * (size_t)m * tsz);
  B.reserve(SLOT(Lf), (d.coupled ? 33 : 27) * (size_t)m * tsz);
  B.put(SLOT(p), std::vector<double>(9 * (size_t)m, 0.0));
  B.reserve(SLOT(contrib), 96 * (size_t)m);
  {
    std::vector<double> zeros3(3 * (size_t)n, 0.0);
    B.put(SLOT(q), zeros3);
    B.put(SLOT(dq), zeros3);
    B.put(SLOT(uz), zeros3);
    std::vector<double> phi, nu;
    modes_layout(hm, phi, nu);
    B.put(SLOT(phi), phi);
    B.put(SLOT(nu), nu);
    std::vector<double> act(std::max(1, hm.ngroups), 0.0);
    B.put(SLOT(act), act);
    B.put(SLOT(vext), zeros3);
    B.put(SLOT(pin_rhs), hm.pin_rhs);
    B.put(SLOT(pin_xyz), hm.pin_xyz);
  }
  // incidence of free vertices (fixed element order)
  {
    std::vector<int32_t> cnt(nf + 1, 0);
    for (int32_t e = 0; e < m; ++e)
      for (int k = 0; k < 4; ++k) {
        int32_t v = vid[(size_t)k * m + e];
        if (v < nf) cnt[v + 1]++;
      }
    for (int32_t v = 0; v < nf; ++v) cnt[v + 1] += cnt[v];
    std::vector<int32_t> inc(cnt[nf]);
    std::vector<int32_t> pos(cnt.begin(), cnt.end() - 1);
    for (int32_t e = 0; e < m; ++e)
      for (int k = 0; k < 4; ++k) {
        int32_t v = vid[(size_t)k * m + e];
        if (v < nf) inc[pos[v]++] = 4 * e + k;
      }
    B.put(SLOT(inc_ptr), cnt);
    B.put(SLOT(inc), inc);
  }
  // factor and level schedule
  {
    // Slot rows of the children's contributions: supernode s with nch
    // children owns nch * h_s rows from slotbase[s]; child k (in child order)
    // adds its update row for parent front position p into row
    // slotbase[s] + k h_s + p.  Rows no child writes stay zero, so the parent
    // adds all nch rows of a position without an index load.
    std::vector<int32_t> slotbase(fac.ns + 1, 0);
    for (int s = 0; s < fac.ns; ++s)
      slotbase[s + 1] = slotbase[s] + (fac.child_ptr[s + 1] - fac.child_ptr[s]) * fac.h[s];
    std::vector<int32_t> dst(std::max<int32_t>(1, fac.rowoff[fac.ns]), 0);
    for (int s = 0; s < fac.ns; ++s) {
      const int w = fac.w[s], h = fac.h[s];
      const int32_t c0 = fac.col0[s];
      const int32_t* rs = fac.rows.data() + fac.rowoff[s];
      for (int k = fac.child_ptr[s]; k < fac.child_ptr[s + 1]; ++k) {
        const int c = fac.child_idx[k];
        const int hb = fac.h[c] - fac.w[c];
        for (int a = 0; a < hb; ++a) {
          const int32_t v = fac.rows[fac.rowoff[c] + a];
          int p = v < c0 + w ? v - c0 : w + (int)(std::lower_bound(rs, rs + (h - w), v) - rs);
          dst[fac.rowoff[c] + a] = slotbase[s] + (k - fac.child_ptr[s]) * h + p;
        }
      }
    }
    std::vector<emu::SweepItem> fwd, bwd;
    auto item = [&](int s, int first) {
      emu::SweepItem it;
      it.valoff = fac.valoff[s];
      it.first = first;
      it.w = fac.w[s];
      it.h = fac.h[s];
      it.col0 = fac.col0[s];
      it.slotbase = slotbase[s];
      it.nslot = fac.child_ptr[s + 1] - fac.child_ptr[s];
      it.end = 0;
      it.rowoff = fac.rowoff[s];
      return it;
    };
    auto& pl = im.plan;
    pl.nlevels = fac.nlevels;
    pl.fwd_ptr.assign(fac.nlevels + 1, 0);
    pl.bwd_ptr.assign(fac.nlevels + 1, 0);
    // Backward levels with few work items at 32 columns per item split the
    // supernodes with long rows into items of 8 (32 lanes per row) instead.
    // Forward items stay at 32 rows (each item assembles its frontal vector
    // from the children's updates, which narrower items would repeat) except
    // for wide root supernodes, whose few items would otherwise serialize.
    auto sparse_level = [&](int L, bool fwd_dir) {
      int64_t items = 0;
      for (int s = 0; s < fac.ns; ++s)
        if (fac.level[s] == L) items += ((fwd_dir ? fac.h[s] : fac.w[s]) + 31) / 32;
      return items < emu::kWideLevelItems;
    };
    // A level runs the narrow sweep variant when it has no wide items and its
    // vectors are short: forward, frontal vectors of at most kNarrowFwdW
    // entries; backward, at most kNarrowBwdH entries from an item's first
    // column.  Measured on the 1.5M-tet hinge limb, these levels gain from
    // the doubled occupancy; levels with longer rows lose to the variant's
    // smaller load window.
    pl.fwd_narrow.assign(fac.nlevels, 1);
    pl.bwd_narrow.assign(fac.nlevels, 1);
    pl.fwd_col.assign(fac.nlevels, 1);
    {
      std::vector<int64_t> col_items(fac.nlevels, 0);
      for (int s = 0; s < fac.ns; ++s) {
        col_items[fac.level[s]] += (fac.h[s] + emu::kColRows - 1) / emu::kColRows;
        if (fac.w[s] > emu::kColW || fac.parent[s] < 0) pl.fwd_col[fac.level[s]] = 0;
      }
      // EMU_FWD_COLUMN=0: never, =1: wherever the widths allow (both for
      // tests and tuning); otherwise levels with enough items
      const char* force = std::getenv("EMU_FWD_COLUMN");
      const int mode = force && force[0] == '0' ? 0 : (force && force[0] == '1' ? 1 : 2);
      for (int L = 0; L < fac.nlevels; ++L)
        if (mode == 0 || (mode == 2 && col_items[L] < emu::kColMinItems)) pl.fwd_col[L] = 0;
    }
    for (int L = 0; L < fac.nlevels; ++L) {
      const size_t n0 = fwd.size();
      for (int s = 0; s < fac.ns; ++s)
        if (fac.level[s] == L) {
          // rows further down need more of the frontal vector: heaviest first
          if (pl.fwd_col[L]) {
            for (int r = (fac.h[s] - 1) / emu::kColRows * emu::kColRows; r >= 0; r -= emu::kColRows)
              fwd.push_back(item(s, r | emu::kItemColBit));
            continue;
          }
          const bool wide = fac.parent[s] < 0 && fac.w[s] >= 256;
          if (wide || fac.w[s] > emu::kNarrowFwdW) pl.fwd_narrow[L] = 0;
          const int step = wide ? 8 : 32;
          for (int r = (fac.h[s] - 1) / step * step; r >= 0; r -= step)
            fwd.push_back(item(s, r | (wide ? emu::kItemWideBit : 0)));
        }
      if (pl.fwd_col[L]) {
        pl.fwd_narrow[L] = 0;
        for (size_t k = n0; k < fwd.size(); ++k) fwd[k].end = (int32_t)fwd.size();
      }
      pl.fwd_ptr[L + 1] = (int)fwd.size();
    }
    for (int L = fac.nlevels - 1, k = 0; L >= 0; --L, ++k) {
      const bool sparse = sparse_level(L, false);
      for (int s = 0; s < fac.ns; ++s)
        if (fac.level[s] == L) {
          const bool wide = sparse && fac.h[s] >= emu::kWideRowMin;
          if (wide || fac.h[s] > emu::kNarrowBwdH) pl.bwd_narrow[k] = 0;
          const int step = wide ? 8 : 32;
          for (int c = 0; c < fac.w[s]; c += step) bwd.push_back(item(s, c | (wide ? emu::kItemWideBit : 0)));
        }
      pl.bwd_ptr[k + 1] = (int)bwd.size();
    }
    B.put(SLOT(rows), fac.rows);
    B.put(SLOT(vals), fac.vals);
    {
      // transposed blocks for the backward sweep: row c holds column c of
      // [Linv; M] from row c down (entries r = c .. h-1)
      std::vector<double> tv(fac.vals.size());
      // in tiles of 64 rows (each column's 64 entries are written together
      // while the 64 source rows are read side by side), supernodes spread
      // over the host's threads, largest first
      auto transpose_sn = [&](int s) {
        const int64_t w = fac.w[s], h = fac.h[s];
        const double* A = fac.vals.data() + fac.valoff[s];
        double* T = tv.data() + fac.valoff[s];
        const int64_t tri = w * (w + 1) / 2;
        for (int64_t r0 = 0; r0 < h; r0 += 64) {
          const int64_t r1 = std::min(h, r0 + 64), cmax = std::min(w, r1);
          for (int64_t c = 0; c < cmax; ++c) {
            double* row = T + c * h - c * (c - 1) / 2 - c;  // row[r]: entry r >= c
            for (int64_t r = std::max(r0, c); r < r1; ++r)
              row[r] = r < w ? A[r * (r + 1) / 2 + c] : A[tri + (r - w) * w + c];
          }
        }
      };
      std::vector<int> order(fac.ns);
      for (int s = 0; s < fac.ns; ++s) order[s] = s;
      std::sort(order.begin(), order.end(), [&](int a, int b) {
        return (int64_t)fac.w[a] * fac.h[a] > (int64_t)fac.w[b] * fac.h[b];
      });
      std::atomic<int> next(0);
      auto worker = [&]() {
        for (int k; (k = next.fetch_add(1)) < fac.ns;) transpose_sn(order[k]);
      };
      const int nt = (int)std::min<unsigned>(16u, std::max(1u, std::thread::hardware_concurrency()));
      std::vector<std::thread> th;
      for (int t = 1; t < nt; ++t) th.emplace_back(worker);
      worker();
      for (auto& t : th) t.join();
      B.put(SLOT(tvals), tv);
    }
    B.put(SLOT(dst), dst);
    B.put(SLOT(fwd_items), fwd);
    B.put(SLOT(bwd_items), bwd);
    B.reserve(SLOT(rhs), 24 * (size_t)nf);
    B.reserve(SLOT(ybuf), 24 * (size_t)nf);
    B.reserve(SLOT(xbuf), 24 * (size_t)nf);
    B.put(SLOT(slots), std::vector<double>(3 * (size_t)std::max<int32_t>(1, slotbase[fac.ns]), 0.0));
  }
  // affine bones (Sec. 3.3): the tets of each bone in internal element order
  {
    std::vector<int32_t> ids;
    if (hm.affine_bones)
      for (int32_t o = 0; o < m; ++o)
        if (hm.bone[o] >= 0) ids.push_back(hm.bone[o]);
    std::sort(ids.begin(), ids.end());
    ids.erase(std::unique(ids.begin(), ids.end()), ids.end());
    d.nbones = (int32_t)ids.size();
    std::vector<int32_t> ptr(d.nbones + 1, 0), el, pos(m, -1);
    for (int b = 0; b < d.nbones; ++b) {
      for (int32_t e = 0; e < m; ++e)
        if (hm.bone[hm.eold[e]] == ids[b]) {
          pos[e] = (int32_t)el.size();
          el.push_back(e);
        }
      ptr[b + 1] = (int32_t)el.size();
    }
    d.nbt = (int32_t)el.size();
    if (el.empty()) el.push_back(0);
    B.put(SLOT(bone_ptr), ptr);
    B.put(SLOT(bone_el), el);
    B.put(SLOT(bone_pos), pos);
    B.reserve(SLOT(bone_gbuf), 72 * (size_t)std::max(1, d.nbt));
  }
  const size_t nparts = (size_t)d.nb + d.nbones;
  B.reserve(SLOT(part_e), 16 * nparts);
  B.reserve(SLOT(part_g), 16 * nparts);
  B.reserve(SLOT(part_cnt), 8 * nparts);
  B.reserve(SLOT(part_gram), 8 * (size_t)emu::kGramEntries * ((size_t)d.nbg + d.nbones));
  B.reserve(SLOT(gram), 8 * (size_t)emu::kGramEntries);
  B.put(SLOT(zbuf), std::vector<double>(48, 0.0));
  B.reserve(SLOT(part_ls), 16 * (size_t)emu::kLsTerms * d.nb);
  B.reserve(SLOT(cfac), 8 * 48 * 48);
  B.reserve(SLOT(cfac_ok), 4);
  B.reserve(SLOT(ctl), sizeof(emu::Ctl));
  B.put(emu::DevImage::kSlotEold, hm.eold);
  B.put(emu::DevImage::kSlotVold, hm.vold);
  return imp;
}

void emu::upload_image(emu_mesh* M, std::shared_ptr<const emu::DevImage> img, hipStream_t stream) {
  HIPCHK(hipGetDevice(&M->device));
  if (stream) {
    M->st = stream;
    M->own_stream = false;
  } else {
    HIPCHK(hipStreamCreateWithFlags(&M->st, hipStreamNonBlocking));
    M->own_stream = true;
  }
  HIPCHK(hipEventCreateWithFlags(&M->ev_a, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&M->ev_b, hipEventDisableTiming));
  HIPCHK(hipEventCreate(&M->ev_t0));
  HIPCHK(hipEventCreate(&M->ev_t1));
  HIPCHK(hipHostMalloc((void**)&M->h_ctl, sizeof(emu::Ctl), hipHostMallocDefault));
  std::memset(M->h_ctl, 0, sizeof(emu::Ctl));
  char* base = M->dalloc<char>(img->total);
  M->d = img->d;
  M->plan = img->plan;
  for (const auto& p : img->pieces) {
    char* ptr = base + p.offset;
    if (p.slot == emu::DevImage::kSlotEold) M->d_eold = (int32_t*)ptr;
    else if (p.slot == emu::DevImage::kSlotVold) M->d_vold = (int32_t*)ptr;
    else std::memcpy((char*)&M->d + p.slot, &ptr, sizeof(ptr));
    if (!p.data.empty()) HIPCHK(hipMemcpyAsync(ptr, p.data.data(), p.data.size(), hipMemcpyHostToDevice, M->st));
  }
  M->act.assign(std::max(1, M->hm.ngroups), 0.0);
  M->img = std::move(img);
}

void emu::fresh_solve(emu_mesh* M) {
  emu::launch_scatter_F(M->d, M->st);
  emu::launch_solve(M->d, M->plan, 1, M->d.q, 0, M->st);
  emu::launch_set_pins(M->d, M->st);
}

void emu::init_ctl(emu_mesh* M, const emu_solve_opts& o, int eval_only) {
  emu::Ctl& c = *M->h_ctl;
  std::memset(&c, 0, sizeof(c));
  c.max_iters = o.max_iters;
  c.eval_only = eval_only;
  c.tol2 = o.grad_tol * o.grad_tol;
  c.rtol2 = o.grad_rtol * o.grad_rtol;
  c.gnorm0_2 = -1.0;
  c.sigma0 = o.sigma0;
  c.armijo_c = o.armijo_c;
  c.rho = o.rho;
  c.stall_rel = M->d.mixed ? o.stall_rel : 0.0;
  c.solves = 1;
  HIPCHK(hipMemcpyAsync(M->d.ctl, &c, sizeof(c), hipMemcpyHostToDevice, M->st));
}

namespace {

void read_ctl(emu_mesh* M) {
  HIPCHK(hipMemcpyAsync(M->h_ctl, M->d.ctl, sizeof(emu::Ctl), hipMemcpyDeviceToHost, M->st));
  HIPCHK(hipStreamSynchronize(M->st));
}

void ensure_graph(emu_mesh* M, int iters) {
  if (M->gexec && M->graph_iters == iters) return;
  if (M->gexec) HIPCHK(hipGraphExecDestroy(M->gexec));
  if (M->graph) HIPCHK(hipGraphDestroy(M->graph));
  M->gexec = nullptr;
  M->graph = nullptr;
  HIPCHK(hipStreamBeginCapture(M->st, hipStreamCaptureModeThreadLocal));
  for (int k = 0; k < iters; ++k) emu::launch_iteration(M->d, M->plan, M->st);
  HIPCHK(hipStreamEndCapture(M->st, &M->graph));
  HIPCHK(hipGraphInstantiate(&M->gexec, M->graph, nullptr, nullptr, 0));
  M->graph_iters = iters;
}

void join_user_stream(emu_mesh* M, void* stream) {
  HIPCHK(hipEventRecord(M->ev_a, (hipStream_t)stream));
  HIPCHK(hipStreamWaitEvent(M->st, M->ev_a, 0));
}
void release_user_stream(emu_mesh* M, void* stream) {
  HIPCHK(hipEventRecord(M->ev_b, M->st));
  HIPCHK(hipStreamWaitEvent((hipStream_t)stream, M->ev_b, 0));
}

}  // namespace

void emu::fill_stats(const emu::Ctl& c, emu_solve_stats* s, float ms) {
  if (!s) return;
  std::memset(s, 0, sizeof(*s));
  s->status = c.status;
  s->iters = c.iter;
  s->ls_trials = c.trials;
  s->acap_solves = c.solves;
  s->inverted = c.inverted;
  s->clamped = c.clamped;
  s->energy = c.energy;
  s->grad_norm = std::sqrt(std::max(0.0, c.gnorm2));
  s->grad_norm0 = std::sqrt(std::max(0.0, c.gnorm0_2));
  s->ms_total = ms;
}

void emu::ensure_modes_of(emu_mesh* M) { ensure_modes(M); }

void emu::launch_to_user_q(emu_mesh* M, double* out) {
  hipLaunchKernelGGL(k_to_user_q, dim3((M->hm.n + 255) / 256), dim3(256), 0, M->st, M->d.q, M->d_vold, M->hm.n,
                     out);
}

namespace {

void update_ext_constant(emu_mesh* M) {
  double c = 0;
  for (size_t k = 0; k < M->vext.size(); ++k) c += M->vext[k] * M->hm.pin_rhs[k];
  M->ext_c0 = c;
}

void drop_graph(emu_mesh* M) {  // kernels take the mesh by value: rebuild the graph
  if (M->gexec) {
    HIPCHK(hipGraphExecDestroy(M->gexec));
    HIPCHK(hipGraphDestroy(M->graph));
    M->gexec = nullptr;
    M->graph = nullptr;
  }
}

void backup_state(emu_mesh* M) {
  const size_t m = M->hm.m, n = M->hm.n;
  if (!M->R_bak) {
    M->R_bak = M->dalloc<double>(9 * m);
    M->S_bak = M->dalloc<double>(6 * m);
    M->q_bak = M->dalloc<double>(3 * n);
  }
  HIPCHK(hipMemcpyAsync(M->R_bak, M->d.R, 72 * m, hipMemcpyDeviceToDevice, M->st));
  HIPCHK(hipMemcpyAsync(M->S_bak, M->d.S, 48 * m, hipMemcpyDeviceToDevice, M->st));
  HIPCHK(hipMemcpyAsync(M->q_bak, M->d.q, 24 * n, hipMemcpyDeviceToDevice, M->st));
}
void restore_state(emu_mesh* M) {
  const size_t m = M->hm.m, n = M->hm.n;
  HIPCHK(hipMemcpyAsync(M->d.R, M->R_bak, 72 * m, hipMemcpyDeviceToDevice, M->st));
  HIPCHK(hipMemcpyAsync(M->d.S, M->S_bak, 48 * m, hipMemcpyDeviceToDevice, M->st));
  HIPCHK(hipMemcpyAsync(M->d.q, M->q_bak, 24 * n, hipMemcpyDeviceToDevice, M->st));
}

}  // namespace

using emu::fresh_solve;
using emu::init_ctl;

extern "C" {

const char* emu_last_error(void) { return emu::last_error_str().c_str(); }

emu_solve_opts emu_solve_opts_default(void) {
  emu_solve_opts o;
  o.grad_tol = 1e-8;
  o.max_iters = 10000;
  o.sigma0 = 10.0;
  o.armijo_c = 1e-4;
  o.rho = 0.5;
  o.warm_start = 1;
  o.iters_per_sync = 16;
  o.stall_rel = 1e-6;
  o.grad_rtol = 0.0;
  o.phase_timing = 0;
  return o;
}

emu_status emu_create_mesh(const emu_mesh_desc* desc, emu_mesh** out) {
  if (!desc || !out) {
    emu::set_error("NULL argument");
    return EMU_E_INVALID;
  }
  *out = nullptr;
  emu_mesh* M = nullptr;
  try {
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0)
      throw emu::Error{EMU_E_HIP, "no HIP device available"};
    M = new emu_mesh(std::make_shared<emu::HostMesh>());
    M->dev_alloc = desc->dev_alloc;
    M->dev_free = desc->dev_free;
    M->alloc_ctx = desc->alloc_ctx;
    emu::Range range("emu_create_mesh");
    auto t0 = std::chrono::steady_clock::now();
    {
      emu::Range r2("emu host setup");
      emu::host_setup(*desc, M->hm, false);
    }
    emu::upload_image(M, emu::prepare_image(M->hm), nullptr);
    ensure_modes(M);
    emu::launch_init_rest(M->d, M->st);
    emu_solve_opts o = emu_solve_opts_default();
    init_ctl(M, o, 0);
    fresh_solve(M);
    HIPCHK(hipStreamSynchronize(M->st));
    HIPCHK(hipGetLastError());
    M->img.reset();  // the uploaded host copy is no longer needed
    M->hm.setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    *out = M;
    return EMU_OK;
  } catch (const emu::Error& e) {
    delete M;
    return fail_with(e);
  } catch (const std::bad_alloc&) {
    delete M;
    emu::set_error("host allocation failed");
    return EMU_E_OOM;
  }
}

emu_status emu_destroy_mesh(emu_mesh* mesh) {
  if (mesh) {
    (void)hipStreamSynchronize(mesh->st);
    delete mesh;
  }
  return EMU_OK;
}

emu_status emu_mesh_get_info(const emu_mesh* M, emu_mesh_info* info) {
  if (!M || !info) {
    emu::set_error("NULL argument");
    return EMU_E_INVALID;
  }
  const auto& hm = M->hm;
  std::memset(info, 0, sizeof(*info));
  info->n_vertices = hm.n;
  info->n_tets = hm.m;
  info->n_free = hm.nf;
  info->n_modes = 3 * hm.k1;
  info->n_supernodes = hm.fac.ns;
  info->n_levels = hm.fac.nlevels;
  info->factor_nnz = hm.fac.nnz();
  info->device_bytes = M->bytes;
  info->mu_ref = hm.mu_ref;
  info->alpha = hm.alpha;
  info->fiber_k = hm.kf;
  info->setup_ms = hm.setup_ms;
  info->mode_captured = hm.mode_captured;
  for (char c : M->plan.fwd_col) info->fwd_column_levels += c ? 1 : 0;
  return EMU_OK;
}

emu_status emu_set_activation(emu_mesh* M, const double* a) {
  if (!M || (!a && M->hm.ngroups > 0)) {
    emu::set_error("NULL argument");
    return EMU_E_INVALID;
  }
  try {
    for (int g = 0; g < M->hm.ngroups; ++g)
      if (!(a[g] >= 0.0) || !std::isfinite(a[g])) throw emu::Error{EMU_E_INVALID, "activations must be finite and >= 0"};
    for (int g = 0; g < M->hm.ngroups; ++g) M->act[g] = a[g];
    HIPCHK(hipMemcpyAsync((void*)M->d.act, M->act.data(), M->act.size() * 8, hipMemcpyHostToDevice, M->st));
    HIPCHK(hipStreamSynchronize(M->st));
    M->converged = false;
    return EMU_OK;
  } catch (const emu::Error& e) {
    return fail_with(e);
  }
}

emu_status emu_set_pin_targets(emu_mesh* M, const double* pin_xyz) {
  if (!M || !pin_xyz) {
    emu::set_error("NULL argument");
    return EMU_E_INVALID;
  }
  try {
    for (int i = 0; i < 3 * M->hm.npins; ++i)
      if (!std::isfinite(pin_xyz[i])) throw emu::Error{EMU_E_INVALID, "non-finite pin target"};
    M->hm.pin_xyz.assign(pin_xyz, pin_xyz + 3 * (size_t)M->hm.npins);
    emu::recompute_pin_rhs(M->hm);
    update_ext_constant(M);
    HIPCHK(hipStreamSynchronize(M->st));
    upload_pins(M);
    M->converged = false;
    return EMU_OK;
  } catch (const emu::Error& e) {
    return fail_with(e);
  }
}

emu_status emu_set_external_forces(emu_mesh* M, const double* f) {
  if (!M) {
    emu::set_error("NULL argument");
    return EMU_E_INVALID;
  }
  try {
    const auto& hm = M->hm;
    const int32_t n = hm.n, nf = hm.nf;
    if (!f) {
      M->vext.clear();
      M->ext_c0 = 0;
      HIPCHK(hipStreamSynchronize(M->st));
      HIPCHK(hipMemset((void*)M->d.vext, 0, 24 * (size_t)n));
      M->d.has_ext = 0;
      drop_graph(M);
      M->converged = false;
      return EMU_OK;
    }
    for (int64_t k = 0; k < 3 * (int64_t)n; ++k)
      if (!std::isfinite(f[k])) throw emu::Error{EMU_E_INVALID, "non-finite external force"};
    // v = L_ff^{-1} f_f in factor order (three right-hand sides)
    std::vector<double> b(3 * (size_t)nf), v(3 * (size_t)nf);
    for (int32_t i = 0; i < nf; ++i)
      for (int c = 0; c < 3; ++c) b[3 * (size_t)i + c] = f[3 * (size_t)hm.vold[i] + c];
    emu::host_factor_solve(hm.fac, 3, b.data(), v.data());
    M->vext = v;
    update_ext_constant(M);
    std::vector<double> full(3 * (size_t)n, 0.0);
    std::copy(v.begin(), v.end(), full.begin());
    HIPCHK(hipStreamSynchronize(M->st));
    HIPCHK(hipMemcpy((void*)M->d.vext, full.data(), full.size() * 8, hipMemcpyHostToDevice));
    M->d.has_ext = 1;
    drop_graph(M);
    M->converged = false;
    return EMU_OK;
  } catch (const emu::Error& e) {
    return fail_with(e);
  }
}

namespace {
// Work arrays of the contact rounds, carved from M->c_work.
struct ContactWork {
  double *x, *x2, *nu, *z, *zc, *scr, *ypart, *part, *fpart;
};
size_t contact_work_doubles(const emu_mesh* M) {
  const size_t n = M->hm.n, m = M->hm.m, nb = M->d.nb;
  return 6 * n + 36 * m + 50 * nb + (size_t)std::max(1, emu::contact_blocks(M->d));
}
ContactWork contact_carve(emu_mesh* M) {
  const size_t n = M->hm.n, m = M->hm.m, nb = M->d.nb;
  ContactWork w;
  double* p = M->c_work;
  w.x = p;
  p += 3 * n;
  w.x2 = p;
  p += 3 * n;
  w.nu = p;
  p += 9 * m;
  w.z = p;
  p += 9 * m;
  w.zc = p;
  p += 9 * m;
  w.scr = p;
  p += 9 * m;
  w.ypart = p;
  p += 48 * nb;
  w.part = p;
  p += 2 * nb;
  w.fpart = p;
  return w;
}
// Algorithm 1's contact rounds after one accepted step (q already holds
// q*(F + sigma P); the step itself is still pending in (R, S, p, sigma)).
void contact_rounds(emu_mesh* M) {
  emu::Range range("emu contact rounds");
  const emu::DevMesh& d = M->d;
  ContactWork w = contact_carve(M);
  const int nbv = std::max(1, emu::contact_blocks(d));
  int r = 0;
  for (; r < M->c_max_rounds; ++r) {
    emu::launch_contact_force(d, M->c_obs, M->c_np, M->c_ns, M->c_k, w.fpart, M->st);
    HIPCHK(hipMemcpyAsync(M->c_host, w.fpart, 8 * (size_t)nbv, hipMemcpyDeviceToHost, M->st));
    HIPCHK(hipStreamSynchronize(M->st));
    double f2 = 0;
    for (int b = 0; b < nbv; ++b) f2 += M->c_host[b];
    if (!(std::sqrt(f2) > M->c_tol)) break;
    if (r == 0) HIPCHK(hipMemsetAsync(w.zc, 0, 72 * (size_t)M->hm.m, M->st));
    emu::launch_sweeps(d, M->plan, w.x, M->st);                                // x = L_ff^{-1} f
    emu::launch_weighted_grad(d, w.x, w.nu, M->st);                            // nu = w G x
    emu::launch_precond(d, w.nu, w.z, w.ypart, w.part, w.scr, M->st);          // z = Htilde^{-1} nu
    emu::launch_field_solve(d, M->plan, w.z, w.x2, M->st);                     // x2 = L^{-1} G^T W z
    emu::launch_contact_accum(d, w.x2, w.z, w.zc, M->st);                      // q += x2, zc += z
  }
  if (r > 0) emu::launch_accept_contact(d, w.zc, M->st);
  HIPCHK(hipGetLastError());
  M->c_rounds += r;
}
}  // namespace

emu_status emu_set_contact(emu_mesh* M, const emu_contact_desc* c) {
  if (!M) {
    emu::set_error("NULL argument");
    return EMU_E_INVALID;
  }
  try {
    const int np = c ? c->n_planes : 0, ns = c ? c->n_spheres : 0;
    if (np < 0 || ns < 0 || np + ns > EMU_MAX_OBSTACLES)
      throw emu::Error{EMU_E_INVALID, "obstacle counts must be in [0, EMU_MAX_OBSTACLES]"};
    if (np + ns == 0) {
      M->c_np = M->c_ns = 0;
      return EMU_OK;
    }
    if (M->d.nbones > 0) throw emu::Error{EMU_E_INVALID, "contact is not available with affine bones"};
    if ((np > 0 && !c->planes) || (ns > 0 && !c->spheres)) throw emu::Error{EMU_E_INVALID, "NULL obstacle rows"};
    if (!(c->stiffness > 0) || !std::isfinite(c->stiffness)) throw emu::Error{EMU_E_INVALID, "stiffness must be > 0"};
    if (!(c->tol >= 0) || !std::isfinite(c->tol)) throw emu::Error{EMU_E_INVALID, "tol must be >= 0"};
    if (c->max_rounds < 1) throw emu::Error{EMU_E_INVALID, "max_rounds must be >= 1"};
    std::vector<double> rows(4 * (size_t)(np + ns));
    for (int o = 0; o < np; ++o) {
      const double* P = c->planes + 4 * o;
      for (int k = 0; k < 4; ++k)
        if (!std::isfinite(P[k])) throw emu::Error{EMU_E_INVALID, "non-finite plane"};
      if (std::abs(std::sqrt(P[0] * P[0] + P[1] * P[1] + P[2] * P[2]) - 1.0) > 1e-9)
        throw emu::Error{EMU_E_INVALID, "plane normals must have unit length"};
      std::copy(P, P + 4, rows.begin() + 4 * o);
    }
    for (int o = 0; o < ns; ++o) {
      const double* Q = c->spheres + 4 * o;
      for (int k = 0; k < 4; ++k)
        if (!std::isfinite(Q[k])) throw emu::Error{EMU_E_INVALID, "non-finite sphere"};
      if (!(Q[3] > 0)) throw emu::Error{EMU_E_INVALID, "sphere radii must be > 0"};
      std::copy(Q, Q + 4, rows.begin() + 4 * (np + o));
    }
    HIPCHK(hipStreamSynchronize(M->st));
    if (!M->c_obs) {
      M->c_obs = M->dalloc<double>(4 * (size_t)EMU_MAX_OBSTACLES);
      const size_t nw = contact_work_doubles(M);
      M->c_work = M->dalloc<double>(nw);
      HIPCHK(hipMemset(M->c_work, 0, 8 * nw));  // the pinned rows of x and x2 stay 0
      HIPCHK(hipHostMalloc((void**)&M->c_host, 8 * (size_t)std::max(1, emu::contact_blocks(M->d))));
    }
    HIPCHK(hipMemcpy(M->c_obs, rows.data(), 8 * rows.size(), hipMemcpyHostToDevice));
    M->c_np = np;
    M->c_ns = ns;
    M->c_k = c->stiffness;
    M->c_tol = c->tol;
    M->c_max_rounds = c->max_rounds;
    M->converged = false;
    return EMU_OK;
  } catch (const emu::Error& e) {
    return fail_with(e);
  }
}

emu_status emu_set_modes(emu_mesh* M, int32_t k1, const double* nu, const double* phi) {
  if (!M || (k1 > 0 && (!nu || !phi))) {
    emu::set_error("NULL argument");
    return EMU_E_INVALID;
  }
  try {
    auto& hm = M->hm;
    if (k1 < 0 || k1 > emu::kMaxK1 || k1 >= hm.nf) throw emu::Error{EMU_E_INVALID, "k1 out of range"};
    for (int j = 0; j < k1; ++j)
      if (!(nu[j] > 0) || !std::isfinite(nu[j])) throw emu::Error{EMU_E_INVALID, "mode eigenvalues must be > 0"};
    hm.k1 = k1;
    hm.nu.assign(nu, nu + k1);
    hm.phi.assign((size_t)k1 * hm.nf, 0.0);
    for (int j = 0; j < k1; ++j)
      for (int32_t f = 0; f < hm.nf; ++f) hm.phi[(size_t)j * hm.nf + f] = phi[(size_t)j * hm.n + hm.vold[f]];
    HIPCHK(hipStreamSynchronize(M->st));
    upload_modes(M);
    M->d.k1 = k1;
    if (M->gexec) {  // kernels take the mesh by value: rebuild the graph
      HIPCHK(hipGraphExecDestroy(M->gexec));
      HIPCHK(hipGraphDestroy(M->graph));
      M->gexec = nullptr;
      M->graph = nullptr;
    }
    return EMU_OK;
  } catch (const emu::Error& e) {
    return fail_with(e);
  }
}

emu_status emu_get_modes(const emu_mesh* M, double* nu, double* phi) {
  if (!M) {
    emu::set_error("NULL argument");
    return EMU_E_INVALID;
  }
  const auto& hm = M->hm;
  if (nu)
    for (int j = 0; j < hm.k1; ++j) nu[j] = hm.nu[j];
  if (phi) {
    std::memset(phi, 0, sizeof(double) * (size_t)hm.k1 * hm.n);
    for (int j = 0; j < hm.k1; ++j)
      for (int32_t f = 0; f < hm.nf; ++f) phi[(size_t)j * hm.n + hm.vold[f]] = hm.phi[(size_t)j * hm.nf + f];
  }
  return EMU_OK;
}

emu_status emu_solve(emu_mesh* M, const emu_solve_opts* opts, double* q_out, emu_solve_stats* stats,
                     void* stream) {
  if (!M) {
    emu::set_error("NULL argument");
    return EMU_E_INVALID;
  }
  try {
    emu::Range range("emu_solve");
    emu_solve_opts o = opts ? *opts : emu_solve_opts_default();
    if (!(o.grad_tol >= 0) || o.max_iters < 0 || !(o.sigma0 > 0) || !(o.rho > 0 && o.rho < 1) ||
        !(o.armijo_c > 0 && o.armijo_c < 1))
      throw emu::Error{EMU_E_INVALID, "invalid solve options"};
    const int per = o.iters_per_sync > 0 ? std::min(o.iters_per_sync, 256) : 16;
    join_user_stream(M, stream);
    HIPCHK(hipEventRecord(M->ev_t0, M->st));
    if (!o.warm_start) emu::launch_init_rest(M->d, M->st);
    init_ctl(M, o, 0);
    fresh_solve(M);
    M->c_rounds = 0;
    const int max_launch = o.max_iters / per + 2;
    double phase_ms[4] = {0, 0, 0, 0};
    if (o.phase_timing && M->c_np + M->c_ns == 0) {
      // the same kernels launched one by one, with events between the phases
      if ((int)M->t_ev.size() < 5 * per) {
        const size_t have = M->t_ev.size();
        M->t_ev.resize(5 * (size_t)per, nullptr);
        for (size_t k = have; k < M->t_ev.size(); ++k) HIPCHK(hipEventCreate(&M->t_ev[k]));
      }
      for (int k = 0; k < max_launch; ++k) {
        for (int it = 0; it < per; ++it) emu::launch_iteration_phased(M->d, M->plan, M->st, &M->t_ev[5 * (size_t)it]);
        read_ctl(M);
        for (int it = 0; it < per; ++it)
          for (int ph = 0; ph < 4; ++ph) {
            float ms = 0;
            HIPCHK(hipEventElapsedTime(&ms, M->t_ev[5 * (size_t)it + ph], M->t_ev[5 * (size_t)it + ph + 1]));
            phase_ms[ph] += ms;
          }
        if (M->h_ctl->done) break;
      }
    } else if (M->c_np + M->c_ns > 0) {
      // contact: the rounds follow every accepted step (one iteration per launch)
      ensure_graph(M, 1);
      for (int k = 0; k < o.max_iters + 2; ++k) {
        HIPCHK(hipGraphLaunch(M->gexec, M->st));
        read_ctl(M);
        if (M->h_ctl->done) break;
        contact_rounds(M);
      }
    } else {
      ensure_graph(M, per);
      for (int k = 0; k < max_launch; ++k) {
        HIPCHK(hipGraphLaunch(M->gexec, M->st));
        read_ctl(M);
        if (M->h_ctl->done) break;
      }
    }
    if (!M->h_ctl->done) {
      // the iteration cap was reached between two checks
      M->h_ctl->status = EMU_E_NOT_CONVERGED;
    }
    if (q_out) {
      hipLaunchKernelGGL(k_to_user_q, dim3((M->hm.n + 255) / 256), dim3(256), 0, M->st, M->d.q, M->d_vold,
                         M->hm.n, q_out);
    }
    HIPCHK(hipEventRecord(M->ev_t1, M->st));
    HIPCHK(hipEventSynchronize(M->ev_t1));
    HIPCHK(hipGetLastError());
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, M->ev_t0, M->ev_t1));
    emu::fill_stats(*M->h_ctl, stats, ms);
    if (stats) {
      stats->energy -= M->ext_c0;
      stats->contact_rounds = M->c_rounds;
      stats->ms_elem = phase_ms[0];
      stats->ms_woodbury = phase_ms[1];
      stats->ms_solve = phase_ms[2];
      stats->ms_linesearch = phase_ms[3];
    }
    release_user_stream(M, stream);
    emu_status st = (emu_status)M->h_ctl->status;
    M->converged = st == EMU_OK;
    if (st != EMU_OK)
      emu::set_error(st == EMU_E_NOT_CONVERGED ? "max_iters reached"
                     : st == EMU_E_LINESEARCH  ? "line search found no Armijo step"
                                               : "non-finite value in the iteration");
    return st;
  } catch (const emu::Error& e) {
    return fail_with(e);
  }
}

emu_status emu_get_state(const emu_mesh* Mc, double* F, double* q, void* stream) {
  emu_mesh* M = const_cast<emu_mesh*>(Mc);
  if (!M) {
    emu::set_error("NULL argument");
    return EMU_E_INVALID;
  }
  try {
    join_user_stream(M, stream);
    if (F) emu::launch_get_F(M->d, F, M->d_eold, M->st);
    if (q)
      hipLaunchKernelGGL(k_to_user_q, dim3((M->hm.n + 255) / 256), dim3(256), 0, M->st, M->d.q, M->d_vold,
                         M->hm.n, q);
    HIPCHK(hipGetLastError());
    release_user_stream(M, stream);
    return EMU_OK;
  } catch (const emu::Error& e) {
    return fail_with(e);
  }
}

emu_status emu_set_state(emu_mesh* M, const double* F, void* stream) {
  if (!M || !F) {
    emu::set_error("NULL argument");
    return EMU_E_INVALID;
  }
  try {
    join_user_stream(M, stream);
    emu::launch_set_F(M->d, F, M->d_eold, M->st);
    emu::launch_bone_sync(M->d, M->st);
    fresh_solve(M);
    HIPCHK(hipGetLastError());
    release_user_stream(M, stream);
    M->converged = false;
    return EMU_OK;
  } catch (const emu::Error& e) {
    return fail_with(e);
  }
}

emu_status emu_evaluate(emu_mesh* M, const double* F, double* q, double* energy, double* grad_norm,
                        double* direction, void* stream) {
  if (!M || !F) {
    emu::set_error("NULL argument");
    return EMU_E_INVALID;
  }
  emu::Range range("emu_evaluate");
  try {
    join_user_stream(M, stream);
    backup_state(M);
    emu::launch_set_F(M->d, F, M->d_eold, M->st);
    emu::launch_bone_sync(M->d, M->st);
    emu_solve_opts o = emu_solve_opts_default();
    init_ctl(M, o, 1);
    fresh_solve(M);
    emu::launch_evaluate(M->d, M->st);
    if (q)
      hipLaunchKernelGGL(k_to_user_q, dim3((M->hm.n + 255) / 256), dim3(256), 0, M->st, M->d.q, M->d_vold,
                         M->hm.n, q);
    if (direction) emu::launch_get_dir(M->d, direction, M->d_eold, M->st);
    read_ctl(M);
    restore_state(M);
    HIPCHK(hipStreamSynchronize(M->st));
    HIPCHK(hipGetLastError());
    release_user_stream(M, stream);
    if (energy) *energy = M->h_ctl->energy - M->ext_c0;
    if (grad_norm) *grad_norm = std::sqrt(std::max(0.0, M->h_ctl->gnorm2));
    return EMU_OK;
  } catch (const emu::Error& e) {
    return fail_with(e);
  }
}

const char* emu_kernel_name(int32_t k) {
  static const char* names[EMU_NUM_KERNELS] = {"element", "gram", "gram_reduce", "control_a", "uz", "direction",
                                               "rhs", "fwd_sweep", "bwd_sweep", "lscoef", "control_b", "add_q"};
  return (k >= 0 && k < EMU_NUM_KERNELS) ? names[k] : nullptr;
}

emu_status emu_profile_kernels(emu_mesh* M, int32_t reps, double* ms_out, void* stream) {
  if (!M || !ms_out || reps <= 0) {
    emu::set_error("invalid argument");
    return EMU_E_INVALID;
  }
  try {
    join_user_stream(M, stream);
    backup_state(M);
    emu_solve_opts o = emu_solve_opts_default();
    o.max_iters = 1 << 30;
    std::vector<hipEvent_t> ev(2 * reps);
    for (auto& e : ev) HIPCHK(hipEventCreate(&e));
    for (int k = 0; k < EMU_NUM_KERNELS; ++k) {
      for (int r = 0; r < reps; ++r) {
        // the control block is copied from one pinned host buffer: let the
        // previous rep's copy finish before it is rewritten
        HIPCHK(hipStreamSynchronize(M->st));
        init_ctl(M, o, 1);
        // a tiny accepted step, so that the element pass times its accept path
        // (polar re-split) as it runs inside an iteration
        M->h_ctl->sigma = 1e-12;
        HIPCHK(hipMemcpyAsync(M->d.ctl, M->h_ctl, sizeof(emu::Ctl), hipMemcpyHostToDevice, M->st));
        HIPCHK(hipEventRecord(ev[2 * r], M->st));
        emu::launch_class(k, M->d, M->plan, M->st);
        HIPCHK(hipEventRecord(ev[2 * r + 1], M->st));
      }
      HIPCHK(hipStreamSynchronize(M->st));
      double tot = 0;
      for (int r = 0; r < reps; ++r) {
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, ev[2 * r], ev[2 * r + 1]));
        tot += ms;
      }
      ms_out[k] = tot / reps;
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
    restore_state(M);
    HIPCHK(hipStreamSynchronize(M->st));
    HIPCHK(hipGetLastError());
    release_user_stream(M, stream);
    return EMU_OK;
  } catch (const emu::Error& e) {
    return fail_with(e);
  }
}

}  // extern "C"

namespace {

// Device work arrays of the adjoint (F-space vectors [9][m], vertex vectors
// [n][3], partial sums) and their total size in doubles.
struct AdjWork {
  double *lam, *r, *z, *p, *hp, *ypart, *part, *vin, *vx, *el, *da;
};
size_t adj_work_doubles(const emu_mesh* M) {
  const size_t m = M->hm.m, n = M->hm.n, nb = M->d.nb, ng = std::max(1, M->hm.ngroups);
  return 5 * 9 * m + 48 * nb + 2 * nb + 2 * 3 * n + m + ng;
}
// Carve the work arrays out of one block of adj_work_doubles(M) doubles
// (each piece starts on a 256-byte boundary; the block is padded for that).
AdjWork adj_carve(const emu_mesh* M, double* base) {
  const size_t m = M->hm.m, n = M->hm.n, nb = M->d.nb, ng = std::max(1, M->hm.ngroups);
  size_t off = 0;
  auto take = [&](size_t count) {
    double* p = base + off;
    off += (count + 31) & ~(size_t)31;
    return p;
  };
  AdjWork w;
  w.lam = take(9 * m);
  w.r = take(9 * m);
  w.z = take(9 * m);
  w.p = take(9 * m);
  w.hp = take(9 * m);
  w.ypart = take(48 * nb);
  w.part = take(2 * nb);
  w.vin = take(3 * n);
  w.vx = take(3 * n);
  w.el = take(m);
  w.da = take(ng);
  return w;
}
size_t adj_block_doubles(const emu_mesh* M) { return adj_work_doubles(M) + 11 * 32; }

// The adjoint of the equilibrium (emu_solve_grad) with the given work arrays.
// Allocates nothing: every device buffer is either the mesh's or in `w`.
emu_status adjoint_run(emu_mesh* M, const AdjWork& w, const double* dL_dq, double* dL_da, emu_solve_stats* stats,
                       void* stream) {
  emu::Range range("emu adjoint");
  auto& d = M->d;
  const size_t m = M->hm.m, n = M->hm.n, nf = M->hm.nf;
  join_user_stream(M, stream);
  HIPCHK(hipEventRecord(M->ev_t0, M->st));
  // element blocks and the Woodbury factor at the converged state
  emu_solve_opts o = emu_solve_opts_default();
  init_ctl(M, o, 1);
  emu::launch_evaluate(d, M->st);
  // right-hand side b = W G L^{-1} (dL/dq)_f  (one ACAP solve); the rows of
  // pinned vertices in vx stay zero (the sweeps write free rows only)
  HIPCHK(hipMemsetAsync(w.vx, 0, 3 * n * 8, M->st));
  hipLaunchKernelGGL(k_from_user_q, dim3((n + 255) / 256), dim3(256), 0, M->st, dL_dq, M->d_vold, (int)n, w.vin);
  HIPCHK(hipMemcpyAsync(d.rhs, w.vin, 3 * nf * 8, hipMemcpyDeviceToDevice, M->st));
  emu::launch_sweeps(d, M->plan, w.vx, M->st);
  emu::launch_weighted_grad(d, w.vx, w.r, M->st);
  HIPCHK(hipMemsetAsync(w.lam, 0, 9 * m * 8, M->st));
  HIPCHK(hipMemsetAsync(w.hp, 0, 9 * m * 8, M->st));
  // preconditioned conjugate gradients on d2E/dF2 lam = b.  alpha, beta, r.z
  // and the stop test are computed on the device (k_cg_scalar); the host
  // launches kCgPerCheck steps at a time and then reads the stop flag, and the
  // steps after the stop return at once.
  constexpr int kMaxSteps = 20000, kCgPerCheck = 8;
  const emu::CgWork cw{w.lam, w.r, w.z, w.p, w.hp, w.ypart, w.part, w.vx, d.p};
  emu::launch_cg_begin(d, kMaxSteps, M->st);
  emu::launch_precond(d, w.r, w.z, w.ypart, w.part, d.p, M->st, 1);
  emu::launch_cg_scalar(d, w.part, emu::kCgInitRz, M->st);
  HIPCHK(hipMemcpyAsync(w.p, w.z, 9 * m * 8, hipMemcpyDeviceToDevice, M->st));
  // alpha = 0: the update only measures |b|^2
  emu::launch_cg_update(d, w.p, w.hp, w.lam, w.r, w.part, M->st);
  emu::launch_cg_scalar(d, w.part, emu::kCgInitR, M->st);
  for (int k = 0; k <= kMaxSteps / kCgPerCheck; ++k) {
    for (int j = 0; j < kCgPerCheck; ++j) emu::launch_cg_step(d, M->plan, cw, M->st);
    read_ctl(M);
    if (M->h_ctl->done) break;
  }
  const emu::Ctl& c = *M->h_ctl;
  const int it = c.cg_it;
  const double rnorm = c.cg_rnorm, bnorm = c.cg_bnorm;
  const int status = c.done ? c.status : EMU_E_NOT_CONVERGED;
  // dL/da_g = -2 kf sum_{i in g} vol (lam_i u).(F_i u)
  emu::launch_adj_da(d, w.lam, w.el, M->st);
  emu::launch_group_sum(d, w.el, -2.0 * M->hm.kf, w.da, M->st);
  if (M->hm.ngroups > 0)
    HIPCHK(hipMemcpyAsync(dL_da, w.da, (size_t)M->hm.ngroups * 8, hipMemcpyDeviceToHost, M->st));
  HIPCHK(hipEventRecord(M->ev_t1, M->st));
  HIPCHK(hipEventSynchronize(M->ev_t1));
  HIPCHK(hipGetLastError());
  float ms = 0;
  HIPCHK(hipEventElapsedTime(&ms, M->ev_t0, M->ev_t1));
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    stats->status = status;
    stats->iters = it;
    stats->acap_solves = it + 1;
    stats->grad_norm = rnorm;
    stats->grad_norm0 = bnorm;
    stats->ms_total = ms;
  }
  release_user_stream(M, stream);
  if (status == EMU_E_NONFINITE) emu::set_error("adjoint conjugate gradients: |b|, |r| or p.Hp not finite, or p.Hp <= 0");
  else if (status != EMU_OK) emu::set_error("adjoint conjugate gradients did not converge");
  return (emu_status)status;
}

emu_status adjoint_args_ok(const emu_mesh* M, const double* dL_dq, const double* dL_da) {
  if (!M || !dL_dq || (!dL_da && M->hm.ngroups > 0)) {
    emu::set_error("NULL argument");
    return EMU_E_INVALID;
  }
  if (M->d.nbones > 0) {
    emu::set_error("the adjoint does not support affine bones");
    return EMU_E_INVALID;
  }
  if (!M->converged) {
    emu::set_error("emu_solve_grad needs a converged emu_solve at the current activations");
    return EMU_E_STATE;
  }
  return EMU_OK;
}

// ---------------------------------------------------------------- scratch
// Fixed device scratch of the allocation-free adjoint entry point
// (emu_solve_grad_noalloc): kScratchDoubles doubles (48 MiB) per GPU, held
// until the process ends.  Host code never uses the symbol itself as an
// address: the per-device address comes from hipGetSymbolAddress.
constexpr size_t kScratchDoubles = (size_t)48 << 17;  // 48 MiB / 8 B
__device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxScratchDevices] = {};

// Device address of `scratch` on `device` (looked up once per device, with
// that device current).
double* scratch_on(int device) {
  if (device < 0 || device >= kMaxScratchDevices) throw emu::Error{EMU_E_INVALID, "device index out of range"};
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    int cur = 0;
    HIPCHK(hipGetDevice(&cur));
    if (cur != device) HIPCHK(hipSetDevice(device));
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != device) HIPCHK(hipSetDevice(cur));
    if (e != hipSuccess || !ptr)
      throw emu::Error{EMU_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)};
    g_scratch_ptr[device] = (double*)ptr;
  }
  return g_scratch_ptr[device];
}

}  // namespace

extern "C" {

emu_status emu_solve_grad(emu_mesh* M, const double* dL_dq, double* dL_da, emu_solve_stats* stats,
                          void* stream) {
  const emu_status ok = adjoint_args_ok(M, dL_dq, dL_da);
  if (ok != EMU_OK) return ok;
  try {
    if (!M->a_work) M->a_work = M->dalloc<double>(adj_block_doubles(M));
    return adjoint_run(M, adj_carve(M, M->a_work), dL_dq, dL_da, stats, stream);
  } catch (const emu::Error& e) {
    return fail_with(e);
  }
}

emu_status emu_solve_grad_noalloc(emu_mesh* M, const double* dL_dq, double* dL_da, emu_solve_stats* stats,
                                  void* stream) {
  if (M && adj_block_doubles(M) > kScratchDoubles) {
    emu::set_error("emu_solve_grad_noalloc: the mesh needs " + std::to_string(adj_block_doubles(M) * 8) +
                   " bytes of scratch, more than the fixed " + std::to_string(kScratchDoubles * 8) +
                   " (use emu_solve_grad)");
    return EMU_E_INVALID;
  }
  const emu_status ok = adjoint_args_ok(M, dL_dq, dL_da);
  if (ok != EMU_OK) return ok;
  try {
    return adjoint_run(M, adj_carve(M, scratch_on(M->device)), dL_dq, dL_da, stats, stream);
  } catch (const emu::Error& e) {
    return fail_with(e);
  }
}

}  // extern "C"
