// Host-side setup: validation, geometry, ACAP weights, weighted Laplacian,
// nested-dissection ordering, supernodal multifrontal factorization in
// partitioned-inverse form, and the lowest eigenpairs of L_ff.
#include "host_setup.hpp"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <numeric>
#include <random>
#include <thread>

namespace emu {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }
const std::string& last_error_str() { return g_last_error; }

[[noreturn]] static void fail(emu_status c, const std::string& m) { throw Error{c, m}; }

static int n_threads() {
  unsigned h = std::thread::hardware_concurrency();
  if (h == 0) h = 4;
  return (int)std::min(16u, h);
}

// Run fn(i) for i in [0, n) on up to n_threads() threads (dynamic chunks).
static void parallel_for(int64_t n, const std::function<void(int64_t)>& fn, int64_t grain = 1) {
  int T = n_threads();
  if (n <= grain || T <= 1) {
    for (int64_t i = 0; i < n; ++i) fn(i);
    return;
  }
  std::atomic<int64_t> next(0);
  auto worker = [&]() {
    for (;;) {
      int64_t i0 = next.fetch_add(grain);
      if (i0 >= n) break;
      int64_t i1 = std::min(n, i0 + grain);
      for (int64_t i = i0; i < i1; ++i) fn(i);
    }
  };
  std::vector<std::thread> th;
  int nt = (int)std::min<int64_t>(T, (n + grain - 1) / grain);
  for (int t = 1; t < nt; ++t) th.emplace_back(worker);
  worker();
  for (auto& t : th) t.join();
}

// ------------------------------------------------------------------ geometry
static double det3(const double* a) {
  return a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6]) +
         a[2] * (a[3] * a[7] - a[4] * a[6]);
}

static void inv3(const double* a, double* o) {
  double d = det3(a);
  o[0] = (a[4] * a[8] - a[5] * a[7]) / d;
  o[1] = (a[2] * a[7] - a[1] * a[8]) / d;
  o[2] = (a[1] * a[5] - a[2] * a[4]) / d;
  o[3] = (a[5] * a[6] - a[3] * a[8]) / d;
  o[4] = (a[0] * a[8] - a[2] * a[6]) / d;
  o[5] = (a[2] * a[3] - a[0] * a[5]) / d;
  o[6] = (a[3] * a[7] - a[4] * a[6]) / d;
  o[7] = (a[1] * a[6] - a[0] * a[7]) / d;
  o[8] = (a[0] * a[4] - a[1] * a[3]) / d;
}

// D_m = [x1-x4 | x2-x4 | x3-x4] (columns)
static void dm_matrix(const double* rest, const int32_t* t, double* D) {
  for (int c = 0; c < 3; ++c)
    for (int j = 0; j < 3; ++j) D[3 * c + j] = rest[3 * t[j] + c] - rest[3 * t[3] + c];
}

static void validate(const emu_mesh_desc& d) {
  if (d.n_vertices <= 0) fail(EMU_E_INVALID, "n_vertices must be > 0");
  if (d.n_tets <= 0) fail(EMU_E_INVALID, "n_tets must be > 0");
  if (d.n_groups < 0) fail(EMU_E_INVALID, "n_groups must be >= 0");
  if (d.n_pins <= 0) fail(EMU_E_INVALID, "at least one pinned vertex is required");
  if (!d.rest_xyz || !d.tets || !d.youngs || !d.poisson || !d.group || !d.pins)
    fail(EMU_E_INVALID, "required array is NULL");
  if (d.n_groups > 0 && !d.fiber) fail(EMU_E_INVALID, "fiber is NULL");
  const int64_t n = d.n_vertices, m = d.n_tets;
  for (int64_t i = 0; i < 3 * n; ++i)
    if (!std::isfinite(d.rest_xyz[i])) fail(EMU_E_INVALID, "non-finite rest position");
  for (int64_t i = 0; i < 4 * m; ++i)
    if (d.tets[i] < 0 || d.tets[i] >= n) fail(EMU_E_INVALID, "tet vertex id out of range");
  for (int64_t i = 0; i < m; ++i) {
    const int32_t* t = d.tets + 4 * i;
    for (int a = 0; a < 4; ++a)
      for (int b = a + 1; b < 4; ++b)
        if (t[a] == t[b]) fail(EMU_E_INVALID, "tet with repeated vertex " + std::to_string(i));
    if (!(d.youngs[i] > 0) || !std::isfinite(d.youngs[i])) fail(EMU_E_INVALID, "youngs must be > 0");
    if (!(d.poisson[i] > -1.0 && d.poisson[i] < 0.5)) fail(EMU_E_INVALID, "poisson must be in (-1, 0.5)");
    if (d.group[i] < -1 || d.group[i] >= d.n_groups) fail(EMU_E_INVALID, "group id out of range");
    if (d.group[i] >= 0) {
      const double* u = d.fiber + 3 * i;
      double nn = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
      if (!std::isfinite(nn) || nn <= 0) fail(EMU_E_INVALID, "zero or non-finite fiber");
    }
  }
  std::vector<char> seen(n, 0);
  for (int i = 0; i < d.n_pins; ++i) {
    int p = d.pins[i];
    if (p < 0 || p >= n) fail(EMU_E_INVALID, "pin id out of range");
    if (seen[p]) fail(EMU_E_INVALID, "duplicate pin");
    seen[p] = 1;
    if (d.pin_xyz)
      for (int c = 0; c < 3; ++c)
        if (!std::isfinite(d.pin_xyz[3 * i + c])) fail(EMU_E_INVALID, "non-finite pin target");
  }
  if (!(d.alpha_hat >= 0) || !std::isfinite(d.alpha_hat)) fail(EMU_E_INVALID, "alpha_hat must be >= 0");
  int k = d.n_modes < 0 ? 48 : d.n_modes;
  if (k % 3 != 0 || k > 48) fail(EMU_E_INVALID, "n_modes must be a multiple of 3 in [0, 48]");
  if (d.weight_mode < 0 || d.weight_mode > 2) fail(EMU_E_INVALID, "weight_mode must be 0, 1 or 2");
  if (d.bone)
    for (int64_t i = 0; i < m; ++i)
      if (d.bone[i] < -1) fail(EMU_E_INVALID, "bone id must be >= -1");
  if ((d.dev_alloc == nullptr) != (d.dev_free == nullptr))
    fail(EMU_E_INVALID, "dev_alloc and dev_free must be given together");
  if (d.precision != 0 && d.precision != 1) fail(EMU_E_INVALID, "precision must be 0 or 1");
  if (d.hessian_blocks != 0 && d.hessian_blocks != 1) fail(EMU_E_INVALID, "hessian_blocks must be 0 or 1");
  if (d.affine_bones != 0 && d.affine_bones != 1) fail(EMU_E_INVALID, "affine_bones must be 0 or 1");
  if (!(d.bone_slack >= 0) || !std::isfinite(d.bone_slack)) fail(EMU_E_INVALID, "bone_slack must be >= 0");
  if (d.affine_bones && d.hessian_blocks != 0)
    fail(EMU_E_INVALID, "affine bones take the split element blocks");
  if (d.affine_bones && d.bone)
    for (int64_t i = 0; i < m; ++i)
      if (d.bone[i] >= 0 && d.group[i] >= 0) fail(EMU_E_INVALID, "affine bone tets must be passive (group -1)");
  if (d.leaf_size < 0) fail(EMU_E_INVALID, "leaf_size must be >= 0");
}

static void geometry(const emu_mesh_desc& d, HostMesh& hm) {
  const int32_t n = d.n_vertices, m = d.n_tets;
  hm.n = n;
  hm.m = m;
  hm.ngroups = d.n_groups;
  hm.npins = d.n_pins;
  hm.rest.assign(d.rest_xyz, d.rest_xyz + 3 * (int64_t)n);
  hm.tets.assign(d.tets, d.tets + 4 * (int64_t)m);
  hm.youngs.assign(d.youngs, d.youngs + m);
  hm.poisson.assign(d.poisson, d.poisson + m);
  hm.group.assign(d.group, d.group + m);
  if (d.bone) hm.bone.assign(d.bone, d.bone + m);
  else hm.bone.assign(m, -1);
  hm.pins.assign(d.pins, d.pins + d.n_pins);
  hm.fiber.assign(3 * (int64_t)m, 0.0);
  for (int32_t i = 0; i < m; ++i) {
    if (d.fiber) {
      const double* u = d.fiber + 3 * (int64_t)i;
      double nn = std::sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
      if (nn > 0 && std::isfinite(nn))
        for (int c = 0; c < 3; ++c) hm.fiber[3 * (int64_t)i + c] = u[c] / nn;
    }
  }
  hm.pin_xyz.resize(3 * (int64_t)d.n_pins);
  for (int i = 0; i < d.n_pins; ++i)
    for (int c = 0; c < 3; ++c)
      hm.pin_xyz[3 * i + c] = d.pin_xyz ? d.pin_xyz[3 * i + c] : hm.rest[3 * (int64_t)d.pins[i] + c];

  // bounding box edge scale for the degeneracy test
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int32_t v = 0; v < n; ++v)
    for (int c = 0; c < 3; ++c) {
      lo[c] = std::min(lo[c], hm.rest[3 * (int64_t)v + c]);
      hi[c] = std::max(hi[c], hm.rest[3 * (int64_t)v + c]);
    }
  hm.dminv.resize(9 * (int64_t)m);
  hm.vol.resize(m);
  std::atomic<int64_t> bad(-1);
  parallel_for(m, [&](int64_t i) {
    int32_t* t = hm.tets.data() + 4 * i;
    double D[9];
    dm_matrix(hm.rest.data(), t, D);
    double dt = det3(D);
    if (dt < 0) {  // orientation fix: swap local vertices 1 and 2
      std::swap(t[0], t[1]);
      dm_matrix(hm.rest.data(), t, D);
      dt = det3(D);
    }
    // degenerate if |det| is tiny relative to the cube of the longest edge
    double e2 = 0;
    for (int j = 0; j < 3; ++j) e2 = std::max(e2, D[j] * D[j] + D[3 + j] * D[3 + j] + D[6 + j] * D[6 + j]);
    if (!(dt > 1e-12 * e2 * std::sqrt(e2))) {
      bad = i;
      return;
    }
    inv3(D, hm.dminv.data() + 9 * i);
    hm.vol[i] = dt / 6.0;
  }, 1024);
  if (bad >= 0) fail(EMU_E_INVALID, "degenerate tet " + std::to_string((int64_t)bad));

  // materials: mu, lhat = lambda + mu
  hm.mu.resize(m);
  hm.lhat.resize(m);
  double mu_min_musc = 1e300, mu_min = 1e300;
  for (int32_t i = 0; i < m; ++i) {
    double E = hm.youngs[i], nu = hm.poisson[i];
    double mu = E / (2.0 * (1.0 + nu));
    double lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
    hm.mu[i] = mu;
    hm.lhat[i] = lam + mu;
    mu_min = std::min(mu_min, mu);
    if (hm.group[i] >= 0) mu_min_musc = std::min(mu_min_musc, mu);
  }
  hm.mu_ref = d.mu_ref > 0 ? d.mu_ref : (mu_min_musc < 1e300 ? mu_min_musc : mu_min);
  hm.kf = d.fiber_k > 0 ? d.fiber_k : hm.mu_ref;
  hm.alpha_hat = d.alpha_hat > 0 ? d.alpha_hat : 10.0;
  hm.alpha = hm.alpha_hat * hm.mu_ref;
  hm.weight_mode = d.weight_mode;
  hm.w.resize(m);
  hm.affine_bones = d.affine_bones;
  hm.bone_slack = d.bone_slack > 0 ? d.bone_slack : 1e-3;
  for (int32_t i = 0; i < m; ++i) {
    const bool stiff = d.weight_mode == EMU_WEIGHT_STIFFNESS || (d.weight_mode == EMU_WEIGHT_PAPER && hm.bone[i] < 0);
    hm.w[i] = stiff ? hm.vol[i] * hm.mu[i] / hm.mu_ref : hm.vol[i];
    // affine bones (Sec. 3.3): the bone constraint with slack eps_2 adds
    // |G_i q - F_b|^2 / (2 |eps_2|) per bone tet, relative to its
    // volume-weighted ACAP term; bones are not stiffness-weighted
    if (hm.affine_bones && hm.bone[i] >= 0) hm.w[i] = hm.vol[i] * (1.0 + 1.0 / hm.bone_slack);
  }
  hm.precision = d.precision;
  hm.hessian_blocks = d.hessian_blocks;
  hm.leaf_size = d.leaf_size > 0 ? d.leaf_size : 64;
  hm.k1 = (d.n_modes < 0 ? 48 : d.n_modes) / 3;
  hm.k1_default = d.n_modes < 0;
}

// hat gradients b_v (rows of D_m^{-1}, b_3 = -(b_0 + b_1 + b_2))
static inline void hat(const double* Dinv, double b[4][3]) {
  for (int v = 0; v < 3; ++v)
    for (int dd = 0; dd < 3; ++dd) b[v][dd] = Dinv[3 * v + dd];
  for (int dd = 0; dd < 3; ++dd) b[3][dd] = -(b[0][dd] + b[1][dd] + b[2][dd]);
}

static void laplacian(HostMesh& hm) {
  const int32_t n = hm.n, m = hm.m;
  // vertex -> incident elements
  std::vector<int32_t> cnt(n + 1, 0);
  for (int64_t i = 0; i < 4 * (int64_t)m; ++i) cnt[hm.tets[i] + 1]++;
  for (int32_t v = 0; v < n; ++v) cnt[v + 1] += cnt[v];
  std::vector<int32_t> inc(4 * (int64_t)m);
  {
    std::vector<int32_t> pos(cnt.begin(), cnt.end() - 1);
    for (int32_t i = 0; i < m; ++i)
      for (int a = 0; a < 4; ++a) inc[pos[hm.tets[4 * (int64_t)i + a]]++] = 4 * i + a;
  }
  hm.lap_ptr.assign(n + 1, 0);
  std::vector<std::vector<std::pair<int32_t, double>>> rowsv(n);
  parallel_for(n, [&](int64_t v) {
    std::vector<std::pair<int32_t, double>> acc;
    for (int32_t k = cnt[v]; k < cnt[v + 1]; ++k) {
      int32_t e = inc[k] >> 2, a = inc[k] & 3;
      double b[4][3];
      hat(hm.dminv.data() + 9 * (int64_t)e, b);
      for (int c = 0; c < 4; ++c) {
        double s = b[a][0] * b[c][0] + b[a][1] * b[c][1] + b[a][2] * b[c][2];
        acc.emplace_back(hm.tets[4 * (int64_t)e + c], hm.w[e] * s);
      }
    }
    std::stable_sort(acc.begin(), acc.end(),
                     [](const std::pair<int32_t, double>& x, const std::pair<int32_t, double>& y) {
                       return x.first < y.first;
                     });
    std::vector<std::pair<int32_t, double>> out;
    for (auto& pr : acc) {
      if (!out.empty() && out.back().first == pr.first)
        out.back().second += pr.second;
      else
        out.push_back(pr);
    }
    rowsv[v].swap(out);
  }, 256);
  for (int32_t v = 0; v < n; ++v) hm.lap_ptr[v + 1] = hm.lap_ptr[v] + (int32_t)rowsv[v].size();
  hm.lap_idx.resize(hm.lap_ptr[n]);
  hm.lap_val.resize(hm.lap_ptr[n]);
  for (int32_t v = 0; v < n; ++v) {
    int32_t o = hm.lap_ptr[v];
    for (size_t k = 0; k < rowsv[v].size(); ++k) {
      hm.lap_idx[o + k] = rowsv[v][k].first;
      hm.lap_val[o + k] = rowsv[v][k].second;
    }
  }
}

// ------------------------------------------------------------------ ordering
struct NDNode {
  std::vector<int32_t> cols;       // free-local vertex indices
  std::vector<int32_t> children;
};

struct NDBuilder {
  const HostMesh& hm;
  const std::vector<int32_t>& fl;        // free-local -> user id
  const std::vector<int32_t>& adj_ptr;   // free-local adjacency
  const std::vector<int32_t>& adj;
  int leaf;
  std::vector<NDNode> nodes;
  std::vector<int8_t> side;

  NDBuilder(const HostMesh& h, const std::vector<int32_t>& f, const std::vector<int32_t>& ap,
            const std::vector<int32_t>& a, int lf)
      : hm(h), fl(f), adj_ptr(ap), adj(a), leaf(lf), side(f.size(), -1) {}

  double coord(int32_t v, int ax) const { return hm.rest[3 * (int64_t)fl[v] + ax]; }

  int make_leaf(std::vector<int32_t>& verts) {
    // order a leaf's vertices lexicographically (z, y, x) for locality
    std::sort(verts.begin(), verts.end(), [&](int32_t a, int32_t b) {
      for (int ax = 2; ax >= 0; --ax) {
        double ca = coord(a, ax), cb = coord(b, ax);
        if (ca != cb) return ca < cb;
      }
      return a < b;
    });
    nodes.push_back(NDNode{verts, {}});
    return (int)nodes.size() - 1;
  }

  std::vector<int> build(std::vector<int32_t> verts) {
    if ((int)verts.size() <= leaf) {
      if (verts.empty()) return {};
      return {make_leaf(verts)};
    }
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int32_t v : verts)
      for (int ax = 0; ax < 3; ++ax) {
        lo[ax] = std::min(lo[ax], coord(v, ax));
        hi[ax] = std::max(hi[ax], coord(v, ax));
      }
    int axes[3] = {0, 1, 2};
    std::sort(axes, axes + 3, [&](int a, int b) { return hi[a] - lo[a] > hi[b] - lo[b]; });
    std::vector<int32_t> A, B;
    bool ok = false;
    for (int t = 0; t < 3 && !ok; ++t) {
      int ax = axes[t];
      std::vector<double> cs(verts.size());
      for (size_t i = 0; i < verts.size(); ++i) cs[i] = coord(verts[i], ax);
      std::nth_element(cs.begin(), cs.begin() + cs.size() / 2, cs.end());
      double xm = cs[cs.size() / 2];
      for (int pass = 0; pass < 2 && !ok; ++pass) {
        A.clear();
        B.clear();
        for (int32_t v : verts) {
          double c = coord(v, ax);
          bool inA = pass == 0 ? (c < xm) : (c <= xm);
          (inA ? A : B).push_back(v);
        }
        ok = !A.empty() && !B.empty();
      }
    }
    if (!ok) return {make_leaf(verts)};
    for (int32_t v : A) side[v] = 0;
    for (int32_t v : B) side[v] = 1;
    std::vector<int32_t> SA, SB;
    for (int32_t v : A)
      for (int32_t k = adj_ptr[v]; k < adj_ptr[v + 1]; ++k)
        if (side[adj[k]] == 1) {
          SA.push_back(v);
          break;
        }
    for (int32_t v : B)
      for (int32_t k = adj_ptr[v]; k < adj_ptr[v + 1]; ++k)
        if (side[adj[k]] == 0) {
          SB.push_back(v);
          break;
        }
    for (int32_t v : verts) side[v] = -1;
    std::vector<int32_t> S;
    if (SB.size() <= SA.size()) {
      S = SB;
      for (int32_t v : SB) side[v] = 2;
      std::vector<int32_t> B2;
      for (int32_t v : B)
        if (side[v] != 2) B2.push_back(v);
      for (int32_t v : SB) side[v] = -1;
      B.swap(B2);
    } else {
      S = SA;
      for (int32_t v : SA) side[v] = 2;
      std::vector<int32_t> A2;
      for (int32_t v : A)
        if (side[v] != 2) A2.push_back(v);
      for (int32_t v : SA) side[v] = -1;
      A.swap(A2);
    }
    std::vector<int> left = build(std::move(A));
    std::vector<int> right = build(std::move(B));
    if (S.empty()) {
      left.insert(left.end(), right.begin(), right.end());
      return left;
    }
    NDNode nd;
    nd.cols = S;
    std::sort(nd.cols.begin(), nd.cols.end(), [&](int32_t a, int32_t b) {
      for (int ax = 2; ax >= 0; --ax) {
        double ca = coord(a, ax), cb = coord(b, ax);
        if (ca != cb) return ca < cb;
      }
      return a < b;
    });
    nd.children = left;
    nd.children.insert(nd.children.end(), right.begin(), right.end());
    nodes.push_back(std::move(nd));
    return {(int)nodes.size() - 1};
  }
};

// The separators of the top levels of the dissection are merged, level by
// level while the total width stays within max_w, into one dense root
// supernode: its factor is dense (the blocks between sibling separators fill
// in), but the top of the elimination tree then costs one level of the
// triangular sweeps instead of several.  Leaves met on the way stay children.
// The width is capped at kMergeWidth and at n_free / 16 (small meshes keep a
// sparse top).
static constexpr int kMergeWidth = 1536;

static int merge_top_separators(NDBuilder& nb, int root, size_t max_w) {
  std::vector<int> absorbed{root};
  std::vector<int> frontier = nb.nodes[root].children;
  size_t width = nb.nodes[root].cols.size();
  for (;;) {
    size_t add = 0;
    bool any = false;
    for (int c : frontier)
      if (!nb.nodes[c].children.empty()) {
        add += nb.nodes[c].cols.size();
        any = true;
      }
    if (!any || width + add > max_w) break;
    std::vector<int> next;
    for (int c : frontier) {
      if (nb.nodes[c].children.empty()) {
        next.push_back(c);
      } else {
        absorbed.push_back(c);
        for (int k : nb.nodes[c].children) next.push_back(k);
      }
    }
    width += add;
    frontier.swap(next);
  }
  if (absorbed.size() == 1) return root;
  NDNode merged;
  // deeper separators first, the top separator last (their original order)
  for (auto it = absorbed.rbegin(); it != absorbed.rend(); ++it)
    merged.cols.insert(merged.cols.end(), nb.nodes[*it].cols.begin(), nb.nodes[*it].cols.end());
  merged.children = frontier;
  nb.nodes.push_back(std::move(merged));
  return (int)nb.nodes.size() - 1;
}

// ------------------------------------------------------------------ dense kernels
// In-place Cholesky of the leading w x w block of a row-major matrix with
// leading dimension ld (lower triangle), right-looking in panels of 64 columns
// (panel solves and trailing updates split over rows when `par`).  Returns
// false on a non-positive pivot.
static bool dense_chol(int w, double* A, int64_t ld, bool par) {
  constexpr int NB = 64;
  for (int j0 = 0; j0 < w; j0 += NB) {
    const int j1 = std::min(w, j0 + NB);
    for (int j = j0; j < j1; ++j) {
      double* rj = A + j * ld;
      double s = rj[j];
      for (int k = j0; k < j; ++k) s -= rj[k] * rj[k];
      if (!(s > 0) || !std::isfinite(s)) return false;
      const double d = std::sqrt(s);
      rj[j] = d;
      const double inv = 1.0 / d;
      for (int i = j + 1; i < j1; ++i) {
        double* ri = A + i * ld;
        double t = ri[j];
        for (int k = j0; k < j; ++k) t -= ri[k] * rj[k];
        ri[j] = t * inv;
      }
    }
    if (j1 == w) break;
    auto panel = [&](int64_t ii) {
      double* ri = A + (j1 + ii) * ld;
      for (int j = j0; j < j1; ++j) {
        const double* rj = A + j * ld;
        double t = ri[j];
        for (int k = j0; k < j; ++k) t -= ri[k] * rj[k];
        ri[j] = t / rj[j];
      }
    };
    auto trail = [&](int64_t ii) {
      const int i = j1 + (int)ii;
      double* ri = A + (int64_t)i * ld;
      for (int k = j1; k <= i; ++k) {
        const double* rk = A + (int64_t)k * ld;
        double t = 0;
        for (int j = j0; j < j1; ++j) t += ri[j] * rk[j];
        ri[k] -= t;
      }
    };
    const int64_t rows = w - j1;
    if (par && rows > 128) {
      parallel_for(rows, panel, 16);
      parallel_for(rows, trail, 8);
    } else {
      for (int64_t r = 0; r < rows; ++r) panel(r);
      for (int64_t r = 0; r < rows; ++r) trail(r);
    }
  }
  return true;
}

static void front_factor(Factor& fac, int s, std::vector<double>& Fm, int h,
                         std::vector<double>& U, bool par) {
  const int w = fac.w[s];
  double* F = Fm.data();
  const int64_t ld = h;
  if (!dense_chol(w, F, ld, par)) fail(EMU_E_SINGULAR, "ACAP operator is not positive definite "
                                  "(a connected part of the mesh has no pinned vertex)");
  const int hb = h - w;
  // The dense products below keep every dot product a single sum in
  // ascending k (the same rounding as one product at a time) and interleave
  // four or eight independent ones, so that the additions do not wait on
  // each other.
  // TRSM: rows r >= w:  L_od[r] = F[r] L_dd^{-T}, four rows at a time
  auto trsm_rows = [&](int64_t blk) {
    const int64_t r0 = 4 * blk, nr = std::min<int64_t>(4, hb - r0);
    double* ri[4];
    for (int q = 0; q < 4; ++q) ri[q] = F + (w + r0 + std::min<int64_t>(q, nr - 1)) * ld;
    for (int j = 0; j < w; ++j) {
      const double* rj = F + j * ld;
      double t0 = ri[0][j], t1 = ri[1][j], t2 = ri[2][j], t3 = ri[3][j];
      for (int k = 0; k < j; ++k) {
        const double x = rj[k];
        t0 -= ri[0][k] * x;
        t1 -= ri[1][k] * x;
        t2 -= ri[2][k] * x;
        t3 -= ri[3][k] * x;
      }
      // rows past hb alias the last row; it is written last with its own value
      ri[3][j] = t3 / rj[j];
      ri[2][j] = t2 / rj[j];
      ri[1][j] = t1 / rj[j];
      ri[0][j] = t0 / rj[j];
    }
  };
  const int64_t hb4 = (hb + 3) / 4;
  if (par) parallel_for(hb4, trsm_rows, 1); else for (int64_t r = 0; r < hb4; ++r) trsm_rows(r);
  // SYRK: U = F_bb - L_od L_od^T (lower, row-major hb x hb), eight entries of
  // a row at a time
  U.assign((size_t)hb * hb, 0.0);
  auto syrk_row = [&](int64_t a) {
    const double* la = F + (w + a) * ld;
    double* ua = U.data() + a * hb;
    const double* fa = F + (w + a) * ld + w;
    int b = 0;
    for (; b + 7 <= a; b += 8) {
      const double* lb = F + (w + b) * ld;
      double t[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      for (int k = 0; k < w; ++k) {
        const double x = la[k];
        for (int q = 0; q < 8; ++q) t[q] += x * lb[q * ld + k];
      }
      for (int q = 0; q < 8; ++q) ua[b + q] = fa[b + q] - t[q];
    }
    for (; b <= a; ++b) {
      const double* lb = F + (w + b) * ld;
      double t = 0;
      for (int k = 0; k < w; ++k) t += la[k] * lb[k];
      ua[b] = fa[b] - t;
    }
  };
  if (par) parallel_for(hb, syrk_row, 4); else for (int a = 0; a < hb; ++a) syrk_row(a);
  // Linv = L_dd^{-1} (lower, packed rows) and M = L_od Linv.  The inverse is
  // built column by column into the rows of LinvT (LinvT[c][k] = Linv[k][c]),
  // so that both the substitutions and the rows of M are contiguous dot
  // products (the same terms in the same order as over the columns of Linv).
  double* out = fac.vals.data() + fac.valoff[s];
  std::vector<double> LinvT((size_t)w * w, 0.0);
  auto inv_col = [&](int64_t cc) {
    // column c of the inverse: forward substitution L x = e_c
    const int c = (int)cc;
    double* x = LinvT.data() + (size_t)c * w;
    x[c] = 1.0 / F[c * ld + c];
    for (int r = c + 1; r < w; ++r) {
      const double* rr = F + r * ld;
      double t = 0;
      for (int k = c; k < r; ++k) t += rr[k] * x[k];
      x[r] = -t / rr[r];
    }
  };
  if (par && w > 128) parallel_for(w, inv_col, 8);
  else for (int c = 0; c < w; ++c) inv_col(c);
  int64_t o = 0;
  for (int r = 0; r < w; ++r)
    for (int c = 0; c <= r; ++c) out[o++] = LinvT[(size_t)c * w + r];
  double* Mo = out + o;
  // rows of M four at a time (rows past hb repeat the last row, stored once)
  auto m_rows = [&](int64_t blk) {
    const int64_t a0 = 4 * blk, na = std::min<int64_t>(4, hb - a0);
    const double* la[4];
    for (int q = 0; q < 4; ++q) la[q] = F + (w + a0 + std::min<int64_t>(q, na - 1)) * ld;
    for (int c = 0; c < w; ++c) {
      const double* xc = LinvT.data() + (size_t)c * w;
      double t0 = 0, t1 = 0, t2 = 0, t3 = 0;
      for (int k = c; k < w; ++k) {
        const double x = xc[k];
        t0 += la[0][k] * x;
        t1 += la[1][k] * x;
        t2 += la[2][k] * x;
        t3 += la[3][k] * x;
      }
      const double tq[4] = {t0, t1, t2, t3};
      for (int q = 0; q < na; ++q) Mo[(a0 + q) * w + c] = tq[q];
    }
  };
  if (par) parallel_for(hb4, m_rows, 1); else for (int64_t r = 0; r < hb4; ++r) m_rows(r);
}

static void order_and_factor(HostMesh& hm) {
  const int32_t n = hm.n;
  std::vector<char> pinned(n, 0);
  for (int32_t p : hm.pins) pinned[p] = 1;
  std::vector<int32_t> fl;             // free-local -> user
  std::vector<int32_t> flocal(n, -1);  // user -> free-local
  for (int32_t v = 0; v < n; ++v)
    if (!pinned[v]) {
      flocal[v] = (int32_t)fl.size();
      fl.push_back(v);
    }
  const int32_t nf = (int32_t)fl.size();
  if (nf == 0) fail(EMU_E_INVALID, "every vertex is pinned");
  // every connected part of the mesh needs a pinned vertex, or L_ff is singular
  {
    std::vector<int32_t> comp(n, -1), stack;
    int32_t nc = 0;
    for (int32_t s0 = 0; s0 < n; ++s0) {
      if (comp[s0] >= 0 || hm.lap_ptr[s0] == hm.lap_ptr[s0 + 1]) continue;
      bool has_pin = false;
      comp[s0] = nc;
      stack.assign(1, s0);
      while (!stack.empty()) {
        int32_t u = stack.back();
        stack.pop_back();
        has_pin = has_pin || pinned[u];
        for (int32_t k = hm.lap_ptr[u]; k < hm.lap_ptr[u + 1]; ++k) {
          int32_t v = hm.lap_idx[k];
          if (comp[v] < 0) {
            comp[v] = nc;
            stack.push_back(v);
          }
        }
      }
      if (!has_pin)
        fail(EMU_E_SINGULAR, "a connected part of the mesh has no pinned vertex (vertex " +
                                 std::to_string(s0) + ")");
      ++nc;
    }
    for (int32_t v = 0; v < n; ++v)
      if (comp[v] < 0 && !pinned[v])
        fail(EMU_E_SINGULAR, "vertex " + std::to_string(v) + " belongs to no tet and is not pinned");
  }
  if (hm.k1_default) hm.k1 = std::min(hm.k1, std::max(0, nf - 1));
  if (hm.k1 > 0 && hm.k1 >= nf) fail(EMU_E_INVALID, "n_modes/3 must be < number of free vertices");
  hm.nf = nf;
  std::vector<int32_t> adj_ptr(nf + 1, 0), adj;
  for (int32_t i = 0; i < nf; ++i) {
    int32_t u = fl[i];
    for (int32_t k = hm.lap_ptr[u]; k < hm.lap_ptr[u + 1]; ++k) {
      int32_t v = hm.lap_idx[k];
      if (v != u && flocal[v] >= 0) adj.push_back(flocal[v]);
    }
    adj_ptr[i + 1] = (int32_t)adj.size();
  }
  NDBuilder nb(hm, fl, adj_ptr, adj, hm.leaf_size);
  std::vector<int32_t> all(nf);
  std::iota(all.begin(), all.end(), 0);
  std::vector<int> roots = nb.build(all);
  for (int& r : roots) r = merge_top_separators(nb, r, std::min<size_t>(kMergeWidth, nf / 16));

  // postorder numbering of supernodes and columns
  Factor& fac = hm.fac;
  fac.nf = nf;
  std::vector<int> post;               // supernode index -> ND node
  std::vector<int32_t> newcol(nf, -1);  // free-local -> factor column
  {
    std::vector<std::pair<int, int>> st;
    for (int r = (int)roots.size() - 1; r >= 0; --r) st.push_back({roots[r], 0});
    while (!st.empty()) {
      auto& top = st.back();
      NDNode& nd = nb.nodes[top.first];
      if (top.second < (int)nd.children.size()) {
        int c = nd.children[top.second++];
        st.push_back({c, 0});
      } else {
        post.push_back(top.first);
        st.pop_back();
      }
    }
  }
  const int ns = (int)post.size();
  fac.ns = ns;
  fac.col0.resize(ns);
  fac.w.resize(ns);
  fac.h.resize(ns);
  fac.parent.assign(ns, -1);
  fac.level.assign(ns, 0);
  std::vector<int> sn_of_node(nb.nodes.size(), -1);
  int32_t col = 0;
  for (int s = 0; s < ns; ++s) {
    NDNode& nd = nb.nodes[post[s]];
    sn_of_node[post[s]] = s;
    fac.col0[s] = col;
    fac.w[s] = (int32_t)nd.cols.size();
    for (int32_t v : nd.cols) newcol[v] = col++;
  }
  for (int s = 0; s < ns; ++s)
    for (int c : nb.nodes[post[s]].children) fac.parent[sn_of_node[c]] = s;
  // children lists and levels
  fac.child_ptr.assign(ns + 1, 0);
  for (int s = 0; s < ns; ++s)
    if (fac.parent[s] >= 0) fac.child_ptr[fac.parent[s] + 1]++;
  for (int s = 0; s < ns; ++s) fac.child_ptr[s + 1] += fac.child_ptr[s];
  fac.child_idx.resize(fac.child_ptr[ns]);
  {
    std::vector<int32_t> pos(fac.child_ptr.begin(), fac.child_ptr.end() - 1);
    for (int s = 0; s < ns; ++s)
      if (fac.parent[s] >= 0) fac.child_idx[pos[fac.parent[s]]++] = s;
  }
  fac.nlevels = 0;
  for (int s = 0; s < ns; ++s) {
    int lv = 0;
    for (int k = fac.child_ptr[s]; k < fac.child_ptr[s + 1]; ++k)
      lv = std::max(lv, fac.level[fac.child_idx[k]] + 1);
    fac.level[s] = lv;
    fac.nlevels = std::max(fac.nlevels, lv + 1);
  }
  // internal vertex numbering: free in factor order, then pinned
  hm.vnew.assign(n, -1);
  hm.vold.assign(n, -1);
  for (int32_t i = 0; i < nf; ++i) {
    hm.vnew[fl[i]] = newcol[i];
    hm.vold[newcol[i]] = fl[i];
  }
  {
    int32_t k = nf;
    for (int32_t p : hm.pins) {
      hm.vnew[p] = k;
      hm.vold[k] = p;
      ++k;
    }
  }
  // symbolic: off-diagonal structure per supernode (postorder)
  std::vector<std::vector<int32_t>> st(ns);
  for (int s = 0; s < ns; ++s) {
    const int32_t c0 = fac.col0[s], c1 = c0 + fac.w[s];
    std::vector<int32_t> rs;
    for (int32_t j = c0; j < c1; ++j) {
      int32_t u = hm.vold[j];
      for (int32_t k = hm.lap_ptr[u]; k < hm.lap_ptr[u + 1]; ++k) {
        int32_t v = hm.vnew[hm.lap_idx[k]];
        if (v < nf && v >= c1) rs.push_back(v);
      }
    }
    for (int k = fac.child_ptr[s]; k < fac.child_ptr[s + 1]; ++k) {
      int c = fac.child_idx[k];
      for (int32_t v : st[c])
        if (v >= c1) rs.push_back(v);
    }
    std::sort(rs.begin(), rs.end());
    rs.erase(std::unique(rs.begin(), rs.end()), rs.end());
    st[s].swap(rs);
  }
  fac.rowoff.resize(ns + 1);
  fac.valoff.resize(ns + 1);
  int64_t ro = 0, vo = 0;
  for (int s = 0; s < ns; ++s) {
    fac.h[s] = fac.w[s] + (int32_t)st[s].size();
    fac.rowoff[s] = (int32_t)ro;
    fac.valoff[s] = vo;
    ro += (int64_t)st[s].size();
    int64_t w = fac.w[s], hh = fac.h[s];
    vo += w * (w + 1) / 2 + (hh - w) * w;
  }
  fac.rowoff[ns] = (int32_t)ro;
  fac.valoff[ns] = vo;
  fac.rows.resize(ro);
  for (int s = 0; s < ns; ++s) std::copy(st[s].begin(), st[s].end(), fac.rows.begin() + fac.rowoff[s]);
  fac.vals.assign(vo, 0.0);

  // numeric multifrontal factorization, level by level (children first)
  std::vector<std::vector<double>> upd(ns);
  std::vector<std::vector<int>> by_level(fac.nlevels);
  for (int s = 0; s < ns; ++s) by_level[fac.level[s]].push_back(s);
  auto do_front = [&](int s, bool par) {
    const int w = fac.w[s], h = fac.h[s];
    const int32_t c0 = fac.col0[s];
    // index list and positions
    std::vector<int32_t> idx(h);
    for (int i = 0; i < w; ++i) idx[i] = c0 + i;
    for (int i = w; i < h; ++i) idx[i] = fac.rows[fac.rowoff[s] + i - w];
    auto pos_of = [&](int32_t v) -> int {
      if (v < c0 + w) return v - c0;
      return w + (int)(std::lower_bound(idx.begin() + w, idx.end(), v) - (idx.begin() + w));
    };
    std::vector<double> Fm((size_t)h * h, 0.0);
    for (int jj = 0; jj < w; ++jj) {
      int32_t j = c0 + jj;
      int32_t u = hm.vold[j];
      for (int32_t k = hm.lap_ptr[u]; k < hm.lap_ptr[u + 1]; ++k) {
        int32_t i = hm.vnew[hm.lap_idx[k]];
        if (i < nf && i >= j) Fm[(size_t)pos_of(i) * h + jj] += hm.lap_val[k];
      }
    }
    for (int k = fac.child_ptr[s]; k < fac.child_ptr[s + 1]; ++k) {
      int c = fac.child_idx[k];
      const int hb = fac.h[c] - fac.w[c];
      const int32_t* cr = fac.rows.data() + fac.rowoff[c];
      std::vector<int> cp(hb);
      for (int a = 0; a < hb; ++a) cp[a] = pos_of(cr[a]);
      const double* Uc = upd[c].data();
      for (int a = 0; a < hb; ++a)
        for (int b = 0; b <= a; ++b) Fm[(size_t)cp[a] * h + cp[b]] += Uc[(size_t)a * hb + b];
      std::vector<double>().swap(upd[c]);
    }
    front_factor(fac, s, Fm, h, upd[s], par);
  };
  for (int lv = 0; lv < fac.nlevels; ++lv) {
    auto& L = by_level[lv];
    if ((int)L.size() >= 2 * n_threads()) {
      std::atomic<int> err(0);
      Error first{EMU_OK, ""};
      parallel_for((int64_t)L.size(), [&](int64_t i) {
        try {
          do_front(L[i], false);
        } catch (const Error& e) {
          if (err.exchange(1) == 0) first = e;
        }
      });
      if (err) throw first;
    } else {
      for (int s : L) do_front(s, true);
    }
  }
  for (int s = 0; s < ns; ++s) std::vector<double>().swap(upd[s]);
}

void recompute_pin_rhs(HostMesh& hm) {
  const int32_t nf = hm.nf;
  hm.pin_rhs.assign(3 * (int64_t)nf, 0.0);
  std::vector<int32_t> pin_index(hm.n, -1);
  for (int i = 0; i < hm.npins; ++i) pin_index[hm.pins[i]] = i;
  parallel_for(nf, [&](int64_t f) {
    int32_t u = hm.vold[f];
    double acc[3] = {0, 0, 0};
    for (int32_t k = hm.lap_ptr[u]; k < hm.lap_ptr[u + 1]; ++k) {
      int32_t p = pin_index[hm.lap_idx[k]];
      if (p >= 0)
        for (int c = 0; c < 3; ++c) acc[c] -= hm.lap_val[k] * hm.pin_xyz[3 * p + c];
    }
    for (int c = 0; c < 3; ++c) hm.pin_rhs[3 * f + c] = acc[c];
  }, 1024);
}

// ------------------------------------------------------------------ host solves
void host_factor_solve(const Factor& f, int nrhs, const double* b, double* x) {
  // Both sweeps level by level (the supernodes of one level are independent),
  // each supernode with all right-hand sides at once, so the factor is read
  // once per sweep.  Per right-hand side the arithmetic and its order are those
  // of a sequential sweep.
  const int ns = f.ns, nr = nrhs;
  if (nr <= 0) return;
  std::vector<std::vector<int>> by_level(std::max<int32_t>(1, f.nlevels));
  for (int s = 0; s < ns; ++s) by_level[f.level[s]].push_back(s);
  std::vector<double> y((size_t)f.nf * nr), u((size_t)f.rowoff[ns] * nr, 0.0);
  for (int lv = 0; lv < f.nlevels; ++lv) {
    const auto& L = by_level[lv];
    parallel_for((int64_t)L.size(), [&](int64_t idx) {
      const int s = L[idx];
      const int w = f.w[s], h = f.h[s];
      const int32_t c0 = f.col0[s];
      std::vector<double> fr((size_t)h * nr, 0.0);
      for (int i = 0; i < w; ++i)
        for (int r = 0; r < nr; ++r) fr[(size_t)i * nr + r] = b[(size_t)(c0 + i) * nrhs + r];
      const int32_t* rows_s = f.rows.data() + f.rowoff[s];
      for (int k = f.child_ptr[s]; k < f.child_ptr[s + 1]; ++k) {
        int c = f.child_idx[k];
        const int hb = f.h[c] - f.w[c];
        const int32_t* cr = f.rows.data() + f.rowoff[c];
        for (int a = 0; a < hb; ++a) {
          int32_t v = cr[a];
          int p = v < c0 + w ? v - c0
                             : w + (int)(std::lower_bound(rows_s, rows_s + (h - w), v) - rows_s);
          for (int r = 0; r < nr; ++r) fr[(size_t)p * nr + r] += u[(size_t)(f.rowoff[c] + a) * nr + r];
        }
      }
      const double* Lv = f.vals.data() + f.valoff[s];
      const int64_t tri = (int64_t)w * (w + 1) / 2;
      // rows of the block are independent: large blocks on levels with few
      // supernodes split their rows over threads as well
      const bool split = L.size() < 4 && (int64_t)w * h * nr > (1 << 22);
      // the right-hand sides are the inner, contiguous loop (same order of
      // the sum over c for each of them)
      auto yrow = [&](int64_t i) {
        const int64_t o = i * (i + 1) / 2;
        double* t = y.data() + (size_t)(c0 + i) * nr;
        for (int r = 0; r < nr; ++r) t[r] = 0;
        for (int c = 0; c <= i; ++c) {
          const double l = Lv[o + c];
          const double* fc = fr.data() + (size_t)c * nr;
          for (int r = 0; r < nr; ++r) t[r] += l * fc[r];
        }
      };
      auto urow = [&](int64_t a) {
        const double* Mr = Lv + tri + a * w;
        double* t = u.data() + (size_t)(f.rowoff[s] + a) * nr;
        for (int r = 0; r < nr; ++r) t[r] = fr[(size_t)(w + a) * nr + r];
        for (int c = 0; c < w; ++c) {
          const double l = Mr[c];
          const double* fc = fr.data() + (size_t)c * nr;
          for (int r = 0; r < nr; ++r) t[r] -= l * fc[r];
        }
      };
      if (split) {
        parallel_for(w, yrow, 16);
        parallel_for(h - w, urow, 16);
      } else {
        for (int i = 0; i < w; ++i) yrow(i);
        for (int a = 0; a < h - w; ++a) urow(a);
      }
    });
  }
  std::vector<double> xs((size_t)f.nf * nr, 0.0);
  for (int lv = f.nlevels - 1; lv >= 0; --lv) {
    const auto& L = by_level[lv];
    parallel_for((int64_t)L.size(), [&](int64_t idx) {
      const int s = L[idx];
      const int w = f.w[s], h = f.h[s];
      const int32_t c0 = f.col0[s];
      const double* Lv = f.vals.data() + f.valoff[s];
      const int32_t* rows_s = f.rows.data() + f.rowoff[s];
      std::vector<double> acc((size_t)w * nr, 0.0);
      int64_t o = 0;
      for (int i = 0; i < w; ++i) {
        for (int c = 0; c <= i; ++c)
          for (int r = 0; r < nr; ++r) acc[(size_t)c * nr + r] += Lv[o + c] * y[(size_t)(c0 + i) * nr + r];
        o += i + 1;
      }
      for (int a = 0; a < h - w; ++a) {
        const double* Mr = Lv + o + (int64_t)a * w;
        const double* xr = xs.data() + (size_t)rows_s[a] * nr;
        for (int c = 0; c < w; ++c)
          for (int r = 0; r < nr; ++r) acc[(size_t)c * nr + r] -= Mr[c] * xr[r];
      }
      for (int c = 0; c < w; ++c)
        for (int r = 0; r < nr; ++r) xs[(size_t)(c0 + c) * nr + r] = acc[(size_t)c * nr + r];
    });
  }
  for (int64_t i = 0; i < f.nf; ++i)
    for (int r = 0; r < nr; ++r) x[(size_t)i * nrhs + r] = xs[(size_t)i * nr + r];
}

void host_lff_apply(const HostMesh& hm, int nrhs, const double* x, double* y) {
  parallel_for(hm.nf, [&](int64_t i) {
    int32_t u = hm.vold[i];
    for (int r = 0; r < nrhs; ++r) y[(size_t)i * nrhs + r] = 0;
    for (int32_t k = hm.lap_ptr[u]; k < hm.lap_ptr[u + 1]; ++k) {
      int32_t j = hm.vnew[hm.lap_idx[k]];
      if (j < hm.nf)
        for (int r = 0; r < nrhs; ++r) y[(size_t)i * nrhs + r] += hm.lap_val[k] * x[(size_t)j * nrhs + r];
    }
  }, 1024);
}

// ------------------------------------------------------------------ eigen
void jacobi_eigh(int n, double* A, double* ev, double* V) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) V[i * n + j] = i == j ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0, tot = 0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        tot += A[i * n + j] * A[i * n + j];
        if (i != j) off += A[i * n + j] * A[i * n + j];
      }
    if (off <= 1e-30 * tot || off == 0) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        double apq = A[p * n + q];
        if (apq == 0) continue;
        double app = A[p * n + p], aqq = A[q * n + q];
        double theta = (aqq - app) / (2 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1));
        double c = 1 / std::sqrt(t * t + 1), s = t * c;
        for (int k = 0; k < n; ++k) {
          double akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = c * akp - s * akq;
          A[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          double apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = c * apk - s * aqk;
          A[q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          double vkp = V[k * n + p], vkq = V[k * n + q];
          V[k * n + p] = c * vkp - s * vkq;
          V[k * n + q] = s * vkp + c * vkq;
        }
      }
  }
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::vector<double> d(n);
  for (int i = 0; i < n; ++i) d[i] = A[i * n + i];
  std::sort(order.begin(), order.end(), [&](int a, int b) { return d[a] < d[b]; });
  std::vector<double> V2((size_t)n * n);
  for (int j = 0; j < n; ++j) {
    ev[j] = d[order[j]];
    for (int i = 0; i < n; ++i) V2[(size_t)i * n + j] = V[i * n + order[j]];
  }
  std::copy(V2.begin(), V2.end(), V);
}

// Deterministic dense helpers over tall row-major blocks (nf rows): partial
// sums over fixed 4096-row chunks, added in chunk order.
static constexpr int64_t kChunk = 4096;

// G = A^T B  (A: nf x pa, B: nf x pb, row-major; G: pa x pb)
static void gram_tn(int64_t nf, int pa, const double* A, int lda, int pb, const double* B, int ldb,
                    std::vector<double>& G) {
  const int64_t nch = (nf + kChunk - 1) / kChunk;
  std::vector<double> part((size_t)nch * pa * pb, 0.0);
  parallel_for(nch, [&](int64_t ch) {
    double* P = part.data() + (size_t)ch * pa * pb;
    const int64_t r0 = ch * kChunk, r1 = std::min(nf, r0 + kChunk);
    for (int64_t i = r0; i < r1; ++i) {
      const double* a = A + i * lda;
      const double* b = B + i * ldb;
      for (int x = 0; x < pa; ++x) {
        const double av = a[x];
        double* Px = P + (size_t)x * pb;
        for (int y = 0; y < pb; ++y) Px[y] += av * b[y];
      }
    }
  });
  G.assign((size_t)pa * pb, 0.0);
  for (int64_t ch = 0; ch < nch; ++ch)
    for (size_t k = 0; k < G.size(); ++k) G[k] += part[(size_t)ch * pa * pb + k];
}

// C = A W  (A: nf x pa, W: pa x pc) -> C row-major nf x pc
static void mul_nn(int64_t nf, int pa, const double* A, int lda, int pc, const double* W, double* C, int ldc) {
  parallel_for(nf, [&](int64_t i) {
    const double* a = A + i * lda;
    double* c = C + i * ldc;
    for (int y = 0; y < pc; ++y) c[y] = 0;
    for (int x = 0; x < pa; ++x) {
      const double av = a[x];
      const double* w = W + (size_t)x * pc;
      for (int y = 0; y < pc; ++y) c[y] += av * w[y];
    }
  }, 2048);
}

// Orthonormalize the columns [c0, c1) of Q (nf x ld) against columns [0, c0)
// (two passes of block Gram-Schmidt) and among themselves (Cholesky QR, twice).
// Returns the number of columns kept (rank-deficient columns are dropped).
static int orth_block(int64_t nf, double* Q, int ld, int c0, int c1) {
  int nb = c1 - c0;
  std::vector<double> G;
  std::vector<double> Wt;
  for (int pass = 0; pass < 2; ++pass) {
    if (c0 > 0) {
      gram_tn(nf, c0, Q, ld, nb, Q + c0, ld, G);  // c0 x nb
      parallel_for(nf, [&](int64_t i) {
        double* q = Q + i * ld;
        for (int x = 0; x < c0; ++x) {
          const double qx = q[x];
          for (int y = 0; y < nb; ++y) q[c0 + y] -= qx * G[(size_t)x * nb + y];
        }
      }, 2048);
    }
    // Cholesky QR of the new block with column dropping
    gram_tn(nf, nb, Q + c0, ld, nb, Q + c0, ld, G);
    std::vector<double> L((size_t)nb * nb, 0.0);
    std::vector<int> keep;
    double maxd = 0;
    for (int j = 0; j < nb; ++j) maxd = std::max(maxd, G[(size_t)j * nb + j]);
    std::vector<double> Linv((size_t)nb * nb, 0.0);
    // pivot-free Cholesky; columns whose remaining norm is tiny are dropped
    std::vector<double> A = G;
    std::vector<char> ok(nb, 0);
    for (int j = 0; j < nb; ++j) {
      double d = A[(size_t)j * nb + j];
      for (int k = 0; k < j; ++k)
        if (ok[k]) d -= L[(size_t)j * nb + k] * L[(size_t)j * nb + k];
      if (d > 1e-20 * maxd && d > 0) {
        ok[j] = 1;
        L[(size_t)j * nb + j] = std::sqrt(d);
        for (int i = j + 1; i < nb; ++i) {
          double t = A[(size_t)i * nb + j];
          for (int k = 0; k < j; ++k)
            if (ok[k]) t -= L[(size_t)i * nb + k] * L[(size_t)j * nb + k];
          L[(size_t)i * nb + j] = t / L[(size_t)j * nb + j];
        }
      }
    }
    for (int j = 0; j < nb; ++j)
      if (ok[j]) keep.push_back(j);
    const int nk = (int)keep.size();
    // Q_new = Q_block L^{-T} restricted to kept columns: solve per row
    parallel_for(nf, [&](int64_t i) {
      double* q = Q + i * ld + c0;
      double tmp[512];
      for (int a = 0; a < nk; ++a) {
        const int j = keep[a];
        double t = q[j];
        for (int b = 0; b < a; ++b) t -= tmp[b] * L[(size_t)j * nb + keep[b]];
        tmp[a] = t / L[(size_t)j * nb + j];
      }
      for (int a = 0; a < nk; ++a) q[a] = tmp[a];
      for (int a = nk; a < nb; ++a) q[a] = 0;
    }, 2048);
    nb = nk;
    if (nb == 0) break;
  }
  return c0 + nb;
}

void host_modes(HostMesh& hm, int k1) {
  const int64_t nf = hm.nf;
  hm.nu.clear();
  hm.phi.clear();
  if (k1 <= 0) return;
  // block Krylov space of L_ff^{-1} (shift-invert about 0), Rayleigh-Ritz with
  // L_ff, thick restart from the lowest Ritz vectors
  const int b = (int)std::min<int64_t>(nf, k1 + 8);
  const int steps = 6;
  const int cap = (int)std::min<int64_t>(nf, (int64_t)b * (steps + 1));
  std::vector<double> Q((size_t)nf * cap, 0.0), LQ((size_t)nf * cap), X((size_t)nf * b);
  std::mt19937_64 rng(20200615ULL);
  std::normal_distribution<double> nd(0.0, 1.0);
  for (auto& v : X) v = nd(rng);
  std::vector<double> T, ev, W, blk, sol;
  for (int cycle = 0; cycle < 40; ++cycle) {
    for (int64_t i = 0; i < nf; ++i)
      for (int j = 0; j < b; ++j) Q[(size_t)i * cap + j] = X[(size_t)i * b + j];
    int nc = orth_block(nf, Q.data(), cap, 0, b);
    int last0 = 0, last1 = nc;
    for (int st = 0; st < steps && nc < cap; ++st) {
      const int nb = std::min(last1 - last0, cap - nc);
      if (nb <= 0) break;
      blk.assign((size_t)nf * nb, 0.0);
      sol.assign((size_t)nf * nb, 0.0);
      for (int64_t i = 0; i < nf; ++i)
        for (int j = 0; j < nb; ++j) blk[(size_t)i * nb + j] = Q[(size_t)i * cap + last0 + j];
      host_factor_solve(hm.fac, nb, blk.data(), sol.data());
      for (int64_t i = 0; i < nf; ++i)
        for (int j = 0; j < nb; ++j) Q[(size_t)i * cap + nc + j] = sol[(size_t)i * nb + j];
      int n2 = orth_block(nf, Q.data(), cap, nc, nc + nb);
      last0 = nc;
      last1 = n2;
      nc = n2;
    }
    // Rayleigh-Ritz: T = Q^T L Q (nc x nc)
    {
      std::vector<double> Qc((size_t)nf * nc), LQc((size_t)nf * nc);
      for (int64_t i = 0; i < nf; ++i)
        for (int j = 0; j < nc; ++j) Qc[(size_t)i * nc + j] = Q[(size_t)i * cap + j];
      host_lff_apply(hm, nc, Qc.data(), LQc.data());
      gram_tn(nf, nc, Qc.data(), nc, nc, LQc.data(), nc, T);
      for (int a = 0; a < nc; ++a)
        for (int c = 0; c < a; ++c) T[(size_t)a * nc + c] = T[(size_t)c * nc + a] = 0.5 * (T[(size_t)a * nc + c] + T[(size_t)c * nc + a]);
      ev.assign(nc, 0.0);
      W.assign((size_t)nc * nc, 0.0);
      jacobi_eigh(nc, T.data(), ev.data(), W.data());
      std::vector<double> Wb((size_t)nc * b);
      for (int a = 0; a < nc; ++a)
        for (int j = 0; j < b; ++j) Wb[(size_t)a * b + j] = W[(size_t)a * nc + j];
      mul_nn(nf, nc, Qc.data(), nc, b, Wb.data(), X.data(), b);
      std::vector<double> LX((size_t)nf * b);
      mul_nn(nf, nc, LQc.data(), nc, b, Wb.data(), LX.data(), b);
      double worst = 0;
      for (int j = 0; j < k1; ++j) {
        double r = 0;
        for (int64_t i = 0; i < nf; ++i) {
          double d = LX[(size_t)i * b + j] - ev[j] * X[(size_t)i * b + j];
          r += d * d;
        }
        worst = std::max(worst, std::sqrt(r) / std::fabs(ev[j]));
      }
      if (worst < 1e-8) break;
    }
  }
  hm.nu.assign(ev.begin(), ev.begin() + k1);
  hm.phi.assign((size_t)k1 * nf, 0.0);
  for (int j = 0; j < k1; ++j) {
    // sign convention: largest-magnitude entry positive
    int64_t im = 0;
    for (int64_t i = 0; i < nf; ++i)
      if (std::fabs(X[(size_t)i * b + j]) > std::fabs(X[(size_t)im * b + j])) im = i;
    double sg = X[(size_t)im * b + j] < 0 ? -1.0 : 1.0;
    double nn = 0;
    for (int64_t i = 0; i < nf; ++i) nn += X[(size_t)i * b + j] * X[(size_t)i * b + j];
    nn = std::sqrt(nn);
    for (int64_t i = 0; i < nf; ++i) hm.phi[(size_t)j * nf + i] = sg * X[(size_t)i * b + j] / nn;
  }
  // captured fraction of trace(L_ff^{-1}) (Hutchinson estimate, 8 probes)
  {
    const int np = 8;
    std::vector<double> Z((size_t)nf * np), ZI((size_t)nf * np);
    std::mt19937_64 r2(7);
    for (auto& v : Z) v = (r2() & 1) ? 1.0 : -1.0;
    host_factor_solve(hm.fac, np, Z.data(), ZI.data());
    double tr = 0;
    for (size_t i = 0; i < Z.size(); ++i) tr += Z[i] * ZI[i];
    tr /= np;
    double capd = 0;
    for (int j = 0; j < k1; ++j) capd += 1.0 / hm.nu[j];
    hm.mode_captured = tr > 0 ? capd / tr : 0;
  }
}

// ------------------------------------------------------------------ driver
void host_setup(const emu_mesh_desc& d, HostMesh& hm, bool compute_modes) {
  auto t0 = std::chrono::steady_clock::now();
  validate(d);
  geometry(d, hm);
  laplacian(hm);
  order_and_factor(hm);
  // internal element order: by smallest internal vertex id (gather locality)
  {
    std::vector<int32_t> key(hm.m);
    for (int32_t i = 0; i < hm.m; ++i) {
      int32_t k = INT32_MAX;
      for (int a = 0; a < 4; ++a) k = std::min(k, hm.vnew[hm.tets[4 * (int64_t)i + a]]);
      key[i] = k;
    }
    hm.eold.resize(hm.m);
    std::iota(hm.eold.begin(), hm.eold.end(), 0);
    std::stable_sort(hm.eold.begin(), hm.eold.end(), [&](int32_t a, int32_t b) { return key[a] < key[b]; });
    hm.enew.resize(hm.m);
    for (int32_t i = 0; i < hm.m; ++i) hm.enew[hm.eold[i]] = i;
  }
  recompute_pin_rhs(hm);
  if (compute_modes) host_modes(hm, hm.k1);
  hm.setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace emu
