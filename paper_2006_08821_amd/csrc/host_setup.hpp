// Host-side mesh setup shared by the device library and the host-only API.
//
// Geometry follows eq. defograd (F = D_s D_m^{-1}); the ACAP energy of
// eq. ACAPEnergy with per-element weights w_i has q-Hessian L_w (x) I_3, where
// L_w is a scalar weighted Laplacian.  Its free block L_ff is factored once
// (the paper prefactors this constant matrix, Sec. 3.2) and its lowest
// eigenpairs give the low-rank modes of eq. low-rank.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/emu.h"

namespace emu {

struct Error {
  emu_status code;
  std::string msg;
};

// Supernodal factor of L_ff in partitioned-inverse form.
//
// Supernode s owns the contiguous columns [col0, col0 + w) and has h >= w rows:
// its own columns followed by the h - w off-diagonal rows (ancestor columns,
// ascending).  Its dense lower-trapezoidal block L_s = [L_dd; L_od] is stored as
//   Linv = L_dd^{-1}   (w x w lower triangle, packed by rows: row r has r+1 entries)
//   M    = L_od L_dd^{-1}  ((h - w) x w, row-major)
// so that both triangular sweeps of a supernode are two independent
// matrix-vector products (no sequential substitution inside a supernode):
//   forward  (L y = b):   y_s = Linv f_top,   u_s = f_bot - M f_top
//   backward (L^T x = y): x_s = Linv^T y_s - M^T x[offdiag rows]
// where f is the frontal vector (b at the columns plus the children's update
// vectors u_c, added at their rows).
struct Factor {
  int32_t nf = 0;
  int32_t ns = 0;                      // supernodes, numbered in postorder
  std::vector<int32_t> col0, w, h;     // per supernode
  std::vector<int32_t> rowoff;         // offset of off-diagonal rows in `rows`
  std::vector<int64_t> valoff;         // offset of the block in `vals`
  std::vector<int32_t> parent;         // -1 for roots
  std::vector<int32_t> level;          // 0 at leaves, 1 + max(children)
  std::vector<int32_t> child_ptr, child_idx;
  std::vector<int32_t> rows;           // off-diagonal row indices (factor order)
  std::vector<double> vals;
  int32_t nlevels = 0;
  int64_t nnz() const { return (int64_t)vals.size(); }
};

struct HostMesh {
  // inputs (user numbering)
  int32_t n = 0, m = 0, ngroups = 0, npins = 0;
  std::vector<double> rest;            // [n][3]
  std::vector<int32_t> tets;           // [m][4] oriented
  std::vector<double> youngs, poisson;
  std::vector<double> fiber;           // [m][3] unit
  std::vector<int32_t> group;
  std::vector<int32_t> bone;           // [m] bone id or -1
  std::vector<int32_t> pins;
  std::vector<double> pin_xyz;         // [npins][3]
  double alpha_hat = 10, mu_ref = 0, kf = 0, alpha = 0;
  int32_t weight_mode = 0, k1 = 16, precision = 0, leaf_size = 64, hessian_blocks = 0, affine_bones = 0;
  double bone_slack = 1e-3;
  bool k1_default = true;            // n_modes not given: capped at n_free - 1

  // derived per element (user order)
  std::vector<double> dminv;           // [m][9] rows of D_m^{-1}
  std::vector<double> vol, mu, lhat, w;

  // vertices: internal id = factor order for free vertices, then pinned
  int32_t nf = 0;
  std::vector<int32_t> vnew;           // user -> internal
  std::vector<int32_t> vold;           // internal -> user
  // elements: internal order sorted by smallest internal vertex id
  std::vector<int32_t> enew, eold;

  // weighted Laplacian over all vertices, CSR in user numbering
  std::vector<int32_t> lap_ptr, lap_idx;
  std::vector<double> lap_val;

  Factor fac;
  std::vector<double> pin_rhs;         // [nf][3] = -L_fp qbar_p (internal order)

  // modes, internal order: nu[k1], phi[k1][nf]
  std::vector<double> nu, phi;
  double mode_captured = 0;

  double setup_ms = 0;
};

// Full host setup; throws Error.
void host_setup(const emu_mesh_desc& d, HostMesh& hm, bool compute_modes = true);
void recompute_pin_rhs(HostMesh& hm);

// Host triangular solves with the factor (nrhs right-hand sides, row-major
// [nf][nrhs] in factor order); used for the eigenpairs and host tests.
void host_factor_solve(const Factor& f, int nrhs, const double* b, double* x);
// y = L_ff x, row-major [nf][nrhs], factor order.
void host_lff_apply(const HostMesh& hm, int nrhs, const double* x, double* y);
// Lowest k eigenpairs of L_ff (subspace iteration with the factor).
void host_modes(HostMesh& hm, int k1);

// small dense symmetric eigensolver (cyclic Jacobi), ascending eigenvalues;
// A is n x n row-major (destroyed), V receives eigenvectors as columns.
void jacobi_eigh(int n, double* A, double* evals, double* V);

void set_error(const std::string& msg);

}  // namespace emu
