// Launch helpers of the HIP kernels (kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/emu.h"
#include "device.hpp"

#define EMU_E_NONFINITE_CODE 5
#define EMU_E_NOT_CONVERGED_CODE 3
#define EMU_E_LINESEARCH_CODE 4

namespace emu {

// Level schedule of the triangular sweeps: work items of forward level L are
// fwd_items[fwd_ptr[L] .. fwd_ptr[L+1]) (leaves first); backward level L
// (root first) uses bwd_ptr likewise.
struct SolvePlan {
  int nlevels = 0;
  std::vector<int> fwd_ptr, bwd_ptr;
  // per level: every item is short (8 lanes per row, one vector chunk of
  // kNarrowChunk), so the level runs the 8-waves-per-SIMD variant
  std::vector<char> fwd_narrow, bwd_narrow;
  // per forward level: column-form items (kItemColBit), four per workgroup
  std::vector<char> fwd_col;
};

// Launch layout of one iteration over several meshes (same precision): for
// each kernel class, `count` blocks whose (mesh, block) pairs start at
// map[offset].  `meshes` and `map` are device arrays.
struct BatchClass {
  int64_t offset = 0;
  int count = 0;
};
struct BatchPlan {
  int n_meshes = 0;
  int mixed = 0;
  const DevMesh* meshes = nullptr;
  const int2* map = nullptr;
  BatchClass element, gram, gram_reduce, one, uz, rhs, add_q;
  std::vector<BatchClass> fwd, bwd;   // per level (forward: leaves first; backward: root first)
};
// Host side of the layout (offsets and the map contents to upload).
void batch_layout(const std::vector<const DevMesh*>& ms, const std::vector<const SolvePlan*>& plans,
                  BatchPlan& b, std::vector<int2>& map);
void launch_batch_iteration(const BatchPlan& b, hipStream_t st);
// copies every mesh's Ctl (as int32 words) to out[j * sizeof(Ctl) / 4 ...]
void launch_batch_gather_ctl(const BatchPlan& b, int32_t* out, hipStream_t st);

void launch_init_rest(const DevMesh& d, hipStream_t st);
void launch_set_F(const DevMesh& d, const double* F, const int32_t* eold, hipStream_t st);
void launch_get_F(const DevMesh& d, double* F, const int32_t* eold, hipStream_t st);
void launch_get_dir(const DevMesh& d, double* out, const int32_t* eold, hipStream_t st);
void launch_scatter_F(const DevMesh& d, hipStream_t st);
void launch_solve(const DevMesh& d, const SolvePlan& pl, int add_pin, double* x, int check_done, hipStream_t st);
void launch_set_pins(const DevMesh& d, hipStream_t st);
void launch_bone_sync(const DevMesh& d, hipStream_t st);
void launch_iteration(const DevMesh& d, const SolvePlan& pl, hipStream_t st);
void launch_iteration_phased(const DevMesh& d, const SolvePlan& pl, hipStream_t st, hipEvent_t* ev);
void launch_evaluate(const DevMesh& d, hipStream_t st);
void launch_class(int k, const DevMesh& d, const SolvePlan& pl, hipStream_t st);
// adjoint building blocks
// check_done 1: every kernel returns at once while ctl->done is set
void launch_sweeps(const DevMesh& d, const SolvePlan& pl, double* x, hipStream_t st, int check_done = 0);
void launch_field_solve(const DevMesh& d, const SolvePlan& pl, const double* V, double* x, hipStream_t st,
                        int check_done = 0);
void launch_weighted_grad(const DevMesh& d, const double* x, double* out, hipStream_t st);
void launch_hvp(const DevMesh& d, const double* V, const double* x, double* out, double* part, hipStream_t st);
// adjoint conjugate gradients; alpha, beta, r.z and the stop test live in the
// control block (k_cg_scalar), so the steps need no host round trip
enum { kCgInitRz, kCgInitR, kCgAlpha, kCgResid, kCgBeta };
struct CgWork {
  double *lam, *r, *z, *p, *hp, *ypart, *part, *vx, *rbar;
};
void launch_cg_update(const DevMesh& d, const double* P, const double* HP, double* lam, double* r, double* part,
                      hipStream_t st);
void launch_cg_dir(const DevMesh& d, const double* Z, double* P, hipStream_t st);
void launch_cg_scalar(const DevMesh& d, const double* part, int what, hipStream_t st);
void launch_cg_begin(const DevMesh& d, int max_steps, hipStream_t st);
// one step (field solve, Hp, alpha, update, |r|, preconditioner, beta, p);
// every kernel returns at once once ctl->done is set
void launch_cg_step(const DevMesh& d, const SolvePlan& pl, const CgWork& w, hipStream_t st);
// z = Htilde^{-1} r (world-frame F fields [9][m]) with the iteration's blocks and
// Woodbury factor; rbar ([9][m]) is scratch.
void launch_precond(const DevMesh& d, const double* r, double* z, double* ypart, double* part, double* rbar,
                    hipStream_t st, int check_done = 0);
// contact loop: penalty forces of the free vertices into d.rhs (block partials
// of |f|^2, contact_blocks(d) of them); q += x2, zc += z; the pending step
// together with zc (then none is pending)
int contact_blocks(const DevMesh& d);
// device eigenpairs of L_ff: blocks of kEigCols columns in packs of three
// ([n][3] vertex fields, pstride doubles apart); partial and reduced column
// products, X = Y W, residual norms, and L_ff x (into d.rhs, V scratch [9][m])
void launch_lff_apply(const DevMesh& d, const double* x, double* V, hipStream_t st);
int eig_gram_blocks(int nf);
void launch_eig_gram(int nf, int64_t pstride, const double* A, const double* B, double* part, double* out,
                     hipStream_t st);
void launch_eig_mul(int nf, int64_t pstride, const double* Y, const double* W, double* X, hipStream_t st);
void launch_eig_resid(int nf, int64_t pstride, const double* X, const double* LX, const double* lam, int ncols,
                      double* part, double* out, hipStream_t st);
void launch_contact_force(const DevMesh& d, const double* obs, int np, int ns, double k, double* part,
                          hipStream_t st);
void launch_contact_accum(const DevMesh& d, const double* x2, const double* z, double* zc, hipStream_t st);
void launch_accept_contact(const DevMesh& d, const double* zc, hipStream_t st);
void launch_adj_da(const DevMesh& d, const double* lam, double* part, hipStream_t st);
void launch_group_sum(const DevMesh& d, const double* per, double scale, double* out, hipStream_t st);

}  // namespace emu
