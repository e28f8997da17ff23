// Device-side data of one mesh and the control block of the iteration.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace emu {

constexpr int kBlock = 256;        // threads per workgroup (4 wave64)
constexpr int kMaxK1 = 16;         // scalar low-rank modes (k = 3 * k1 <= 48)
constexpr int kGramEntries = 6 * 256 + 48;   // 6 coordinate-pair 16x16 blocks + y
constexpr int kLsTerms = 6;        // coefficients of the line-search polynomial
// Triangular-sweep work items: 32 rows (8 lanes per row) or, flagged by
// kItemWideBit in the first row, 8 rows (32 lanes per row).  Items of a level
// with fewer than kWideLevelItems 32-row items use the wide form for
// supernodes whose rows are at least kWideRowMin long.
constexpr int kItemWideBit = 1 << 30;
constexpr int kWideLevelItems = 256;
constexpr int kWideRowMin = 64;
// Forward levels whose supernodes are all at most kColW wide and that have at
// least kColMinItems such items run in column form instead: one wave per
// item of kColRows rows (flag kItemColBit in the first row), one lane per
// row, walking the columns of the column-major block.  With fewer items (two
// waves per SIMD) the 8-lane rows of the row form spread the work wider.
constexpr int kItemColBit = 1 << 29;
constexpr int kColW = 128;
constexpr int kColRows = 64;
constexpr int kColMinItems = 2048;
constexpr int kNarrowChunk = 512;     // vector chunk of the narrow sweep variant (12 KB of LDS)
constexpr int kNarrowFwdW = 64;       // widest supernode of a forward level run narrow
constexpr int kNarrowBwdH = 256;      // tallest supernode of a backward level run narrow
constexpr int kEigCols = 33;          // columns of the device eigen block (11 packs of 3)

// Iteration control block (device memory, one per mesh).
struct Ctl {
  int32_t done;        // 1: every kernel of the iteration returns immediately
  int32_t status;      // emu_status
  int32_t iter;        // accepted iterations
  int32_t trials;      // Armijo trials
  int32_t solves;      // factored ACAP solves
  int32_t max_iters;
  int32_t eval_only;   // 1: never stop on convergence (single evaluation)
  int32_t clamped;     // blocks clamped in the last element pass
  int32_t inverted;    // tets with det F <= 0 in the last element pass
  int32_t chol_fail;   // Woodbury systems that were not SPD (fallback z = 0)
  int32_t pad0, pad1;
  double sigma;        // accepted step of the previous iteration (0: none)
  double tol2;         // grad_tol^2
  double gnorm2;       // |dE/dF|^2 of the last element pass
  double gnorm0_2;     // at the first pass of the solve
  double energy;
  double gtp;          // g . p of the last direction
  double sigma0, armijo_c, rho;
  double stall_rel;
  double rtol2;        // relative stop: |g|^2 <= rtol2 |g_0|^2
  // conjugate gradients of the adjoint (set and read by k_cg_scalar)
  double cg_rz;        // r . z of the current residual
  double cg_alpha, cg_beta;
  double cg_rnorm, cg_bnorm, cg_tol;  // |r|, |b|, stop at |r| <= cg_tol
  int32_t cg_it, cg_max;  // steps taken, step cap
};

// Plain pointers to every device array of a mesh (passed by value).
// A work item of a triangular sweep with its supernode's metadata, read by
// the workgroup in one scalar load: first row (forward) or column (backward),
// with kItemWideBit marking 32 lanes per row and kItemColBit a column-form
// item; supernode width w, height h, first column col0, first slot row of the
// children's contributions and the number of children (nslot), row offset,
// value offset; for column-form items, `end` is one past the last item of the
// level (a workgroup takes four consecutive items, one per wave).
struct SweepItem {
  int64_t valoff;
  int32_t first, w, h, col0, slotbase, nslot, rowoff, end;
};

struct DevMesh {
  int32_t n, nf, m, k1, npins, ngroups;
  int32_t nb;          // workgroups of the element passes (fixed: deterministic sums)
  int32_t nbg;         // workgroups of the Woodbury Gram pass
  int32_t mixed;       // FP32 element Hessian / Gram / direction
  int32_t has_ext;     // external vertex forces set (vext nonzero)
  int32_t coupled;     // 9x9 element blocks with the fiber coupling (else 6x6 + 3x3)
  int32_t nbones;      // affine bones (one shared F per bone; 0: none)
  int32_t nbt;         // tets in all affine bones
  int32_t pad_b;
  double alpha, kf;

  // elements, internal order, structure of arrays
  const int32_t* vid;     // [4][m] internal vertex ids
  const double* dminv;    // [9][m] rows of D_m^{-1}
  const double* vol;
  const double* mu;
  const double* lhat;
  const double* w;        // ACAP weights (beta = alpha w)
  const double* fib;      // [3][m]
  const int32_t* grp;     // [m]
  double* R;              // [9][m]
  double* S;              // [6][m]
  void* gbar;             // [9][m]  (double or float)
  void* Lf;               // [27][m] inverses of the 6x6 and 3x3 blocks (packed
                          // symmetric); coupled: [33][m], + K^{-1} (kernels.hip)
  double* p;              // [9][m]  step in the rotated (sym, skew) basis
  double* contrib;        // [m][12] ACAP right-hand-side contributions

  // vertices, internal order (free in factor order, then pinned)
  double* q;              // [n][3]
  double* dq;             // [n][3]
  double* uz;             // [n][3]
  const double* phi;      // [n][16]
  const double* nu;       // [16]
  const double* act;      // [ngroups]
  const double* vext;     // [n][3] L_ff^{-1} f at free vertices, 0 at pins
  const double* pin_rhs;  // [nf][3]
  const double* pin_xyz;  // [npins][3]  (internal ids nf..n-1)
  const int32_t* inc_ptr; // [nf+1]
  const int32_t* inc;     // element*4 + local vertex

  // factor (partitioned-inverse supernodes)
  const int32_t* rows;
  const double* vals;         // forward blocks [Linv; M], packed rows
  const double* tvals;        // the same blocks transposed (columns of L as rows)
  const int32_t* dst;        // per update row: its slot row (slotbase of the parent +
                             // child index * parent height + position in the parent front)
  const SweepItem* fwd_items;  // per forward work item: first row and its supernode
  const SweepItem* bwd_items;  // per backward work item: first column and its supernode
  double* rhs;               // [nf][3]
  double* ybuf;              // [nf][3]
  double* xbuf;              // [nf][3]
  double* slots;             // [sum nchildren * h][3] children's contributions per parent
                             // front position; rows no child writes stay zero

  // reductions
  double* part_e;            // [nb][2]
  double* part_g;            // [nb][2]
  int32_t* part_cnt;         // [nb][2]
  double* part_gram;         // [nbg][kGramEntries]
  double* gram;              // [kGramEntries]
  double* zbuf;              // [48]
  double* cfac;              // [48][48] Cholesky factor of the last Woodbury system
  int32_t* cfac_ok;          // [1] 1 if that factorization succeeded
  double* part_ls;           // [nb][2*kLsTerms]
  // affine bones: partial-sum slots nb .. nb + nbones - 1 (part_e, part_g,
  // part_cnt) and Gram rows nbg .. nbg + nbones - 1 belong to the bones
  const int32_t* bone_ptr;   // [nbones + 1] into bone_el
  const int32_t* bone_el;    // bone tets (internal ids, ascending per bone)
  const int32_t* bone_pos;   // [m] position of the tet in bone_el, -1 if not a bone tet
  double* bone_gbuf;         // [9][nbt] gradient of each bone tet (rotated frame, y coordinates)
  Ctl* ctl;
};

}  // namespace emu
