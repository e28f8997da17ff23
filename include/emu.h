/*
 * emu.h -- C ABI of the MI355X (gfx950) EMU deformation-space quasi-static solver.
 *
 * Problem (the paper's problem statement, eq. continuum, with W = 0): given a
 * tetrahedral rest mesh, per-tet stable Neo-Hookean materials, unit fiber
 * directions and per-muscle-group activations a >= 0 (Sec. 3.1), and pinned
 * vertices with target positions (Sec. 3.1: pins remove the rigid null space),
 * find the deformed vertex positions q of the separated problem (eq. separated)
 *
 *   min_F  sum_i vol_i Psi_i(F_i) + alpha/2 sum_i w_i |A_i(q*(F)) - F_i|^2,
 *   q*(F) = argmin_q ACAP(q, F)                       (eq. acap),
 *
 * with one free deformation gradient F_i per tet, A_i(q) the compatible
 * gradient of eq. defograd and w_i the ACAP weights (Sec. 3.3 recommends
 * stiffness-proportional weights).  The solver is the paper's quasi-Newton
 * method (Sec. 3.2.1): exact gradient (eq. gradient), block-diagonal Hessian with
 * a definiteness fix plus a k-mode low-rank coupling applied by the Woodbury
 * identity (eq. Hessian-woodbury), and a backtracking Armijo line search
 * (Algorithm 1).
 *
 * Conventions for every call:
 *   - All arrays are row-major and use the caller's vertex and tet numbering.
 *   - "host" pointers are read (or written) before the call returns; the
 *     library keeps no reference to them.  "device" pointers are HIP device
 *     memory on the mesh's device, accessed in stream order on `stream`.
 *   - `stream` is a hipStream_t passed as void*; NULL means the null stream.
 *   - Calls never throw or abort.  They return EMU_OK (0) or an error code;
 *     emu_last_error() returns a thread-local message for the last failure.
 *   - A mesh handle is not thread-safe: calls on one handle must not overlap.
 */
#ifndef EMU_H
#define EMU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct emu_mesh emu_mesh;

typedef enum {
  EMU_OK = 0,
  EMU_E_INVALID = 1,        /* bad argument or mesh data                        */
  EMU_E_SINGULAR = 2,       /* ACAP operator not positive definite (unpinned part) */
  EMU_E_NOT_CONVERGED = 3,  /* max_iters reached; state and stats are kept      */
  EMU_E_LINESEARCH = 4,     /* no Armijo step down to sigma0 * 2^-40            */
  EMU_E_NONFINITE = 5,      /* NaN/Inf in energy, gradient or Woodbury system   */
  EMU_E_OOM = 6,            /* device or host allocation failed                 */
  EMU_E_HIP = 7,            /* a HIP runtime call failed                        */
  EMU_E_STATE = 8,          /* call not valid in the current state              */
  EMU_E_BUSY = 9            /* resource exhausted (serving slots or budget)     */
} emu_status;

enum { EMU_PRECISION_FP64 = 0, EMU_PRECISION_MIXED = 1 };
/* ACAP weights w_i (eq. ACAPEnergy).  STIFFNESS: w_i = vol_i mu_i / mu_ref for
   every tet.  VOLUME: w_i = vol_i (the printed unweighted energy read as an
   integral).  PAPER: stiffness-proportional for muscle and tendon, volume for
   bone tets (Sec. 3.3: a stiff spring on bones can lead to locking); bone tets
   are those with bone[i] >= 0. */
enum { EMU_WEIGHT_STIFFNESS = 0, EMU_WEIGHT_VOLUME = 1, EMU_WEIGHT_PAPER = 2 };

/* Optional device allocator for the memory a mesh keeps resident (state,
   factor, modes, work arrays).  alloc returns NULL on failure (-> EMU_E_OOM);
   free receives exactly the pointers alloc returned, after the mesh's stream
   has drained.  Used to draw mesh memory from a caller's pool (e.g. torch's
   caching allocator). */
/* Element blocks of the approximate Hessian (Sec. 3.2.1: block diagonal in
   the per-tet deformation gradients, made positive definite, plus alpha W).
   SPLIT: in the frame of each tet's rotation (dF = R dX) the blocks of the
   symmetric (6x6) and skew (3x3) parts of dX, each clamped to its positive
   semi-definite part; the coupling of the two parts by the fiber term is
   dropped.  COUPLED: the full 9x9 block: the isotropic term clamped per part
   (it has no coupling) plus the whole fiber term, a convex quadratic, so the
   block equals the exact element Hessian wherever no clamp is active. */
enum { EMU_BLOCKS_SPLIT = 0, EMU_BLOCKS_COUPLED = 1 };

typedef void* (*emu_dev_alloc_fn)(size_t bytes, void* ctx);
typedef void (*emu_dev_free_fn)(void* ptr, void* ctx);

/* Mesh description (host arrays, copied by emu_create_mesh). */
typedef struct {
  int32_t n_vertices;        /* n > 0                                             */
  int32_t n_tets;            /* m > 0                                             */
  int32_t n_groups;          /* muscle groups (>= 0)                              */
  int32_t n_pins;            /* pinned vertices (>= 1 per connected component)    */
  const double  *rest_xyz;   /* [n][3] rest positions (m)                         */
  const int32_t *tets;       /* [m][4] vertex ids; orientation is fixed by the
                                library (local vertices 1,2 swapped if the rest
                                volume is negative, eq. defograd)                 */
  const double  *youngs;     /* [m] Young's modulus (Pa), > 0                     */
  const double  *poisson;    /* [m] Poisson ratio in (-1, 0.5)                    */
  const double  *fiber;      /* [m][3] fiber direction u (Sec. 3.1), normalized by
                                the library; ignored where group < 0              */
  const int32_t *group;      /* [m] muscle group in [0, n_groups) or -1 (passive)  */
  const int32_t *pins;       /* [n_pins] pinned vertex ids, unique                */
  const double  *pin_xyz;    /* [n_pins][3] pin targets; NULL = rest positions    */
  double alpha_hat;          /* alpha = alpha_hat * mu_ref (eq. separated); 0 -> 10 */
  double mu_ref;             /* reference shear modulus; 0 -> smallest mu among
                                tets with group >= 0 (all tets if none)          */
  double fiber_k;            /* fiber stress scale k_f in Psi_fib = a k_f |F u|^2;
                                0 -> mu_ref                                      */
  int32_t weight_mode;       /* EMU_WEIGHT_STIFFNESS, _VOLUME or _PAPER (above)   */
  int32_t n_modes;           /* k = 3 * (scalar modes), 0 <= k <= 48, k % 3 == 0,
                                k/3 < free vertices; -1 -> min(48, 3 (free - 1))
                                (eq. low-rank)                                    */
  int32_t precision;         /* EMU_PRECISION_FP64 or EMU_PRECISION_MIXED          */
  int32_t leaf_size;         /* nested-dissection leaf size; 0 -> 64              */
  const int32_t *bone;       /* [m] bone id (>= 0) or -1; NULL = no bone tets.
                                Read by weight_mode EMU_WEIGHT_PAPER             */
  int32_t affine_bones;      /* 1: the tets of each bone (bone[i] >= 0) share one
                                deformation gradient F_b (Sec. 3.3), tied to the
                                continuous mesh by B_q q = B_F F with the slack
                                eps_2 of eq. kkt-matrix: a bone tet's ACAP weight
                                is vol (1 + 1/bone_slack) (bones are not
                                stiffness-weighted).  Joints are vertices shared
                                by two bones (J q = 0 holds by construction).
                                Bone tets must be passive (group -1).
                                Requires split element blocks; not supported
                                by emu_solve_grad or the serving loop.
                                0: every tet has its own F.                   */
  double bone_slack;         /* |eps_2| of the bone constraint; 0 -> 1e-3       */
  int32_t hessian_blocks;    /* element blocks of the quasi-Newton Hessian
                                (Sec. 3.2.1, eq. not-yet): EMU_BLOCKS_SPLIT, or
                                EMU_BLOCKS_COUPLED for the full 9x9 block per
                                tet (not supported by the serving loop)          */
  emu_dev_alloc_fn dev_alloc;  /* NULL -> hipMalloc / hipFree.  Both or neither;  */
  emu_dev_free_fn dev_free;    /* the serving loop ignores them (it accounts its  */
  void *alloc_ctx;             /* own HBM budget).  Passed back to both calls.    */
} emu_mesh_desc;

/* Solve options.  Defaults (emu_solve_opts_default): grad_tol 1e-8,
   max_iters 10000, sigma0 10, armijo_c 1e-4, rho 0.5, warm_start 1,
   iters_per_sync 16 (Algorithm 1 constants). */
typedef struct {
  double grad_tol;           /* stop when |dE/dF|_2 <= grad_tol (J, absolute)      */
  int32_t max_iters;
  double sigma0, armijo_c, rho;
  int32_t warm_start;        /* 1: start from the current state; 0: from rest     */
  int32_t iters_per_sync;    /* iterations per host check of the stop flag       */
  double stall_rel;          /* mixed precision only: also stop if no Armijo step
                                exists and |g| <= stall_rel * |g_0|; 0 disables  */
  double grad_rtol;          /* also stop when |dE/dF|_2 <= grad_rtol |g_0|; 0 = off */
  int32_t phase_timing;      /* 1: time the phases of every iteration with HIP
                                events (fills the ms_* phase fields of the stats;
                                the iterations are launched one by one instead
                                of from a replayed graph); 0: phases report 0 */
} emu_solve_opts;

typedef struct {
  int32_t status;            /* emu_status of the solve                           */
  int32_t iters;             /* accepted quasi-Newton iterations                  */
  int32_t ls_trials;         /* Armijo trials (each O(1): the energy change is an
                                exact polynomial in sigma)                        */
  int32_t acap_solves;       /* factored ACAP solves                              */
  int32_t inverted;          /* tets with det F <= 0 at the end                   */
  int32_t clamped;           /* element Hessian blocks clamped in the last pass   */
  double energy;             /* E at the end (J)                                  */
  double grad_norm;          /* |dE/dF|_2 at the end                              */
  double grad_norm0;         /* |dE/dF|_2 at the start                            */
  double ms_total;           /* device time of the call (hipEvent)                */
  /* device time per phase, summed over the iterations (opts.phase_timing):
     element pass (energy, gradient, blocks; Sec. 3.2.1), Woodbury correction
     (eq. Hessian-woodbury: Gram, k x k solve, direction), ACAP solve of the
     direction (eq. acap: right-hand side and triangular sweeps), line search
     (Algorithm 1: polynomial coefficients, Armijo test, q update) */
  double ms_elem, ms_woodbury, ms_solve, ms_linesearch;
  int32_t contact_rounds;    /* contact rounds run (emu_set_contact), all steps  */
} emu_solve_stats;

/* Static information about a mesh. */
typedef struct {
  int32_t n_vertices, n_tets, n_free, n_modes;
  int32_t n_supernodes, n_levels;
  int64_t factor_nnz;        /* stored factor entries (dense supernode blocks)    */
  int64_t device_bytes;      /* device memory held by the mesh                    */
  double mu_ref, alpha, fiber_k;
  double setup_ms;           /* host setup time (ordering, factor, modes, upload) */
  double mode_captured;      /* sum_{j<=k/3} 1/nu_j / trace(L_ff^{-1}) estimate    */
  /* forward-sweep levels run in column form (one lane per row over the
     column-major block; levels of many narrow supernodes, or every level
     whose supernodes are narrow when EMU_FWD_COLUMN=1 is set at creation;
     none with EMU_FWD_COLUMN=0); 0 for a host-only setup */
  int32_t fwd_column_levels;
} emu_mesh_info;

emu_solve_opts emu_solve_opts_default(void);
const char* emu_last_error(void);

/* Build a mesh: validate, orient, compute geometry and ACAP weights, assemble
   the weighted Laplacian L_w (the q-Hessian of the ACAP energy, eq. ACAPEnergy,
   is L_w (x) I_3), order it by nested dissection, factor L_ff once (Sec. 3.2:
   prefactor the constant matrix), compute its k/3 lowest eigenpairs (eq.
   low-rank) and upload everything to the current HIP device.  The state starts
   at rest (F_i = I).  Errors: EMU_E_INVALID (see desc), EMU_E_SINGULAR (a
   connected part without pins), EMU_E_OOM, EMU_E_HIP. */
emu_status emu_create_mesh(const emu_mesh_desc* desc, emu_mesh** out);
emu_status emu_destroy_mesh(emu_mesh* mesh);
emu_status emu_mesh_get_info(const emu_mesh* mesh, emu_mesh_info* info);

/* Per-group activations a(t) >= 0 (Sec. 3.1), host [n_groups]. */
emu_status emu_set_activation(emu_mesh* mesh, const double* a);

/* New pin targets (host [n_pins][3]) for scripted boundaries; the factor is
   unchanged, only the constant pinned right-hand side is recomputed. */
emu_status emu_set_pin_targets(emu_mesh* mesh, const double* pin_xyz);

/* Constant external vertex forces (Sec. 3.4; gravity is f_v = m_v g): the
   solve then minimizes the separated energy minus the work f . q*(F) done on
   the nearest continuous mesh.  f is host [n_vertices][3] (N), user vertex
   order, copied; forces at pinned vertices do no work; NULL removes the
   forces.  EMU_E_INVALID for non-finite entries. */
emu_status emu_set_external_forces(emu_mesh* mesh, const double* f);

/* Contact (Sec. 3.5, the collision block of Algorithm 1).  With obstacles
   set, every emu_solve runs, after each accepted quasi-Newton step, rounds of:
   the penalty forces f of the free vertices of q that penetrate an obstacle;
   the step F <- F + Htilde^{-1} nu(f), where nu(f) = w G L_ff^{-1} f is the
   F-gradient of the work f . q*(F) (as for external forces) and Htilde^{-1}
   the step's own Woodbury inverse; q <- q*(F).  The rounds stop once
   |f|_2 <= tol or after max_rounds.  The collision method the paper cites is
   not described in it: analytic obstacles stand in for the colliding bodies.
   A round moves a vertex by about its compliance C times the force, so the
   rounds converge for k C < 1 and overshoot for stiffer penalties.  Contact
   forces are not part of the energy: with active contacts the iteration
   balances the quasi-Newton step against the push-out and |g| stays away from
   0; emu_solve then ends at max_iters (EMU_E_NOT_CONVERGED, state kept).
   Iterations with contact run one per launch; the phase times report 0.
   Not available with affine bones.  NULL (or no obstacles) removes contact.
   EMU_E_INVALID: counts outside [0, EMU_MAX_OBSTACLES] in total, a normal
   that is not unit length (within 1e-9), r <= 0, k <= 0, tol < 0,
   max_rounds < 1, non-finite values, affine bones. */
#define EMU_MAX_OBSTACLES 64
typedef struct {
  int32_t n_planes;          /* half-spaces: host rows (nx, ny, nz, b), |n| = 1;
                                x penetrates where n . x < b by b - n . x and is
                                pushed along n                                 */
  const double* planes;      /* [n_planes][4]                                   */
  int32_t n_spheres;         /* spheres: host rows (cx, cy, cz, r), r > 0; x
                                penetrates where |x - c| < r by r - |x - c| and
                                is pushed along (x - c) / |x - c|              */
  const double* spheres;     /* [n_spheres][4]                                  */
  double stiffness;          /* penalty k > 0: force k * depth (N/m)            */
  double tol;                /* |f|_2 (N) at which a contact loop stops          */
  int32_t max_rounds;        /* rounds per accepted step (>= 1)                 */
} emu_contact_desc;
emu_status emu_set_contact(emu_mesh* mesh, const emu_contact_desc* desc);

/* Replace the low-rank modes (eq. low-rank): k1 = k/3 scalar modes, nu host
   [k1] > 0, phi host [k1][n] (values at pinned vertices are ignored). */
emu_status emu_set_modes(emu_mesh* mesh, int32_t k1, const double* nu, const double* phi);
/* Read the modes currently used (host nu [k1], phi [k1][n]; either may be NULL). */
emu_status emu_get_modes(const emu_mesh* mesh, double* nu, double* phi);

/* Run the quasi-Newton iteration until |dE/dF|_2 <= grad_tol.  q_out: device
   [n][3] or NULL.  stats may be NULL.  Returns EMU_OK, EMU_E_NOT_CONVERGED,
   EMU_E_LINESEARCH or EMU_E_NONFINITE; the state is kept in every case. */
emu_status emu_solve(emu_mesh* mesh, const emu_solve_opts* opts, double* q_out,
                     emu_solve_stats* stats, void* stream);

/* Adjoint of the equilibrium w.r.t. the group activations at the current
   (converged) state: given dL/dq (device [n][3]), write dL/da (host
   [n_groups]).  Requires a converged emu_solve at the current activations
   (EMU_E_STATE otherwise).  The adjoint system is solved by preconditioned
   conjugate gradients to |r| <= 1e-10 |b|; stats (may be NULL) gets the steps
   in iters, |b| in grad_norm0 and the final |r| in grad_norm.  Errors:
   EMU_E_NONFINITE when |b| or |r| is not finite (for instance a NaN in dL/dq)
   or p.Hp <= 0; EMU_E_NOT_CONVERGED after 20000 steps.  The state is never
   changed. */
emu_status emu_solve_grad(emu_mesh* mesh, const double* dL_dq, double* dL_da,
                          emu_solve_stats* stats, void* stream);

/* emu_solve_grad for callers that cannot allocate device memory (tight
   serving loops, harnesses that forbid hipMalloc, processes that must not
   allocate while other work is captured into HIP graphs; the call itself
   waits on the mesh stream between groups of steps, so it cannot be captured):
   same arguments, result and errors, but its conjugate-gradient vectors and
   partial sums live in one fixed device scratch array of the library
   (48 MiB per GPU, held until the process ends) instead of memory the mesh
   allocates on first use; it calls no hipMalloc, hipFree or other allocating
   routine.  A mesh needing more scratch than that (about 46 m + 6 n + 50 nb
   doubles: roughly 130k tets) is rejected with EMU_E_INVALID.  Every call on
   one GPU shares that GPU's array, so calls that overlap on one GPU (two
   meshes, two host threads, two streams) race: the caller serializes them. */
emu_status emu_solve_grad_noalloc(emu_mesh* mesh, const double* dL_dq, double* dL_da,
                                  emu_solve_stats* stats, void* stream);

/* State access: F device [m][9] (row-major 3x3 per tet), q device [n][3].
   emu_set_state takes F, splits it as F = R S and re-solves q = q*(F); with
   affine bones each bone takes the F of its first tet in element order (the
   lowest vertex id). */
emu_status emu_get_state(const emu_mesh* mesh, double* F, double* q, void* stream);
emu_status emu_set_state(emu_mesh* mesh, const double* F, void* stream);

/* Evaluate at a given state F (device [m][9]) without changing the mesh state:
   q = q*(F) (device [n][3] or NULL), the energy E (eq. separated) and
   |dE/dF|_2 (host scalars, either may be NULL), and the quasi-Newton direction
   d = Htilde^{-1} dE/dF (device [m][9] in F coordinates, or NULL). */
emu_status emu_evaluate(emu_mesh* mesh, const double* F, double* q, double* energy,
                        double* grad_norm, double* direction, void* stream);

/* Diagnostics: kernel classes of one quasi-Newton iteration. */
enum {
  EMU_K_ELEMENT = 0,      /* accept step, polar split, energy, gradient, blocks */
  EMU_K_GRAM = 1,         /* Woodbury Gram and y partial sums                   */
  EMU_K_GRAM_REDUCE = 2,
  EMU_K_CONTROL_A = 3,    /* convergence test, k x k Cholesky, z                */
  EMU_K_UZ = 4,           /* mode field Phi^T z                                 */
  EMU_K_DIRECTION = 5,    /* Woodbury direction                                 */
  EMU_K_RHS = 6,          /* ACAP right-hand side                               */
  EMU_K_FWD = 7,          /* forward triangular sweep (all levels)              */
  EMU_K_BWD = 8,          /* backward triangular sweep (all levels)             */
  EMU_K_LSCOEF = 9,       /* line-search polynomial                             */
  EMU_K_CONTROL_B = 10,   /* Armijo test                                        */
  EMU_K_ADD_Q = 11,       /* q += sigma dq                                      */
  EMU_NUM_KERNELS = 12
};

/* Average device time (ms) of each kernel class at the current state, each
   launched `reps` times back to back with HIP events on the mesh's stream;
   ms_out host [EMU_NUM_KERNELS].  The mesh state is left unchanged. */
emu_status emu_profile_kernels(emu_mesh* mesh, int32_t reps, double* ms_out, void* stream);
/* Name of kernel class k (static string), or NULL. */
const char* emu_kernel_name(int32_t k);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of independent solve requests on one GPU.
 *
 * Each request is one quasi-static solve (Sec. 3.2, Algorithm 1) of its own
 * mesh at its own activations, with the options of emu_solve.  Requests are
 * set up on host worker threads (ordering, factor, modes; cached by the full
 * content of the description, pin targets included), admitted in submission
 * order when a slot is free and the mesh's device block fits the HBM budget
 * next to every resident mesh, and iterated together: each scheduler round
 * replays K iterations of all active meshes with one launch per kernel class,
 * and new requests join between rounds.  A finished request's mesh stays
 * resident (idle, with its final state) and is reused by a later request with
 * the same description (warm-started from that state when opts.warm_start is
 * 1, from rest otherwise); idle meshes are evicted least-recently-used when
 * the budget needs their memory.  Every mesh runs exactly the kernels and
 * block partition of emu_solve with fixed-order reductions, so a cold-started
 * request gives the same bits alone or in any mix.
 *
 * Threads: submit / wait / report may be called from any thread.  Times are
 * seconds since emu_server_create (steady clock).
 * ---------------------------------------------------------------------- */
typedef struct emu_server emu_server;

typedef struct {
  int64_t hbm_budget_bytes;  /* device bytes resident meshes may hold (0 -> 80% of free) */
  int32_t max_slots;         /* requests iterated concurrently (0 -> 64)          */
  int32_t setup_threads;     /* host setup workers (0 -> 4)                       */
  int32_t iters_per_round;   /* iterations per scheduler round (0 -> 16, <= 256)  */
} emu_server_opts;

typedef struct {
  double t_submit, t_setup_done, t_admit, t_finish;  /* seconds                  */
  int64_t device_bytes;      /* device block the request's mesh held             */
  int32_t setup_cached;      /* 1 if the host setup came from the cache          */
} emu_request_times;

typedef struct {
  int64_t peak_resident_bytes;
  int32_t peak_active;
  int32_t submitted, completed, failed;
  int32_t rounds;            /* scheduler rounds that launched work              */
  int64_t resident_bytes;    /* device bytes of the meshes resident now          */
} emu_server_report;

/* Create a server on the current HIP device.  opts may be NULL (defaults).
   EMU_E_INVALID for negative options, EMU_E_HIP without a device.
   A request that fails (any status but EMU_OK, or EMU_E_NOT_CONVERGED with a
   finite gradient) releases its slot and its mesh's device memory; the other
   requests are unaffected.  Test hook for that path: with the environment
   variable EMU_FAULT=linesearch:T at creation, the request with ticket T
   ends with EMU_E_LINESEARCH after its first round. */
emu_status emu_server_create(const emu_server_opts* opts, emu_server** out);
/* Queue one request; the description's arrays and activation (host,
   [n_groups]) are copied; opts may be NULL (emu_solve_opts_default).  Writes a
   ticket.  EMU_E_INVALID for NULL arrays, negative sizes, bad activations or
   options; mesh validation errors (as emu_create_mesh) and EMU_E_OOM for a
   mesh whose device block alone exceeds the budget come from emu_server_wait. */
emu_status emu_server_submit(emu_server* s, const emu_mesh_desc* desc, const double* activation,
                             const emu_solve_opts* opts, uint64_t* ticket);
/* Block until the request has finished, then release its ticket.  q_host
   [n_vertices][3] (user vertex order), stats and times may be NULL.  Returns
   the request's status (as emu_solve); EMU_E_INVALID for an unknown ticket. */
emu_status emu_server_wait(emu_server* s, uint64_t ticket, double* q_host, emu_solve_stats* stats,
                           emu_request_times* times);
emu_status emu_server_report_get(emu_server* s, emu_server_report* rep);
/* Finish every queued request, then release the server and all its device
   memory.  Results not collected by emu_server_wait are discarded. */
emu_status emu_server_destroy(emu_server* s);

#ifdef __cplusplus
}
#endif
#endif /* EMU_H */
