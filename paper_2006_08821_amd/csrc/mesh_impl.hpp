// Internal definition of a device mesh, shared by the single-mesh C ABI
// (api.hip) and the serving loop (serve.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <cstddef>
#include <memory>
#include <string>
#include <vector>

#include "../../include/emu.h"
#include "device.hpp"
#include "host_setup.hpp"
#include "kernels.hpp"

#define HIPCHK(x)                                                                   \
  do {                                                                              \
    hipError_t e_ = (x);                                                            \
    if (e_ != hipSuccess)                                                           \
      throw emu::Error{EMU_E_HIP, std::string(#x) + ": " + hipGetErrorString(e_)}; \
  } while (0)

namespace emu {

const std::string& last_error_str();

// roctx range over a scope: marks the library's host-side phases (mesh setup,
// device eigenpairs, solves, contact rounds, adjoint, serving rounds) for
// rocprofv3 --marker-trace; no cost without a profiler attached.
struct Range {
  explicit Range(const char* what) { roctxRangePushA(what); }
  ~Range() { roctxRangePop(); }
  Range(const Range&) = delete;
  Range& operator=(const Range&) = delete;
};

// Everything a mesh uploads at creation, laid out in one device block: the
// piece for DevMesh member `slot` (a byte offset into DevMesh, or one of the
// extra slots below) starts at `offset` and is filled from `data` (left
// uninitialised when `data` is empty).  A pure function of the host setup, so
// the serving loop prepares it once per distinct mesh.
struct DevImage {
  static constexpr size_t kSlotEold = (size_t)1 << 30;
  static constexpr size_t kSlotVold = kSlotEold + 1;
  struct Piece {
    size_t slot;
    size_t offset;
    size_t bytes;
    std::vector<char> data;
  };
  std::vector<Piece> pieces;
  size_t total = 0;   // bytes of the block
  DevMesh d{};        // sizes and scalars (pointers are set at upload)
  SolvePlan plan;
};
std::shared_ptr<const DevImage> prepare_image(const HostMesh& hm);

}  // namespace emu

struct emu_mesh {
  std::shared_ptr<emu::HostMesh> hmp;
  emu::HostMesh& hm;
  std::shared_ptr<const emu::DevImage> img;
  emu::DevMesh d{};
  emu::SolvePlan plan;
  int device = 0;
  hipStream_t st = nullptr;
  bool own_stream = true;
  hipEvent_t ev_a = nullptr, ev_b = nullptr, ev_t0 = nullptr, ev_t1 = nullptr;
  std::vector<void*> allocs;
  int64_t bytes = 0;
  // caller's device allocator (emu_mesh_desc.dev_alloc); null: hipMalloc
  emu_dev_alloc_fn dev_alloc = nullptr;
  emu_dev_free_fn dev_free = nullptr;
  void* alloc_ctx = nullptr;
  int32_t* d_eold = nullptr;
  int32_t* d_vold = nullptr;
  emu::Ctl* h_ctl = nullptr;  // pinned host copy
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  int graph_iters = 0;
  std::vector<double> act;
  bool converged = false;
  // external forces: L_ff^{-1} f (factor order, free vertices) and the
  // constant part of the work, f . q* = sum_i nu_i . F_i + ext_c0
  std::vector<double> vext;
  double ext_c0 = 0;
  // backup of the state for emu_evaluate
  double *R_bak = nullptr, *S_bak = nullptr, *q_bak = nullptr;
  // adjoint work arrays, one block (allocated on the first emu_solve_grad)
  double* a_work = nullptr;
  // phase-timing events (emu_solve_opts.phase_timing), 5 per iteration of a sync block
  std::vector<hipEvent_t> t_ev;
  // contact (emu_set_contact): obstacle rows (planes, then spheres), the
  // parameters, the work arrays of the rounds and a pinned host copy of the
  // force partials (all allocated on the first call)
  int32_t c_np = 0, c_ns = 0, c_max_rounds = 0;
  double c_k = 0, c_tol = 0;
  double* c_obs = nullptr;
  double* c_work = nullptr;
  double* c_host = nullptr;
  int32_t c_rounds = 0;

  explicit emu_mesh(std::shared_ptr<emu::HostMesh> p) : hmp(std::move(p)), hm(*hmp) {}
  emu_mesh(const emu_mesh&) = delete;
  emu_mesh& operator=(const emu_mesh&) = delete;

  template <typename T>
  T* dalloc(size_t count) {
    void* p = nullptr;
    size_t nb = std::max<size_t>(1, count * sizeof(T));
    if (dev_alloc) {
      p = dev_alloc(nb, alloc_ctx);
      if (!p) throw emu::Error{EMU_E_OOM, "the caller's device allocator returned NULL"};
    } else {
      hipError_t e = hipMalloc(&p, nb);
      if (e != hipSuccess) throw emu::Error{EMU_E_OOM, std::string("hipMalloc failed: ") + hipGetErrorString(e)};
    }
    allocs.push_back(p);
    bytes += (int64_t)nb;
    return (T*)p;
  }
  template <typename T>
  T* upload(const std::vector<T>& v) {
    T* p = dalloc<T>(v.size());
    if (!v.empty()) HIPCHK(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return p;
  }
  ~emu_mesh() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    if (st) (void)hipStreamSynchronize(st);
    for (void* p : allocs) {
      if (dev_free) dev_free(p, alloc_ctx);
      else (void)hipFree(p);
    }
    if (h_ctl) (void)hipHostFree(h_ctl);
    if (c_host) (void)hipHostFree(c_host);
    if (t_ev.size())
      for (hipEvent_t e : t_ev) (void)hipEventDestroy(e);
    if (ev_a) (void)hipEventDestroy(ev_a);
    if (ev_b) (void)hipEventDestroy(ev_b);
    if (ev_t0) (void)hipEventDestroy(ev_t0);
    if (ev_t1) (void)hipEventDestroy(ev_t1);
    if (st && own_stream) (void)hipStreamDestroy(st);
  }
};

namespace emu {
// Allocate and fill the device block of `img` on `stream` (the mesh's own
// stream is created when `stream` is null).  Leaves the state uninitialised.
void upload_image(emu_mesh* M, std::shared_ptr<const DevImage> img, hipStream_t stream);
void init_ctl(emu_mesh* M, const emu_solve_opts& o, int eval_only);
void fresh_solve(emu_mesh* M);
void fill_stats(const emu::Ctl& c, emu_solve_stats* s, float ms);
void launch_to_user_q(emu_mesh* M, double* out);
// The modes of a mesh uploaded without them (host_setup without modes): the
// cached ones of its host setup, else computed on the device (host solver as
// the fallback) and kept in the host setup for later copies of the mesh.
void ensure_modes_of(emu_mesh* M);
}  // namespace emu
