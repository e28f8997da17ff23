// Serving loop: continuous batching of independent quasi-static solves on one
// GPU (C ABI in include/emu.h, emu_server_*).
//
// * Host setup (ordering, supernodal factor, low-rank modes, device image) runs
//   on worker threads and is cached by the full content of the mesh
//   description, so repeated meshes are set up once.
// * A request is admitted, in submission order, when a slot is free and its
//   device block fits the HBM budget next to every resident mesh; idle meshes
//   (finished requests) stay resident with their last state and are reused by
//   a later request on the same mesh, or evicted least-recently-used when the
//   budget needs their memory.
// * Each round replays one HIP graph of K iterations over every active mesh:
//   one launch per kernel class covers all meshes (per-mesh block maps), the
//   triangular sweeps of all meshes advance level by level together, and each
//   mesh stops on its own device flag.  New requests join and finished ones
//   leave between rounds.
// * A mesh runs exactly the kernels and block partition of the single-mesh
//   solve, with fixed-order reductions, so its result does not depend on what
//   else is in the batch.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <future>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "mesh_impl.hpp"

namespace {

using Clock = std::chrono::steady_clock;

// Owned copy of a mesh description (every input of the host setup).
struct DescCopy {
  emu_mesh_desc d{};
  std::vector<double> rest, youngs, poisson, fiber, pin_xyz;
  std::vector<int32_t> tets, group, pins, bone;
  std::vector<char> key;  // canonical bytes of everything above
  uint64_t hash = 0;
};

template <typename T>
void copy_arr(std::vector<T>& dst, const T* src, int64_t count, const char* what) {
  if (count < 0) throw emu::Error{EMU_E_INVALID, std::string("negative size of ") + what};
  if (count > 0 && !src) throw emu::Error{EMU_E_INVALID, std::string("NULL array ") + what};
  dst.assign(src, src + count);
}

template <typename T>
void key_append(std::vector<char>& k, const std::vector<T>& v) {
  const uint64_t n = v.size();
  k.insert(k.end(), (const char*)&n, (const char*)&n + 8);
  k.insert(k.end(), (const char*)v.data(), (const char*)v.data() + n * sizeof(T));
}
template <typename T>
void key_scalar(std::vector<char>& k, T v) {
  k.insert(k.end(), (const char*)&v, (const char*)&v + sizeof(T));
}

void copy_desc(const emu_mesh_desc& s, DescCopy& c) {
  const int64_t n = s.n_vertices, m = s.n_tets, np = s.n_pins;
  copy_arr(c.rest, s.rest_xyz, 3 * n, "rest_xyz");
  copy_arr(c.tets, s.tets, 4 * m, "tets");
  copy_arr(c.youngs, s.youngs, m, "youngs");
  copy_arr(c.poisson, s.poisson, m, "poisson");
  copy_arr(c.fiber, s.fiber, 3 * m, "fiber");
  copy_arr(c.group, s.group, m, "group");
  copy_arr(c.pins, s.pins, np, "pins");
  if (s.pin_xyz) copy_arr(c.pin_xyz, s.pin_xyz, 3 * np, "pin_xyz");
  if (s.bone) copy_arr(c.bone, s.bone, m, "bone");
  c.d = s;
  c.d.bone = s.bone ? c.bone.data() : nullptr;
  // served meshes live in the server's own HBM budget
  c.d.dev_alloc = nullptr;
  c.d.dev_free = nullptr;
  c.d.alloc_ctx = nullptr;
  c.d.rest_xyz = c.rest.data();
  c.d.tets = c.tets.data();
  c.d.youngs = c.youngs.data();
  c.d.poisson = c.poisson.data();
  c.d.fiber = c.fiber.data();
  c.d.group = c.group.data();
  c.d.pins = c.pins.data();
  c.d.pin_xyz = s.pin_xyz ? c.pin_xyz.data() : nullptr;
  auto& k = c.key;
  key_scalar(k, s.n_vertices);
  key_scalar(k, s.n_tets);
  key_scalar(k, s.n_groups);
  key_scalar(k, s.n_pins);
  key_scalar(k, s.alpha_hat);
  key_scalar(k, s.mu_ref);
  key_scalar(k, s.fiber_k);
  key_scalar(k, s.weight_mode);
  key_scalar(k, s.n_modes);
  key_scalar(k, s.precision);
  key_scalar(k, s.leaf_size);
  key_scalar(k, s.hessian_blocks);
  key_append(k, c.rest);
  key_append(k, c.tets);
  key_append(k, c.youngs);
  key_append(k, c.poisson);
  key_append(k, c.fiber);
  key_append(k, c.group);
  key_append(k, c.pins);
  key_append(k, c.pin_xyz);
  key_append(k, c.bone);
  uint64_t h = 1469598103934665603ull;  // FNV-1a
  for (char ch : k) {
    h ^= (uint8_t)ch;
    h *= 1099511628211ull;
  }
  c.hash = h;
}

struct Setup {
  std::shared_ptr<emu::HostMesh> hm;
  std::shared_ptr<const emu::DevImage> img;
  emu_status code = EMU_OK;
  std::string msg;
};

struct CacheEntry {
  std::vector<char> key;
  std::shared_future<std::shared_ptr<const Setup>> fut;
  Clock::time_point used;
};

struct Request {
  uint64_t ticket = 0;
  DescCopy desc;
  std::vector<double> act;
  emu_solve_opts opts{};
  std::shared_ptr<const Setup> setup;
  bool cached = false;
  // results
  bool finished = false;
  emu_status status = EMU_OK;
  std::string msg;
  std::vector<double> q;
  emu_solve_stats stats{};
  emu_request_times times{};
  int rounds = 0;
};

// A device-resident mesh: active (owned by a request) or idle (kept for reuse).
struct Resident {
  std::vector<char> key;
  uint64_t hash = 0;
  std::shared_ptr<const Setup> setup;
  std::unique_ptr<emu_mesh> mesh;
  Clock::time_point used;
  // the state left by the last request may seed a warm start: that request
  // ended EMU_OK, or EMU_E_NOT_CONVERGED with a finite gradient norm
  bool state_ok = false;
};

struct Active {
  Request* req;
  std::unique_ptr<Resident> res;
};

}  // namespace

struct emu_server {
  emu_server_opts opts{};
  int device = 0;
  hipStream_t st = nullptr;
  Clock::time_point t0;

  std::mutex mu;
  std::condition_variable cv_setup, cv_sched, cv_done;
  bool stop = false;
  uint64_t next_ticket = 1;
  uint64_t fault_ticket = 0;  // EMU_FAULT=linesearch:T (0: none)
  std::map<uint64_t, std::unique_ptr<Request>> reqs;
  std::deque<Request*> setup_q;
  std::map<uint64_t, Request*> ready;  // by ticket: admission order
  int in_setup = 0;
  std::unordered_map<uint64_t, std::vector<CacheEntry>> cache;
  size_t cache_entries = 0;

  // scheduler-thread state
  std::vector<Active> active;
  std::list<std::unique_ptr<Resident>> idle;  // front = least recently used
  int64_t resident = 0;
  emu_server_report rep{};

  // batch of the current active set
  bool dirty = true;
  std::vector<emu::BatchPlan> plans;
  std::vector<std::vector<int>> plan_members;  // active indices per plan
  void* plan_mem = nullptr;
  int32_t* d_ctl = nullptr;
  int32_t* h_ctl = nullptr;
  int ctl_cap = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  double* d_qout = nullptr;
  size_t qout_cap = 0;

  std::vector<std::thread> workers;
  std::thread sched;
  std::string fatal;

  double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
};

namespace {

constexpr int kCtlWords = (int)(sizeof(emu::Ctl) / 4);
constexpr size_t kMaxCacheEntries = 256;

std::shared_ptr<const Setup> run_setup(const DescCopy& dc) {
  emu::Range range("emu_server host setup");
  auto s = std::make_shared<Setup>();
  try {
    s->hm = std::make_shared<emu::HostMesh>();
    emu::host_setup(dc.d, *s->hm, false);  // the modes follow on the device at admission
    s->img = emu::prepare_image(*s->hm);
  } catch (const emu::Error& e) {
    s->code = e.code;
    s->msg = e.msg;
    s->hm.reset();
  } catch (const std::bad_alloc&) {
    s->code = EMU_E_OOM;
    s->msg = "host allocation failed in setup";
    s->hm.reset();
  }
  return s;
}

// Whether a finished request's final state may seed a later warm start of
// the same mesh: not after a failure that can leave NaN or a diverged state.
bool warm_start_ok(emu_status code, double grad_norm) {
  return code == EMU_OK || (code == EMU_E_NOT_CONVERGED && std::isfinite(grad_norm));
}

void finish_request(emu_server* S, Request* r, emu_status code, const std::string& msg) {
  // caller holds S->mu
  r->status = code;
  r->msg = msg;
  r->finished = true;
  r->times.t_finish = S->now();
  if (code == EMU_OK) S->rep.completed++;
  else S->rep.failed++;
  S->cv_done.notify_all();
}

void worker_loop(emu_server* S) {
  for (;;) {
    Request* r = nullptr;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv_setup.wait(lk, [&] { return S->stop || !S->setup_q.empty(); });
      if (S->setup_q.empty()) return;  // stopping and nothing left
      r = S->setup_q.front();
      S->setup_q.pop_front();
      S->in_setup++;
    }
    // content-addressed cache of host setups (one computation per mesh)
    std::shared_future<std::shared_ptr<const Setup>> fut;
    std::promise<std::shared_ptr<const Setup>> prom;
    bool compute = false;
    {
      std::lock_guard<std::mutex> lk(S->mu);
      auto& bucket = S->cache[r->desc.hash];
      for (auto& e : bucket)
        if (e.key == r->desc.key) {
          fut = e.fut;
          e.used = Clock::now();
          r->cached = true;
          break;
        }
      if (!fut.valid()) {
        if (S->cache_entries >= kMaxCacheEntries) {
          // drop the least recently used finished entry
          uint64_t bh = 0;
          size_t bi = 0;
          bool found = false;
          Clock::time_point bt = Clock::time_point::max();
          for (auto& kv : S->cache)
            for (size_t i = 0; i < kv.second.size(); ++i) {
              auto& e = kv.second[i];
              if (e.fut.wait_for(std::chrono::seconds(0)) == std::future_status::ready && e.used < bt) {
                bt = e.used;
                bh = kv.first;
                bi = i;
                found = true;
              }
            }
          if (found) {
            auto& b = S->cache[bh];
            b.erase(b.begin() + (long)bi);
            S->cache_entries--;
          }
        }
        CacheEntry e;
        e.key = r->desc.key;
        e.fut = prom.get_future().share();
        e.used = Clock::now();
        fut = e.fut;
        S->cache[r->desc.hash].push_back(std::move(e));
        S->cache_entries++;
        compute = true;
      }
    }
    if (compute) prom.set_value(run_setup(r->desc));
    std::shared_ptr<const Setup> s = fut.get();
    {
      std::lock_guard<std::mutex> lk(S->mu);
      S->in_setup--;
      r->setup = s;
      r->times.t_setup_done = S->now();
      r->times.setup_cached = r->cached ? 1 : 0;
      if (s->code != EMU_OK) {
        finish_request(S, r, s->code, s->msg);
      } else {
        const emu::HostMesh& hm = *s->hm;
        if ((int)r->act.size() != hm.ngroups) {
          finish_request(S, r, EMU_E_INVALID, "activation length does not match n_groups");
        } else {
          S->ready[r->ticket] = r;
        }
      }
      S->cv_sched.notify_all();
    }
  }
}

void free_batch(emu_server* S) {
  if (S->gexec) (void)hipGraphExecDestroy(S->gexec);
  if (S->graph) (void)hipGraphDestroy(S->graph);
  S->gexec = nullptr;
  S->graph = nullptr;
  if (S->plan_mem) (void)hipFree(S->plan_mem);
  S->plan_mem = nullptr;
  S->plans.clear();
  S->plan_members.clear();
}

// Build the batch layout of the active set (one plan per precision), upload
// the mesh tables and block maps, and capture K iterations as one graph.
void rebuild_batch(emu_server* S) {
  HIPCHK(hipStreamSynchronize(S->st));
  free_batch(S);
  const int na = (int)S->active.size();
  if (na == 0) return;
  std::vector<int> groups[2];
  for (int j = 0; j < na; ++j) groups[S->active[j].res->mesh->d.mixed ? 1 : 0].push_back(j);
  std::vector<std::vector<int2>> maps;
  std::vector<std::vector<emu::DevMesh>> tables;
  for (int g = 0; g < 2; ++g) {
    if (groups[g].empty()) continue;
    std::vector<const emu::DevMesh*> ms;
    std::vector<const emu::SolvePlan*> pls;
    std::vector<emu::DevMesh> tab;
    for (int j : groups[g]) {
      ms.push_back(&S->active[j].res->mesh->d);
      pls.push_back(&S->active[j].res->mesh->plan);
      tab.push_back(S->active[j].res->mesh->d);
    }
    emu::BatchPlan bp;
    std::vector<int2> map;
    emu::batch_layout(ms, pls, bp, map);
    bp.mixed = g;
    S->plans.push_back(bp);
    S->plan_members.push_back(groups[g]);
    maps.push_back(std::move(map));
    tables.push_back(std::move(tab));
  }
  size_t total = 0;
  std::vector<size_t> off_tab, off_map;
  for (size_t p = 0; p < S->plans.size(); ++p) {
    off_tab.push_back(total);
    total += (tables[p].size() * sizeof(emu::DevMesh) + 255) & ~(size_t)255;
    off_map.push_back(total);
    total += (std::max<size_t>(1, maps[p].size()) * sizeof(int2) + 255) & ~(size_t)255;
  }
  HIPCHK(hipMalloc(&S->plan_mem, total));
  for (size_t p = 0; p < S->plans.size(); ++p) {
    char* base = (char*)S->plan_mem;
    HIPCHK(hipMemcpy(base + off_tab[p], tables[p].data(), tables[p].size() * sizeof(emu::DevMesh),
                     hipMemcpyHostToDevice));
    if (!maps[p].empty())
      HIPCHK(hipMemcpy(base + off_map[p], maps[p].data(), maps[p].size() * sizeof(int2), hipMemcpyHostToDevice));
    S->plans[p].meshes = (const emu::DevMesh*)(base + off_tab[p]);
    S->plans[p].map = (const int2*)(base + off_map[p]);
  }
  if (na > S->ctl_cap) {
    if (S->d_ctl) HIPCHK(hipFree(S->d_ctl));
    if (S->h_ctl) HIPCHK(hipHostFree(S->h_ctl));
    S->d_ctl = nullptr;
    S->h_ctl = nullptr;
    const int cap = std::max(na, 2 * S->ctl_cap);
    HIPCHK(hipMalloc((void**)&S->d_ctl, (size_t)cap * kCtlWords * 4));
    HIPCHK(hipHostMalloc((void**)&S->h_ctl, (size_t)cap * kCtlWords * 4, hipHostMallocDefault));
    S->ctl_cap = cap;
  }
  const int K = S->opts.iters_per_round;
  HIPCHK(hipStreamBeginCapture(S->st, hipStreamCaptureModeThreadLocal));
  for (int k = 0; k < K; ++k)
    for (const auto& bp : S->plans) emu::launch_batch_iteration(bp, S->st);
  HIPCHK(hipStreamEndCapture(S->st, &S->graph));
  HIPCHK(hipGraphInstantiate(&S->gexec, S->graph, nullptr, nullptr, 0));
  S->dirty = false;
}

// Admit ready requests in submission order while a slot is free and the
// budget allows (caller holds the lock; device work happens here too).
void admit(emu_server* S, std::unique_lock<std::mutex>& lk) {
  emu::Range range("emu_server admit");
  (void)lk;
  while (!S->ready.empty() && (int)S->active.size() < S->opts.max_slots) {
    Request* r = S->ready.begin()->second;
    const Setup& s = *r->setup;
    // a resident idle copy of the same mesh?
    std::unique_ptr<Resident> res;
    for (auto it = S->idle.begin(); it != S->idle.end(); ++it)
      if ((*it)->hash == r->desc.hash && (*it)->key == r->desc.key) {
        res = std::move(*it);
        S->idle.erase(it);
        break;
      }
    const int64_t need = res ? 0 : (int64_t)s.img->total;
    if (!res && need > S->opts.hbm_budget_bytes) {
      S->ready.erase(S->ready.begin());
      finish_request(S, r, EMU_E_OOM, "mesh alone exceeds the serving HBM budget");
      continue;
    }
    while (!res && S->resident + need > S->opts.hbm_budget_bytes && !S->idle.empty()) {
      S->resident -= S->idle.front()->mesh->bytes;
      S->idle.pop_front();  // frees device memory (least recently used)
    }
    if (!res && S->resident + need > S->opts.hbm_budget_bytes) break;  // wait for active meshes to finish
    S->ready.erase(S->ready.begin());
    bool fresh = false;
    try {
      if (!res) {
        res.reset(new Resident());
        res->key = r->desc.key;
        res->hash = r->desc.hash;
        res->setup = r->setup;
        res->mesh.reset(new emu_mesh(s.hm));
        emu::upload_image(res->mesh.get(), s.img, S->st);
        res->mesh->img.reset();
        emu::ensure_modes_of(res->mesh.get());
        S->resident += res->mesh->bytes;
        fresh = true;
      }
      emu_mesh* M = res->mesh.get();
      r->times.device_bytes = M->bytes;
      for (int g = 0; g < M->hm.ngroups; ++g) M->act[g] = r->act[g];
      HIPCHK(hipMemcpyAsync((void*)M->d.act, M->act.data(), M->act.size() * 8, hipMemcpyHostToDevice, S->st));
      if (fresh || !r->opts.warm_start || !res->state_ok) emu::launch_init_rest(M->d, S->st);
      emu::init_ctl(M, r->opts, 0);
      emu::fresh_solve(M);
      HIPCHK(hipGetLastError());
    } catch (const emu::Error& e) {
      if (res && res->mesh && fresh) S->resident -= res->mesh->bytes;
      finish_request(S, r, e.code, e.msg);
      continue;
    }
    res->used = Clock::now();
    r->times.t_admit = S->now();
    S->active.push_back(Active{r, std::move(res)});
    S->dirty = true;
  }
  S->rep.peak_active = std::max<int32_t>(S->rep.peak_active, (int32_t)S->active.size());
  S->rep.peak_resident_bytes = std::max<int64_t>(S->rep.peak_resident_bytes, S->resident);
}

// One round: K iterations of every active mesh, then retire finished ones.
void run_round(emu_server* S, std::unique_lock<std::mutex>& lk) {
  emu::Range range("emu_server round");
  if (S->dirty) rebuild_batch(S);
  const int na = (int)S->active.size();
  HIPCHK(hipGraphLaunch(S->gexec, S->st));
  std::vector<int> order;  // active index of each gathered control block
  int pos = 0;
  for (size_t p = 0; p < S->plans.size(); ++p) {
    emu::launch_batch_gather_ctl(S->plans[p], S->d_ctl + (size_t)pos * kCtlWords, S->st);
    for (int j : S->plan_members[p]) order.push_back(j);
    pos += S->plans[p].n_meshes;
  }
  HIPCHK(hipMemcpyAsync(S->h_ctl, S->d_ctl, (size_t)na * kCtlWords * 4, hipMemcpyDeviceToHost, S->st));
  lk.unlock();
  hipError_t e = hipStreamSynchronize(S->st);
  lk.lock();
  HIPCHK(e);
  S->rep.rounds++;
  std::vector<bool> done(na, false);
  for (int k = 0; k < na; ++k) {
    const int j = order[k];
    emu::Ctl c;
    std::memcpy(&c, S->h_ctl + (size_t)k * kCtlWords, sizeof(c));
    Active& a = S->active[j];
    a.req->rounds++;
    const bool cap = a.req->rounds > a.req->opts.max_iters / std::max(1, S->opts.iters_per_round) + 2;
    const bool fault = a.req->ticket == S->fault_ticket;  // the test hook fails this request now
    if (!c.done && !cap && !fault) continue;
    done[j] = true;
    emu_mesh* M = a.res->mesh.get();
    std::memcpy(M->h_ctl, &c, sizeof(c));
    Request* r = a.req;
    const size_t n3 = 3 * (size_t)M->hm.n;
    if (n3 > S->qout_cap) {
      if (S->d_qout) HIPCHK(hipFree(S->d_qout));
      S->d_qout = nullptr;
      HIPCHK(hipMalloc((void**)&S->d_qout, n3 * 8));
      S->qout_cap = n3;
    }
    emu::launch_to_user_q(M, S->d_qout);
    r->q.resize(n3);
    HIPCHK(hipMemcpyAsync(r->q.data(), S->d_qout, n3 * 8, hipMemcpyDeviceToHost, S->st));
    HIPCHK(hipStreamSynchronize(S->st));
    const double t = S->now();
    emu::fill_stats(c, &r->stats, (float)((t - r->times.t_admit) * 1e3));
    emu_status code = fault ? EMU_E_LINESEARCH : c.done ? (emu_status)c.status : EMU_E_NOT_CONVERGED;
    r->stats.status = code;
    finish_request(S, r, code,
                   code == EMU_OK                ? ""
                   : code == EMU_E_NOT_CONVERGED ? "max_iters reached"
                   : code == EMU_E_LINESEARCH    ? "line search found no Armijo step"
                                                 : "non-finite value in the iteration");
    a.res->used = Clock::now();
    a.res->state_ok = warm_start_ok(code, r->stats.grad_norm);
    if (a.res->state_ok) {
      S->idle.push_back(std::move(a.res));  // stays resident for reuse
    } else {
      S->resident -= a.res->mesh->bytes;  // a failed request releases its device memory
      a.res.reset();
    }
  }
  std::vector<Active> keep;
  for (int j = 0; j < na; ++j)
    if (!done[j]) keep.push_back(std::move(S->active[j]));
    else S->dirty = true;
  S->active.swap(keep);
}

void fail_active(emu_server* S, emu_status code, const std::string& msg) {
  for (auto& a : S->active) {
    finish_request(S, a.req, code, msg);
    if (a.res && a.res->mesh) S->resident -= a.res->mesh->bytes;
  }
  S->active.clear();
  S->dirty = true;
}

void sched_loop(emu_server* S) {
  (void)hipSetDevice(S->device);
  std::unique_lock<std::mutex> lk(S->mu);
  for (;;) {
    admit(S, lk);
    if (S->active.empty()) {
      if (S->stop && S->ready.empty() && S->setup_q.empty() && S->in_setup == 0) break;
      S->cv_sched.wait(lk);
      continue;
    }
    try {
      run_round(S, lk);
    } catch (const emu::Error& e) {
      S->fatal = e.msg;
      fail_active(S, e.code, e.msg);
    }
  }
}

}  // namespace

extern "C" {

emu_status emu_server_create(const emu_server_opts* opts, emu_server** out) {
  if (!out) {
    emu::set_error("NULL argument");
    return EMU_E_INVALID;
  }
  *out = nullptr;
  emu_server* S = nullptr;
  try {
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) throw emu::Error{EMU_E_HIP, "no HIP device available"};
    S = new emu_server();
    if (opts) S->opts = *opts;
    if (S->opts.max_slots < 0 || S->opts.setup_threads < 0 || S->opts.iters_per_round < 0 ||
        S->opts.hbm_budget_bytes < 0)
      throw emu::Error{EMU_E_INVALID, "invalid server options"};
    if (S->opts.max_slots == 0) S->opts.max_slots = 64;
    if (S->opts.setup_threads == 0) S->opts.setup_threads = 4;
    if (S->opts.iters_per_round == 0) S->opts.iters_per_round = 16;
    if (const char* f = std::getenv("EMU_FAULT")) {
      const std::string spec(f);
      if (spec.rfind("linesearch:", 0) == 0) S->fault_ticket = std::strtoull(spec.c_str() + 11, nullptr, 10);
    }
    S->opts.iters_per_round = std::min(S->opts.iters_per_round, 256);
    HIPCHK(hipGetDevice(&S->device));
    if (S->opts.hbm_budget_bytes == 0) {
      size_t fr = 0, tot = 0;
      HIPCHK(hipMemGetInfo(&fr, &tot));
      S->opts.hbm_budget_bytes = (int64_t)(0.8 * (double)fr);
    }
    HIPCHK(hipStreamCreateWithFlags(&S->st, hipStreamNonBlocking));
    S->t0 = Clock::now();
    for (int i = 0; i < S->opts.setup_threads; ++i) S->workers.emplace_back(worker_loop, S);
    S->sched = std::thread(sched_loop, S);
    *out = S;
    return EMU_OK;
  } catch (const emu::Error& e) {
    delete S;
    emu::set_error(e.msg);
    return e.code;
  } catch (const std::system_error&) {
    emu::set_error("could not start server threads");
    return EMU_E_INVALID;
  }
}

emu_status emu_server_submit(emu_server* S, const emu_mesh_desc* desc, const double* activation,
                             const emu_solve_opts* opts, uint64_t* ticket) {
  if (!S || !desc || !ticket) {
    emu::set_error("NULL argument");
    return EMU_E_INVALID;
  }
  try {
    std::unique_ptr<Request> r(new Request());
    r->times.t_submit = S->now();
    if (desc->hessian_blocks != EMU_BLOCKS_SPLIT)
      throw emu::Error{EMU_E_INVALID, "the serving loop runs the split element blocks only"};
    if (desc->affine_bones) throw emu::Error{EMU_E_INVALID, "the serving loop does not run affine bones"};
    copy_desc(*desc, r->desc);
    if (desc->n_groups < 0) throw emu::Error{EMU_E_INVALID, "negative n_groups"};
    if (desc->n_groups > 0 && !activation) throw emu::Error{EMU_E_INVALID, "NULL activation"};
    r->act.assign(activation, activation + desc->n_groups);
    for (double a : r->act)
      if (!(a >= 0.0) || !std::isfinite(a)) throw emu::Error{EMU_E_INVALID, "activations must be finite and >= 0"};
    r->opts = opts ? *opts : emu_solve_opts_default();
    const emu_solve_opts& o = r->opts;
    if (!(o.grad_tol >= 0) || o.max_iters < 0 || !(o.sigma0 > 0) || !(o.rho > 0 && o.rho < 1) ||
        !(o.armijo_c > 0 && o.armijo_c < 1) || !(o.grad_rtol >= 0))
      throw emu::Error{EMU_E_INVALID, "invalid solve options"};
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) throw emu::Error{EMU_E_STATE, "server is shutting down"};
    r->ticket = S->next_ticket++;
    *ticket = r->ticket;
    S->setup_q.push_back(r.get());
    S->reqs[r->ticket] = std::move(r);
    S->rep.submitted++;
    S->cv_setup.notify_one();
    return EMU_OK;
  } catch (const emu::Error& e) {
    emu::set_error(e.msg);
    return e.code;
  } catch (const std::bad_alloc&) {
    emu::set_error("host allocation failed");
    return EMU_E_OOM;
  }
}

emu_status emu_server_wait(emu_server* S, uint64_t ticket, double* q_host, emu_solve_stats* stats,
                           emu_request_times* times) {
  if (!S) {
    emu::set_error("NULL argument");
    return EMU_E_INVALID;
  }
  std::unique_ptr<Request> r;
  {
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) {
      emu::set_error("unknown or already collected ticket");
      return EMU_E_INVALID;
    }
    Request* rp = it->second.get();
    S->cv_done.wait(lk, [&] { return rp->finished; });
    r = std::move(it->second);
    S->reqs.erase(it);
  }
  if (q_host && !r->q.empty()) std::memcpy(q_host, r->q.data(), r->q.size() * 8);
  if (stats) *stats = r->stats;
  if (times) *times = r->times;
  if (r->status != EMU_OK) emu::set_error(r->msg);
  return r->status;
}

emu_status emu_server_report_get(emu_server* S, emu_server_report* rep) {
  if (!S || !rep) {
    emu::set_error("NULL argument");
    return EMU_E_INVALID;
  }
  std::lock_guard<std::mutex> lk(S->mu);
  *rep = S->rep;
  rep->resident_bytes = S->resident;
  return EMU_OK;
}

emu_status emu_server_destroy(emu_server* S) {
  if (!S) return EMU_OK;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv_setup.notify_all();
  S->cv_sched.notify_all();
  for (auto& t : S->workers) t.join();
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->cv_sched.notify_all();
  }
  if (S->sched.joinable()) S->sched.join();
  (void)hipStreamSynchronize(S->st);
  free_batch(S);
  S->active.clear();
  S->idle.clear();
  if (S->d_ctl) (void)hipFree(S->d_ctl);
  if (S->h_ctl) (void)hipHostFree(S->h_ctl);
  if (S->d_qout) (void)hipFree(S->d_qout);
  if (S->st) (void)hipStreamDestroy(S->st);
  const bool bad = !S->fatal.empty();
  const std::string msg = S->fatal;
  delete S;
  if (bad) {
    emu::set_error(msg);
    return EMU_E_HIP;
  }
  return EMU_OK;
}

}  // extern "C"
