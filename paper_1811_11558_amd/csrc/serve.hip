// Continuous-batching solve server (host code, part of libfvim.so).
//
// Requests (an elastoplastic contact solve: grid, material, rigid surface,
// cumulative loads, options) are copied at submission into a queue.  A
// request is admitted when a worker slot is free and its device footprint
// fits in what is left of the HBM budget; the first pending request that fits
// is taken, so small requests flow past a large one that is waiting for
// memory.  Each slot is a host thread with its own HIP stream (default
// priority), so admitted requests run concurrently on the device while new
// ones keep arriving.  A request's state lives in device memory from
// admission until its result has been copied back; the slot then frees the
// memory for the next admission, unless the slot keeps it: each slot
// retains the context and state memory of its last request and reuses them
// for a later request of the same grid, material, precision and depth nodes
// (the operator and solver workspaces, mode tables and captured graphs carry
// over; the state is cleared), so a stream of same-sized requests allocates
// nothing after its first.  Retained memory counts against the budget and is
// dropped when a pending request cannot be admitted otherwise.  Every request
// runs the same deterministic kernels with the default depth-pass layout, so
// its result depends neither on what else is running nor on which request
// the slot served before.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/fvim.h"
#include "solver.hpp"
#include "solver.hpp"

namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Job {
  uint64_t id = 0;
  fvim_request req;
  std::vector<double> h;       // host copy of the surface
  std::vector<double> z;       // host copy of the depth nodes (empty: uniform)
  size_t bytes = 0;            // admission footprint
  fvim_result res;
  std::vector<double> p_host, u3_host;
  bool done = false;
};

// The context and state memory a slot keeps from its last request.
struct SlotCache {
  fvim_ctx* ctx = nullptr;
  double* mem = nullptr;
  size_t held = 0;             // budget bytes it holds (0: nothing kept)
  fvim_grid grid{};
  fvim_material mat{};
  int precision = -1;
  std::vector<double> z;
};

bool cache_matches(const SlotCache& c, const Job* j) {
  const fvim_request& r = j->req;
  return c.ctx && c.precision == r.precision && memcmp(&c.grid, &r.grid, sizeof(fvim_grid)) == 0 &&
         memcmp(&c.mat, &r.mat, sizeof(fvim_material)) == 0 && c.z == j->z;
}

// Budget bytes the slot holds once it has taken job j.
size_t held_after(const SlotCache& c, const Job* j) {
  return cache_matches(c, j) ? std::max(c.held, j->bytes) : j->bytes;
}

void cache_drop(SlotCache& c, hipStream_t st) {
  if (!c.ctx) return;
  std::lock_guard<std::recursive_mutex> dev(fvim::device_lock());
  hipStreamSynchronize(st);
  if (c.mem) hipFree(c.mem);
  fvim_destroy(c.ctx);
  c.ctx = nullptr;
  c.mem = nullptr;
  c.z.clear();
}

}  // namespace

struct fvim_server {
  size_t budget = 0, in_use = 0, peak = 0;
  int device = 0;
  uint64_t next_id = 1;
  bool stop = false;
  int running = 0;
  uint64_t completed = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Job*> pending;
  std::map<uint64_t, std::unique_ptr<Job>> jobs;
  std::vector<std::thread> workers;
  double t0 = 0.0;
};

namespace {

size_t request_bytes(const fvim_request* r) {
  const fvim_grid& g = r->grid;
  const size_t V = (size_t)g.nx * g.ny * g.nz, ns = (size_t)g.nx * g.ny;
  // operator + solver workspace, plus the caller-side state of a solve
  return fvim_footprint_bytes(&g, r->precision, 1) + sizeof(double) * (13 * V + 4 * ns + 3 * ns) +
         fvim::krylov_footprint(&g, &r->opts) + (r->opts.mu_f > 0 ? fvim::friction_footprint(&g) : 0);
}

int run_job(fvim_server* s, Job* j, hipStream_t st, SlotCache& cache) {
  const fvim_request& r = j->req;
  const fvim_grid& g = r.grid;
  const size_t V = (size_t)g.nx * g.ny * g.nz, ns = (size_t)g.nx * g.ny;
  const size_t nd = 13 * V + 5 * ns;
  int rc = FVIM_OK;
  if (!cache_matches(cache, j)) {
    cache_drop(cache, st);
    fvim_ctx* ctx = nullptr;
    rc = fvim_create(&g, &r.mat, r.precision, FVIM_K0_INCLUDE, st, &ctx);
    if (rc) return rc;
    if (!j->z.empty() && (rc = fvim_set_depth_nodes(ctx, j->z.data()))) {
      fvim_destroy(ctx);
      return rc;
    }
    double* mem = nullptr;
    {
      // allocation does not overlap another slot's graph capture
      std::lock_guard<std::recursive_mutex> dev(fvim::device_lock());
      if (hipMalloc((void**)&mem, sizeof(double) * nd) != hipSuccess) {
        fvim_destroy(ctx);
        return FVIM_ENOMEM;
      }
    }
    cache.ctx = ctx;
    cache.mem = mem;
    cache.grid = g;
    cache.mat = r.mat;
    cache.precision = r.precision;
    cache.z = j->z;
  }
  fvim_ctx* ctx = cache.ctx;
  double* mem = cache.mem;
  hipError_t e = hipMemsetAsync(mem, 0, sizeof(double) * nd, st);
  fvim_state state;
  state.eps_p = mem;
  state.sigma = mem + 6 * V;
  state.ep = mem + 12 * V;
  state.traction = mem + 13 * V;
  state.u3p = state.traction + 3 * ns;
  double* h = state.u3p + ns;
  {
    // copies from pageable host memory do not overlap a graph capture
    std::lock_guard<std::recursive_mutex> dev(fvim::device_lock());
    if (e == hipSuccess) e = hipMemcpyAsync(h, j->h.data(), sizeof(double) * ns, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
  }
  if (e != hipSuccess) rc = FVIM_EHIP;
  std::vector<fvim_ep_info> info(r.n_steps);
  if (!rc) rc = elastoplastic_solve(ctx, h, r.W_steps, r.n_steps, &r.opts, &state, info.data());
  if (rc) {
    // the record of the step that failed (the first one not committed)
    for (const fvim_ep_info& i : info)
      if (!i.committed) {
        j->res.info = i;
        break;
      }
  } else {
    std::lock_guard<std::recursive_mutex> dev(fvim::device_lock());
    j->res.info = info[r.n_steps - 1];
    j->p_host.resize(ns);
    j->u3_host.resize(ns);
    e = hipMemcpyAsync(j->p_host.data(), state.traction + 2 * ns, sizeof(double) * ns, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(j->u3_host.data(), state.u3p, sizeof(double) * ns, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) rc = FVIM_EHIP;
    size_t nc = 0;
    for (double v : j->p_host) nc += v > 0.0;
    j->res.contact_fraction = (double)nc / (double)ns;
  }
  hipStreamSynchronize(st);
  // a failed solve does not leave its context to the next request
  if (rc) cache_drop(cache, st);
  return rc;
}

void worker(fvim_server* s) {
  hipSetDevice(s->device);
  hipStream_t st = nullptr;
  {
    std::lock_guard<std::recursive_mutex> dev(fvim::device_lock());
    hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
  }
  SlotCache cache;
  for (;;) {
    Job* j = nullptr;
    bool drop = false;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      for (;;) {
        if (s->stop && s->pending.empty()) break;
        // first pending request that fits in the remaining budget, counting
        // the slot's retained memory as reusable (same grid) or freed
        std::vector<size_t> sizes;
        sizes.reserve(s->pending.size());
        for (Job* q : s->pending) sizes.push_back(held_after(cache, q));
        int k = fvim_admit_index(sizes.data(), (int)sizes.size(), s->budget, s->in_use - cache.held);
        if (k >= 0) {
          j = s->pending[k];
          s->pending.erase(s->pending.begin() + k);
          const size_t held = sizes[k];
          if (!cache_matches(cache, j) && cache.ctx) {
            // the slot frees its context outside the lock; its bytes are
            // released now and the new request's counted
            drop = true;
          }
          s->in_use = s->in_use - cache.held + held;
          cache.held = held;
          s->peak = std::max(s->peak, s->in_use);
          s->running++;
          break;
        }
        if (!s->pending.empty() && cache.held > 0) {
          // nothing fits: give the retained memory back so that some slot
          // can admit a pending request
          s->in_use -= cache.held;
          cache.held = 0;
          drop = true;
          break;
        }
        s->cv_work.wait(lk);
      }
    }
    if (drop) {
      cache_drop(cache, st);
      s->cv_work.notify_all();
      if (!j) continue;
    }
    if (!j) break;
    j->res.t_admit = now_s() - s->t0;
    int rc = run_job(s, j, st, cache);
    {
      std::lock_guard<std::mutex> lk(s->mu);
      j->res.status = rc;
      if (rc) snprintf(j->res.error, sizeof(j->res.error), "%s", fvim_last_error());
      j->res.t_done = now_s() - s->t0;
      j->res.p = j->p_host.empty() ? nullptr : j->p_host.data();
      j->res.u3p = j->u3_host.empty() ? nullptr : j->u3_host.data();
      j->done = true;
      if (!cache.ctx) {              // nothing kept (a failed solve)
        s->in_use -= cache.held;
        cache.held = 0;
      }
      s->running--;
      s->completed++;
    }
    s->cv_done.notify_all();
    s->cv_work.notify_all();
  }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->in_use -= cache.held;
    cache.held = 0;
  }
  cache_drop(cache, st);
  if (st) {
    std::lock_guard<std::recursive_mutex> dev(fvim::device_lock());
    hipStreamDestroy(st);
  }
}

}  // namespace

extern "C" {

int fvim_admit_index(const size_t* pending_bytes, int n, size_t budget, size_t in_use) {
  for (int i = 0; i < n; ++i)
    if (pending_bytes[i] <= budget && in_use + pending_bytes[i] <= budget) return i;
  return -1;
}

size_t fvim_request_bytes(const fvim_request* r) { return r ? request_bytes(r) : 0; }

int fvim_server_create(size_t hbm_budget_bytes, int max_slots, int device, fvim_server** out) {
  if (!out || max_slots < 1 || max_slots > 64 || hbm_budget_bytes == 0) return FVIM_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return FVIM_ENODEV;
  fvim_server* s = new fvim_server();
  s->budget = hbm_budget_bytes;
  s->device = device;
  s->t0 = now_s();
  for (int i = 0; i < max_slots; ++i) s->workers.emplace_back(worker, s);
  *out = s;
  return FVIM_OK;
}

int fvim_server_submit(fvim_server* s, const fvim_request* r, uint64_t* id) {
  if (!s || !r || !id || !r->h) return FVIM_EINVAL;
  if (r->n_steps < 1 || r->n_steps > FVIM_MAX_STEPS) return FVIM_EINVAL;
  const fvim_grid& g = r->grid;
  if (fvim_footprint_bytes(&g, r->precision, 1) == 0) return FVIM_EINVAL;
  std::unique_ptr<Job> j(new Job());
  j->req = *r;
  const size_t ns = (size_t)g.nx * g.ny;
  j->h.assign(r->h, r->h + ns);
  j->req.h = nullptr;
  if (r->z) j->z.assign(r->z, r->z + g.nz);
  j->req.z = nullptr;
  j->bytes = request_bytes(r);
  if (j->bytes > s->budget) return FVIM_ENOMEM;
  memset(&j->res, 0, sizeof(j->res));
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return FVIM_EINVAL;
    j->id = s->next_id++;
    j->res.t_submit = now_s() - s->t0;
    *id = j->id;
    s->pending.push_back(j.get());
    s->jobs[j->id] = std::move(j);
  }
  s->cv_work.notify_all();
  return FVIM_OK;
}

int fvim_server_poll(fvim_server* s, uint64_t id, int wait, fvim_result* out) {
  if (!s || !out) return FVIM_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->jobs.find(id);
  if (it == s->jobs.end()) return FVIM_EINVAL;
  Job* j = it->second.get();
  if (wait) s->cv_done.wait(lk, [&] { return j->done; });
  if (!j->done) return 0;
  *out = j->res;
  return 1;
}

int fvim_server_release(fvim_server* s, uint64_t id) {
  if (!s) return FVIM_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->jobs.find(id);
  if (it == s->jobs.end() || !it->second->done) return FVIM_EINVAL;
  s->jobs.erase(it);
  return FVIM_OK;
}

int fvim_server_get_stats(fvim_server* s, fvim_server_stats* out) {
  if (!s || !out) return FVIM_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  out->pending = (int)s->pending.size();
  out->running = s->running;
  out->completed = s->completed;
  out->bytes_in_use = s->in_use;
  out->peak_bytes = s->peak;
  out->budget = s->budget;
  return FVIM_OK;
}

void fvim_server_destroy(fvim_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  for (auto& t : s->workers) t.join();
  delete s;
}

}  // extern "C"
