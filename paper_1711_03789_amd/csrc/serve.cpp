// Solve server: continuous batching of independent absorptive-Maxwell solves on one GPU.
//
// Each request is a unit-cube problem (n cubes per side, wavenumber k, absorption xi, p^3
// subdomains, Gaussian source) solved by the one-level Schwarz-preconditioned (F)GMRES path.  A
// fixed number of slots (worker threads, each with its own HIP stream and GMRES workspace) pull
// requests in arrival order.  A slot first does the host work of a request (mesh, assembly,
// partition, local problems and orderings), which fixes the request's exact device footprint;
// the request is then admitted when that footprint fits in what the budget has left, runs its
// device work (upload, batched factorisation, GMRES) on the slot's stream concurrently with the
// other admitted requests, and returns its memory.  Device memory comes from the stream-ordered
// allocator of the slot's stream, so requests never synchronise each other.  All kernels are
// deterministic (fixed reduction orders, schedule-independent sweep accumulation), so a request
// returns the same solution whether it runs alone or among others.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>

#include "objects.hpp"

namespace mx {

static double wall() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct SrvRequest {
  mx_request req;
  double t_submit = 0, t_admit = 0, t_host_done = 0, t_done = 0;
  bool done = false;
  bool injected = false;  // the last device-phase failure was an injected one
  mx_result res{};
  std::string msg;
  std::vector<double> x;  // interleaved complex128 solution
};

// Batches the preconditioner applications of the requests in their GMRES phase.  A request's
// GMRES calls apply() (through the preconditioner's apply hook) from its slot thread: the
// application joins the pending batch, and the call returns once the batch has been launched on
// the batcher's stream, after making the request's stream wait for it.  The batcher launches
// when every request in its GMRES phase has an application pending, or when the window since
// the first pending one has passed.  A batch of one is handed back and launched on the
// request's own stream, so lone applications keep running concurrently on the requests'
// streams.  At most one application per request is pending (apply blocks until launched), so a
// batch holds at most one per slot.
struct Batcher {
  struct Job {
    mx_precond *P = nullptr;
    const void *v = nullptr;
    void *z = nullptr;
    hipEvent_t ready = nullptr, done = nullptr;
    bool pending = false, launched = false, alone = false;
  };
  int device = 0, cus = 256, window_us = 200;
  std::mutex mu;
  std::condition_variable cv_submit, cv_launched;
  std::vector<Job> jobs;  // one per slot
  int active = 0;         // slots whose request is in its GMRES phase
  int npending = 0;
  bool stop = false;
  std::thread th;
  hipStream_t st = nullptr;
  DevBuf jobs_dev, ctrl;
  uint64_t batches = 0, applications = 0;

  void start(int dev, int ncus, int slots, int window) {
    device = dev, cus = ncus, window_us = window > 0 ? window : 50;
    MX_HIP(hipSetDevice(device));
    MX_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    jobs.resize(slots);
    for (auto &j : jobs) {
      MX_HIP(hipEventCreateWithFlags(&j.ready, hipEventDisableTiming));
      MX_HIP(hipEventCreateWithFlags(&j.done, hipEventDisableTiming));
    }
    jobs_dev.alloc(batch_job_bytes() * slots);
    ctrl.alloc(64);
    th = std::thread([this] { run(); });
  }
  void finish() {
    {
      std::lock_guard<std::mutex> lk(mu);
      stop = true;
    }
    cv_submit.notify_all();
    if (th.joinable()) th.join();
    if (st) (void)hipStreamSynchronize(st);
    jobs_dev.release();
    ctrl.release();
    for (auto &j : jobs) {
      if (j.ready) (void)hipEventDestroy(j.ready);
      if (j.done) (void)hipEventDestroy(j.done);
    }
    if (st) (void)hipStreamDestroy(st);
    st = nullptr;
  }
  // a slot's request enters (P materialised) or leaves its GMRES phase
  void enter(int slot, mx_precond *P) {
    batch_job_write(P, jobs_dev.p, slot);
    std::lock_guard<std::mutex> lk(mu);
    jobs[slot].P = P;
    ++active;
  }
  void leave(int slot) {
    {
      std::lock_guard<std::mutex> lk(mu);
      jobs[slot].P = nullptr;
      --active;
    }
    cv_submit.notify_all();  // the others may now be complete
  }
  void apply(int slot, const void *v, void *z, hipStream_t rst) {
    Job &j = jobs[slot];
    MX_HIP(hipEventRecord(j.ready, rst));
    std::unique_lock<std::mutex> lk(mu);
    j.v = v, j.z = z, j.pending = true, j.launched = false, j.alone = false;
    ++npending;
    cv_submit.notify_all();
    cv_launched.wait(lk, [&] { return j.launched || stop; });
    if (!j.launched) fail(MX_EDEVICE, "server stopped with an application pending");
    const bool alone = j.alone;
    lk.unlock();
    if (alone) precond_apply_direct(j.P, v, z, rst);
    else MX_HIP(hipStreamWaitEvent(rst, j.done, 0));
  }
  void run() {
    (void)hipSetDevice(device);
    std::vector<int> slots;
    std::vector<mx_precond *> Ps;
    std::vector<const void *> vin;
    std::vector<void *> zout;
    while (true) {
      std::unique_lock<std::mutex> lk(mu);
      cv_submit.wait(lk, [&] { return stop || npending > 0; });
      if (stop) break;
      cv_submit.wait_for(lk, std::chrono::microseconds(window_us),
                         [&] { return stop || npending >= active; });
      if (stop) break;
      slots.clear(), Ps.clear(), vin.clear(), zout.clear();
      for (int s = 0; s < (int)jobs.size(); ++s)
        if (jobs[s].pending) {
          slots.push_back(s), Ps.push_back(jobs[s].P), vin.push_back(jobs[s].v), zout.push_back(jobs[s].z);
          jobs[s].pending = false;
        }
      npending = 0;
      if (slots.size() == 1) {  // nothing to merge with: launched on the request's stream
        jobs[slots[0]].alone = true;
        jobs[slots[0]].launched = true;
        lk.unlock();
        cv_launched.notify_all();
        continue;
      }
      lk.unlock();
      std::string err;
      try {
        for (int s : slots) MX_HIP(hipStreamWaitEvent(st, jobs[s].ready, 0));
        batch_apply((int)slots.size(), slots.data(), Ps.data(), vin.data(), zout.data(), jobs_dev.p,
                    ctrl.as<int>(), cus, st);
        for (int s : slots) MX_HIP(hipEventRecord(jobs[s].done, st));
      } catch (const Error &e) {
        err = e.msg;
      }
      lk.lock();
      ++batches;
      applications += slots.size();
      for (int s : slots) jobs[s].launched = err.empty();
      if (!err.empty()) stop = true;  // a launch failure ends batching: pending callers fail
      lk.unlock();
      cv_launched.notify_all();
    }
    cv_launched.notify_all();
  }
};

static void batch_hook(void *arg, mx_precond *P, const void *v, void *z, hipStream_t st);

struct SlotHook {  // what the apply hook of a slot's preconditioner needs
  Batcher *b;
  int slot;
};

static void batch_hook(void *arg, mx_precond *P, const void *v, void *z, hipStream_t st) {
  (void)P;
  SlotHook *h = (SlotHook *)arg;
  h->b->apply(h->slot, v, z, st);
}

struct Server {
  mx_server_opts opts{};
  int device = 0;
  int cus = 256;
  uint64_t budget = 0, used = 0, peak = 0;
  std::mutex mu;
  std::condition_variable cv_queue, cv_mem, cv_done;
  std::deque<uint64_t> queue;
  std::map<uint64_t, std::unique_ptr<SrvRequest>> reqs;
  uint64_t next_id = 1;
  bool stop = false;
  int admitted = 0, max_admitted = 0;
  uint64_t finished = 0;  // device phases ended (successfully or not)
  // test hook: the next `inject_enomem` device phases fail with MX_ENOMEM right after their
  // preconditioner is materialised (the path a late allocation failure takes); such a failure
  // is retried even when the request is alone on the device
  std::atomic<int> inject_enomem{0};
  std::vector<std::thread> workers;
  Batcher batcher;         // used when opts.batch_applies
  std::vector<SlotHook> hooks;

  void run_request(int slot, mx_ctx *ctx, hipStream_t st, SrvRequest *R);
  void device_phase(int slot, mx_ctx *ctx, hipStream_t st, SrvRequest *R, mx_matrix *A, mx_precond *P,
                    PrecondPlan &plan, const std::vector<double> &f, int64_t E);
  void release_request(mx_ctx *ctx, hipStream_t st, mx_matrix *A, mx_precond *P);
  void worker(int slot);
};

void Server::run_request(int slot, mx_ctx *ctx, hipStream_t st, SrvRequest *R) {
  const mx_request &q = R->req;
  // ---- host phase (no device memory) ----
  auto mesh = std::make_unique<mx_mesh>();
  build_mesh(mesh->m, q.n, q.n, q.n, 1.0, 1.0, 1.0);
  auto A = std::make_unique<mx_matrix>();
  A->k = q.k, A->xi = q.xi, A->bc = MX_BC_IMPEDANCE, A->device = device;
  assemble_global(mesh->m, q.k, q.xi, MX_BC_IMPEDANCE, A->h);
  auto part = std::make_unique<mx_partition>();
  build_partition(mesh->m, q.p, q.p, q.p, nullptr, nullptr, nullptr, opts.layers, part->p);
  mx_precond_opts po{};
  po.kind = opts.kind;
  po.xi_prec = q.xi;
  po.precision = opts.precision;
  auto P = std::make_unique<mx_precond>();
  PrecondPlan plan;
  precond_plan(ctx, A.get(), mesh.get(), part.get(), &po, P.get(), plan);
  const int64_t E = mesh->m.ne;
  std::vector<double> f(2 * E);
  rhs_gaussian(mesh->m, MX_BC_IMPEDANCE, q.center, q.pol, q.sigma, f.data());
  const uint64_t need = plan.device_bytes + matrix_device_bytes(A.get()) +
                        gmres_device_bytes(E, opts.restart, opts.flexible != 0) + 2 * 16 * (uint64_t)E;
  R->res.n_dof = E;
  R->res.footprint_bytes = need;
  R->t_host_done = wall();
  if (need > budget) fail(MX_EHBM, "request footprint exceeds the server's HBM budget");
  // The factorisation gets the request's own footprint as its tile-pool cap (one group), instead
  // of sizing itself from what the device has free at that moment, which other requests share.
  P->pool_limit = (int64_t)precond_one_group_bytes(P.get(), plan);
  // Admission by footprint, then the device phase.  The footprints are exact, but freed memory
  // held by the block cache and by the stream-ordered pools of other slots is not in the
  // budget: a device allocation can still fail.  Then this slot's stream is drained, its device
  // memory freed and the caches emptied before the reservation is returned, and the request waits
  // for another one to finish before it tries again (at most kMemRetries times; alone on the
  // device it gives up).
  constexpr int kMemRetries = 8;
  for (int attempt = 0;; ++attempt) {
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_mem.wait(lk, [&] { return used + need <= budget; });
      used += need;
      peak = std::max(peak, used);
      ++admitted;
      max_admitted = std::max(max_admitted, admitted);
      if (attempt == 0) R->t_admit = wall();
    }
    struct Release {
      Server *s;
      uint64_t n;
      ~Release() {
        std::lock_guard<std::mutex> lk(s->mu);
        s->used -= n;
        --s->admitted;
        ++s->finished;
        s->cv_mem.notify_all();
      }
    };
    int others = 0;
    uint64_t seen = 0;
    {
      // declared first, destroyed last: a failed attempt's device memory goes back (below)
      // before its reservation does, as on success
      Release rel{this, need};
      {
        std::lock_guard<std::mutex> lk(mu);
        others = admitted - 1;
        seen = finished;
      }
      try {
        R->injected = false;
        device_phase(slot, ctx, st, R, A.get(), P.get(), plan, f, E);
        return;
      } catch (const Error &e) {
        release_request(ctx, st, A.get(), P.get());
        if (e.code != MX_ENOMEM || attempt >= kMemRetries || (others == 0 && !R->injected)) throw;
      } catch (...) {
        release_request(ctx, st, A.get(), P.get());
        throw;
      }
      big_trim(device);
      hipMemPool_t pool;
      if (hipDeviceGetDefaultMemPool(&pool, device) == hipSuccess) (void)hipMemPoolTrimTo(pool, 0);
    }
    std::unique_lock<std::mutex> lk(mu);
    // `finished` counts this attempt too: wait for one more (another request) or an idle device
    cv_mem.wait_for(lk, std::chrono::seconds(10), [&] { return finished > seen + 1 || admitted == 0; });
  }
}

void Server::device_phase(int slot, mx_ctx *ctx, hipStream_t st, SrvRequest *R, mx_matrix *A,
                          mx_precond *P, PrecondPlan &plan, const std::vector<double> &f, int64_t E) {
  AllocScope scope(st);
  matrix_upload(A);
  precond_materialize(P, plan, st);
  for (int n = inject_enomem.load(); n > 0; n = inject_enomem.load())
    if (inject_enomem.compare_exchange_weak(n, n - 1)) {
      R->injected = true;
      fail(MX_ENOMEM, "injected allocation failure after the preconditioner setup");
    }
  DevBuf b, x;
  b.alloc(16 * (size_t)E);
  x.alloc(16 * (size_t)E);
  MX_HIP(hipMemcpyAsync(b.p, f.data(), 16 * (size_t)E, hipMemcpyHostToDevice, st));
  MX_HIP(hipMemsetAsync(x.p, 0, 16 * (size_t)E, st));
  mx_gmres_opts go{};
  go.restart = opts.restart;
  go.max_iters = opts.max_iters;
  go.flexible = opts.flexible;
  go.spmv_c64 = opts.spmv_c64;
  go.rtol = opts.rtol;
  mx_gmres_stats gs{};
  if (opts.batch_applies) {  // the GMRES phase: applications go through the batcher
    struct Phase {
      Server *s;
      int slot;
      mx_precond *P;
      Phase(Server *s_, int sl, mx_precond *P_) : s(s_), slot(sl), P(P_) {
        s->batcher.enter(slot, P);
        P->apply_hook = batch_hook;
        P->apply_hook_arg = &s->hooks[slot];
      }
      ~Phase() {
        P->apply_hook = nullptr;
        P->apply_hook_arg = nullptr;
        s->batcher.leave(slot);
      }
    } phase(this, slot, P);
    gmres_run(ctx, A, P, b.p, x.p, &go, &gs, nullptr, st);
  } else {
    gmres_run(ctx, A, P, b.p, x.p, &go, &gs, nullptr, st);
  }
  R->x.resize(2 * E);
  MX_HIP(hipMemcpyAsync(R->x.data(), x.p, 16 * (size_t)E, hipMemcpyDeviceToHost, st));
  MX_HIP(hipStreamSynchronize(st));
  R->res.iters = gs.iters;
  R->res.converged = gs.converged;
  R->res.relres_true = gs.relres_true;
  // device memory of the request goes back before its reservation does
  b.release();
  x.release();
  release_request(ctx, st, A, P);
}

// Frees every device buffer a request holds.  The frees are stream-ordered on the slot's stream,
// so the stream is drained before (work that reads the buffers) and after (the frees themselves).
// Errors are ignored: this also runs while an error propagates.
void Server::release_request(mx_ctx *ctx, hipStream_t st, mx_matrix *A, mx_precond *P) {
  (void)hipStreamSynchronize(st);
  precond_release_device(P);
  A->rowptr.release();
  A->col.release();
  A->val.release();
  A->val32.release();
  ctx->krylov.buf.release();
  (void)hipStreamSynchronize(st);
  (void)hipGetLastError();  // the ignored errors above are not reported by a later launch check
}

void Server::worker(int slot) {
  hipStream_t st = nullptr;
  mx_ctx ctx;
  ctx.device = device;
  ctx.cus = cus;
  bool ok = hipSetDevice(device) == hipSuccess &&
            hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess &&
            hipHostMalloc((void **)&ctx.pinned, 4096, hipHostMallocDefault) == hipSuccess;
  while (true) {
    uint64_t id;
    SrvRequest *R;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_queue.wait(lk, [&] { return stop || !queue.empty(); });
      if (queue.empty()) break;
      id = queue.front();
      queue.pop_front();
      R = reqs[id].get();
    }
    int code = MX_OK;
    std::string msg;
    (void)hipGetLastError();  // nothing left over from an earlier request of this slot
    if (!ok) {
      code = MX_EDEVICE;
      msg = "server slot could not create its stream";
    } else {
      try {
        run_request(slot, &ctx, st, R);
      } catch (const Error &e) {
        code = e.code;
        msg = e.msg;
      } catch (const std::bad_alloc &) {
        code = MX_ENOMEM;
        msg = "host allocation failed";
      } catch (const std::exception &e) {
        code = MX_EINVAL;
        msg = e.what();
      }
    }
    {
      std::lock_guard<std::mutex> lk(mu);
      R->res.status = code;
      R->t_done = wall();
      R->res.t_host = R->t_host_done - R->t_submit;
      R->res.t_queue = (R->t_admit > 0 ? R->t_admit : R->t_done) - R->t_submit;
      R->res.t_device = R->t_admit > 0 ? R->t_done - R->t_admit : 0.0;
      R->res.t_total = R->t_done - R->t_submit;
      R->done = true;
      R->msg = msg;
    }
    cv_done.notify_all();
  }
  ctx.krylov.buf.release();
  if (ctx.pinned) (void)hipHostFree(ctx.pinned);
  ctx.pinned = nullptr;
  if (st) (void)hipStreamDestroy(st);
}

}  // namespace mx

struct mx_server {
  mx::Server s;
};

using mx::Error;

extern "C" {

int mx_server_create(int device, const mx_server_opts *opts, mx_server **out) {
  try {
    if (!opts || !out) mx::fail(MX_EINVAL, "NULL argument");
    if (opts->slots < 1 || opts->restart < 1 || opts->max_iters < 1 || !(opts->rtol > 0))
      mx::fail(MX_EINVAL, "bad server options");
    if (opts->kind < MX_AS || opts->kind > MX_ORAS) mx::fail(MX_EINVAL, "unknown kind");
    if (opts->precision != MX_C128 && opts->precision != MX_C64) mx::fail(MX_EINVAL, "unknown precision");
    MX_HIP(hipSetDevice(device));
    hipDeviceProp_t prop;
    MX_HIP(hipGetDeviceProperties(&prop, device));
    auto S = std::make_unique<mx_server>();
    S->s.opts = *opts;
    S->s.device = device;
    S->s.cus = prop.multiProcessorCount;
    size_t free_b = 0, total_b = 0;
    {  // memory parked in the block cache or the stream-ordered pool by earlier setups counts as free
      MX_HIP(hipDeviceSynchronize());
      mx::big_trim(device);
      hipMemPool_t pool;
      MX_HIP(hipDeviceGetDefaultMemPool(&pool, device));
      MX_HIP(hipMemPoolTrimTo(pool, 0));
    }
    MX_HIP(hipMemGetInfo(&free_b, &total_b));
    S->s.budget = opts->hbm_budget ? opts->hbm_budget : (uint64_t)(0.85 * (double)free_b);
    if (opts->slots > mx::kMaxBatchJobs) mx::fail(MX_EINVAL, "at most 16 slots");
    if (opts->batch_applies) {
      S->s.hooks.resize(opts->slots);
      for (int i = 0; i < opts->slots; ++i) S->s.hooks[i] = {&S->s.batcher, i};
      S->s.batcher.start(device, S->s.cus, opts->slots, opts->batch_window_us);
    }
    try {
      for (int i = 0; i < opts->slots; ++i)
        S->s.workers.emplace_back([p = &S->s, i] { p->worker(i); });
    } catch (...) {  // the workers already started are stopped and joined before S goes away
      {
        std::lock_guard<std::mutex> lk(S->s.mu);
        S->s.stop = true;
      }
      S->s.cv_queue.notify_all();
      for (auto &t : S->s.workers) t.join();
      S->s.batcher.finish();
      throw;
    }
    *out = S.release();
    return MX_OK;
  } catch (const Error &e) {
    mx::set_error(e.code, e.msg);
    return e.code;
  } catch (const std::bad_alloc &) {
    mx::set_error(MX_ENOMEM, "host allocation failed");
    return MX_ENOMEM;
  } catch (const std::exception &e) {
    mx::set_error(MX_EINVAL, e.what());
    return MX_EINVAL;
  }
}

int mx_server_submit(mx_server *S, const mx_request *req, uint64_t *ticket) {
  try {
    if (!S || !req || !ticket) mx::fail(MX_EINVAL, "NULL argument");
    if (req->n < 1 || req->p < 1 || req->p > req->n || !(req->k > 0) || !(req->sigma > 0))
      mx::fail(MX_EINVAL, "bad request");
    auto R = std::make_unique<mx::SrvRequest>();
    R->req = *req;
    R->t_submit = mx::wall();
    std::lock_guard<std::mutex> lk(S->s.mu);
    if (S->s.stop) mx::fail(MX_EINVAL, "server is shutting down");
    uint64_t id = S->s.next_id++;
    S->s.reqs[id] = std::move(R);
    S->s.queue.push_back(id);
    *ticket = id;
    S->s.cv_queue.notify_one();
    return MX_OK;
  } catch (const Error &e) {
    mx::set_error(e.code, e.msg);
    return e.code;
  } catch (const std::bad_alloc &) {
    mx::set_error(MX_ENOMEM, "host allocation failed");
    return MX_ENOMEM;
  } catch (const std::exception &e) {
    mx::set_error(MX_EINVAL, e.what());
    return MX_EINVAL;
  }
}

int mx_server_wait(mx_server *S, uint64_t ticket, double timeout_s, mx_result *res) {
  try {
    if (!S || !res) mx::fail(MX_EINVAL, "NULL argument");
    std::unique_lock<std::mutex> lk(S->s.mu);
    auto it = S->s.reqs.find(ticket);
    if (it == S->s.reqs.end()) mx::fail(MX_EINVAL, "unknown ticket");
    mx::SrvRequest *R = it->second.get();
    auto pred = [&] { return R->done; };
    if (timeout_s < 0) S->s.cv_done.wait(lk, pred);
    else if (!S->s.cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), pred))
      mx::fail(MX_ETIMEOUT, "request not finished yet");
    *res = R->res;
    if (R->res.status != MX_OK) mx::set_error(R->res.status, R->msg);
    return MX_OK;
  } catch (const Error &e) {
    mx::set_error(e.code, e.msg);
    return e.code;
  } catch (const std::bad_alloc &) {
    mx::set_error(MX_ENOMEM, "host allocation failed");
    return MX_ENOMEM;
  } catch (const std::exception &e) {
    mx::set_error(MX_EINVAL, e.what());
    return MX_EINVAL;
  }
}

int mx_server_solution(mx_server *S, uint64_t ticket, double *x_host, int64_t n) {
  try {
    if (!S || !x_host) mx::fail(MX_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(S->s.mu);
    auto it = S->s.reqs.find(ticket);
    if (it == S->s.reqs.end()) mx::fail(MX_EINVAL, "unknown ticket");
    mx::SrvRequest *R = it->second.get();
    if (!R->done) mx::fail(MX_ETIMEOUT, "request not finished yet");
    if (R->res.status != MX_OK) mx::fail(R->res.status, "request failed");
    if ((int64_t)R->x.size() != 2 * n) mx::fail(MX_EINVAL, "n does not match the request's DOF count");
    std::memcpy(x_host, R->x.data(), 16 * (size_t)n);
    return MX_OK;
  } catch (const Error &e) {
    mx::set_error(e.code, e.msg);
    return e.code;
  } catch (const std::bad_alloc &) {
    mx::set_error(MX_ENOMEM, "host allocation failed");
    return MX_ENOMEM;
  } catch (const std::exception &e) {
    mx::set_error(MX_EINVAL, e.what());
    return MX_EINVAL;
  }
}

int mx_server_release(mx_server *S, uint64_t ticket) {
  try {
    if (!S) mx::fail(MX_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(S->s.mu);
    auto it = S->s.reqs.find(ticket);
    if (it == S->s.reqs.end()) mx::fail(MX_EINVAL, "unknown ticket");
    if (!it->second->done) mx::fail(MX_EINVAL, "request still running");
    S->s.reqs.erase(it);
    return MX_OK;
  } catch (const Error &e) {
    mx::set_error(e.code, e.msg);
    return e.code;
  } catch (const std::bad_alloc &) {
    mx::set_error(MX_ENOMEM, "host allocation failed");
    return MX_ENOMEM;
  } catch (const std::exception &e) {
    mx::set_error(MX_EINVAL, e.what());
    return MX_EINVAL;
  }
}

int mx_server_stats(mx_server *S, uint64_t *budget, uint64_t *peak_used, int *max_admitted) {
  try {
    if (!S) mx::fail(MX_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(S->s.mu);
    if (budget) *budget = S->s.budget;
    if (peak_used) *peak_used = S->s.peak;
    if (max_admitted) *max_admitted = S->s.max_admitted;
    return MX_OK;
  } catch (const Error &e) {
    mx::set_error(e.code, e.msg);
    return e.code;
  } catch (const std::bad_alloc &) {
    mx::set_error(MX_ENOMEM, "host allocation failed");
    return MX_ENOMEM;
  } catch (const std::exception &e) {
    mx::set_error(MX_EINVAL, e.what());
    return MX_EINVAL;
  }
}

int mx_server_batch_stats(mx_server *S, uint64_t *batches, uint64_t *applications) {
  try {
    if (!S) mx::fail(MX_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(S->s.batcher.mu);
    if (batches) *batches = S->s.batcher.batches;
    if (applications) *applications = S->s.batcher.applications;
    return MX_OK;
  } catch (const Error &e) {
    mx::set_error(e.code, e.msg);
    return e.code;
  }
}

int mx_server_inject_enomem(mx_server *S, int n) {
  try {
    if (!S || n < 0) mx::fail(MX_EINVAL, "NULL server or negative count");
    S->s.inject_enomem.store(n);
    return MX_OK;
  } catch (const Error &e) {
    mx::set_error(e.code, e.msg);
    return e.code;
  }
}

void mx_server_destroy(mx_server *S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->s.mu);
    S->s.stop = true;
  }
  S->s.cv_queue.notify_all();
  for (auto &t : S->s.workers) t.join();
  S->s.batcher.finish();
  delete S;
}

}  // extern "C"
