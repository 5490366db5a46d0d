// Definitions of the opaque C-ABI handles.
#pragma once

#include <hip/hip_runtime.h>

#include <memory>
#include <string>
#include <vector>

#include "mx_internal.hpp"

// A failed HIP call also leaves its error as the thread's last error; it is cleared here, so a
// later hipGetLastError() check (after a kernel launch) does not report it a second time.
#define MX_HIP(call)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess) {                                                               \
      (void)hipGetLastError();                                                            \
      ::mx::fail(e_ == hipErrorOutOfMemory ? MX_ENOMEM : MX_EDEVICE,                      \
                 std::string(#call) + ": " + hipGetErrorString(e_));                      \
    }                                                                                     \
  } while (0)

namespace mx {

// Stream used for device allocations and uploads made by this host thread: inside an
// AllocScope (the null stream included) buffers come from the stream-ordered allocator and are
// freed on that stream, so concurrent requests on different streams do not synchronise the whole
// device and freed memory stays mapped in the device's pool for the next setup.
extern thread_local hipStream_t t_alloc_stream;
extern thread_local int t_alloc_scoped;
struct AllocScope {
  hipStream_t prev;
  int prev_scoped;
  explicit AllocScope(hipStream_t s) : prev(t_alloc_stream), prev_scoped(t_alloc_scoped) {
    t_alloc_stream = s;
    t_alloc_scoped = 1;
  }
  ~AllocScope() {
    t_alloc_stream = prev;
    t_alloc_scoped = prev_scoped;
  }
};

// Process-wide cache of large device blocks (factor tiles, trimmed factors, big vectors):
// freed blocks stay mapped, tagged with an event recorded on their stream at release, and are
// handed out again (best fit within 1.5x of the request, after that event has completed)
// instead of being unmapped and remapped, which costs seconds for the tens of GB of a
// factorisation.  A failed allocation
// returns the cached blocks of the device to HIP and retries once.  Implemented in devcache.cpp.
constexpr size_t kBigBlock = size_t(64) << 20;
void *big_alloc(size_t n, size_t *capacity);
void big_free(void *p, size_t capacity, hipStream_t st);
void big_trim(int device);
size_t big_cached(int device);  // bytes of the device's blocks held in the cache

// Owning device buffer.
struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  size_t cap = 0;  // capacity of a cached large block
  hipStream_t st = nullptr;
  bool async = false, big = false;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  ~DevBuf() { release(); }
  void alloc(size_t n) {
    release();
    if (n == 0) n = 16;
    if (n >= kBigBlock) {
      p = big_alloc(n, &cap);
      st = t_alloc_scoped ? t_alloc_stream : nullptr;
      big = true;
    } else if (t_alloc_scoped) {
      MX_HIP(hipMallocAsync(&p, n, t_alloc_stream));
      st = t_alloc_stream;
      async = true;
    } else {
      MX_HIP(hipMalloc(&p, n));
      async = false;
    }
    bytes = n;
  }
  void release() {
    if (p) {
      if (big) big_free(p, cap, st);
      else if (async) (void)hipFreeAsync(p, st);
      else (void)hipFree(p);
    }
    p = nullptr;
    bytes = cap = 0;
    big = async = false;
  }
  template <class T>
  T *as() const { return (T *)p; }
  template <class V>
  void upload(const V &v) {
    typedef typename V::value_type T;
    alloc(v.size() * sizeof(T));
    if (!v.empty()) {
      MX_HIP(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, t_alloc_stream));
      MX_HIP(hipStreamSynchronize(t_alloc_stream));
    }
  }
};

struct Workspace {  // grow-only scratch owned by a context
  DevBuf buf;
  void *get(size_t n) {
    if (buf.bytes < n) buf.alloc(n);
    return buf.p;
  }
};

}  // namespace mx

namespace mx {
// process-wide counter: every matrix and preconditioner gets a distinct id at creation, so a
// cached graph keyed by ids never matches an object created later at the same address
uint64_t next_object_id();

// Arnoldi steps captured as HIP graphs (one per position j in the cycle), valid for one key
struct GraphCache {
  uint64_t a_id = 0, p_id = 0, d_id = 0;
  const void *ws = nullptr, *coarse = nullptr;
  int64_t n = 0;
  int m = 0;
  bool flex = false, c64 = false;
  std::vector<hipGraphExec_t> steps;
  void clear() {
    for (auto &e : steps)
      if (e) (void)hipGraphExecDestroy(e);
    steps.clear();
  }
  ~GraphCache() { clear(); }
};
}  // namespace mx

struct mx_ctx {
  int device = 0;
  int cus = 256;
  mx::Workspace krylov;
  double *pinned = nullptr;  // small host-visible status area
  mx::GraphCache graphs;
  hipStream_t capture = nullptr;  // stream the graphs are captured on (the null stream cannot be)
  ~mx_ctx() {
    graphs.clear();
    if (capture) (void)hipStreamDestroy(capture);
  }
};

struct mx_mesh {
  mx::Mesh m;
  // second-order topology and element integrals, built on first use
  mutable std::once_flag o2_once;
  mutable std::unique_ptr<mx::Order2> o2;
  const mx::Order2 &order2() const {
    std::call_once(o2_once, [this] {
      auto p = std::make_unique<mx::Order2>();
      mx::build_order2(m, *p);
      o2 = std::move(p);
    });
    return *o2;
  }
  int64_t ndof(int order) const { return order == 2 ? order2().N : m.ne; }
};

struct mx_partition {
  mx::Partition p;
};

struct mx_matrix {
  uint64_t id = mx::next_object_id();
  mx::HostCSR h;
  double k = 0, xi = 0;
  int bc = MX_BC_IMPEDANCE;
  bool weight = false;  // the Gram matrix D_k of the weighted inner product, not a Galerkin matrix
  int order = 1;        // Nedelec order of the space the matrix is assembled on (1 or 2)
  int device = 0;
  mx::DevBuf rowptr, col, val, val32;
};

namespace mx {
// Host-side product of a preconditioner setup: everything needed to materialise it on a device,
// and its exact device footprint.
struct PrecondPlan {
  std::vector<int64_t> brow_off;
  std::vector<int32_t> bfirst, blast;
  std::vector<int64_t> off;   // scatter of the permuted lower-triangle entries into the tile pool
  std::vector<double> val;
  std::vector<int32_t> glob;
  std::vector<int64_t> src, sum_ptr, sum_idx;
  std::vector<int32_t> sched_sub, sched_blk;
  std::vector<int64_t> rmeta, cmeta;  // trimmed-tile (base, row mask) pairs: tile order, block-column order
  std::vector<int64_t> cptr;          // start of each block column in cmeta
  std::vector<int64_t> scat;          // start of each subdomain's entries in off / val
  size_t device_bytes = 0;    // peak device bytes of materialising and holding the preconditioner
};
}  // namespace mx

namespace mx {
struct CoarseLevel;                 // the coarse level of a two-level preconditioner (krylov.hip)
void coarse_free(CoarseLevel *c);
}  // namespace mx

struct mx_precond {
  uint64_t id = mx::next_object_id();
  int kind = MX_ORAS, prec = MX_C128, nsub = 0, device = 0, sub_begin = 0;
  double k = 0, xi_prec = 0;       // wavenumber and absorption the local problems were built with
  int bc = MX_BC_IMPEDANCE;
  int order = 1;                    // Nedelec order of the space
  bool share = false;               // built for a resident share of the subdomains only
  // when set, one-level applications go to this function instead of being launched here (a
  // server batching the applications of several requests)
  void (*apply_hook)(void *arg, mx_precond *P, const void *vin, void *zout, hipStream_t st) = nullptr;
  void *apply_hook_arg = nullptr;
  mx::CoarseLevel *coarse = nullptr;  // set by mx_precond_add_coarse (owned)
  std::unique_ptr<mx::PrecondPlan> plan;  // set between mx_precond_plan and mx_precond_materialize
  int64_t pool_limit = 0;                 // bytes of full tiles at a time (0: what device memory allows)
  int schedule = 0;                       // factorisation schedule (MX_FACTOR_*; 0 = automatic)
  int width = 4;                          // block columns per look-ahead trailing update
  int n_groups = 0;                       // subdomain groups the factorisation ran in
  int64_t E = 0;
  int max_nb = 0;
  int64_t vec_total = 0, blocks_total = 0, tiles_total = 0;
  std::vector<mx::Skyline> sky;
  std::vector<int64_t> sub_vec_base, sub_tile_base;
  std::vector<int32_t> sub_brow_base, sub_nb;
  std::vector<int32_t> panel_pref, update_pref;  // [max_nb][nsub+1]
  std::vector<int32_t> intra_pref, next_pref, rest_pref;  // look-ahead groups: [max_nb][nsub+1]
  // device
  mx::DevBuf d_sub_nb, d_sub_brow_base, d_sub_tile_base, d_sub_vec_base;
  mx::DevBuf d_brow_off, d_bfirst, d_blast;
  mx::DevBuf pool;                          // 64x64 tiles (factorisation only)
  bool staged = false;                      // mx_precond_stage copied the metadata and entries
  mx::DevBuf d_off_all, d_val_all;          // staged scatter of the local matrices' entries
  mx::DevBuf pack, d_rmeta, d_cmeta, d_cptr;  // trimmed tiles of the factor (sweeps)
  int64_t pack_entries = 0;
  mx::DevBuf d_r, d_y, d_z;                 // local vectors (factor precision)
  mx::DevBuf d_glob, d_src, d_sum_ptr, d_sum_idx;
  mx::DevBuf d_ctrl, d_sched_sub, d_sched_blk;
  mx::DevBuf d_panel_pref, d_update_pref, d_intra_pref, d_next_pref, d_rest_pref;
  int n_items = 0, trsv_grid = 0, sweep_grid = 0;
  // MX_ESTALL or MX_EPIVOT once a device error word has been reported; the preconditioner is
  // then refused by every later application (its device flags stay set)
  int failed = 0;
  mx_precond_info info{};
  // optional per-launch timing of the sweep kernel
  bool timing = false;
  std::vector<hipEvent_t> ev_start, ev_mid, ev_stop;
  size_t n_timed = 0;
  ~mx_precond() {
    if (coarse) mx::coarse_free(coarse);
    for (auto e : ev_start) (void)hipEventDestroy(e);
    for (auto e : ev_mid) (void)hipEventDestroy(e);
    for (auto e : ev_stop) (void)hipEventDestroy(e);
  }
};

namespace mx {
// implemented in precond.hip / krylov.hip
void precond_setup(mx_ctx *ctx, const mx_matrix *A, const mx_mesh *m, const mx_partition *p,
                   const mx_precond_opts *opts, mx_precond *P, hipStream_t st);
void precond_plan(mx_ctx *ctx, const mx_matrix *A, const mx_mesh *m, const mx_partition *p,
                  const mx_precond_opts *opts, mx_precond *P, PrecondPlan &plan);
void precond_stage(mx_precond *P, PrecondPlan &plan);
// persistent sweep grid from the requested sweep_grid (0: one workgroup per compute unit)
void set_sweep_grid(mx_precond *P, int cus);
// device bytes of the full factor tiles and staged entries of all subdomains at once (the
// tile-pool cap that makes the factorisation run in one group)
size_t precond_one_group_bytes(const mx_precond *P, const PrecondPlan &plan);
// frees every device buffer of P (host state kept: P can be materialised again from its plan)
void precond_release_device(mx_precond *P);
void precond_materialize(mx_precond *P, PrecondPlan &plan, hipStream_t st);
size_t matrix_device_bytes(const mx_matrix *A);
size_t gmres_device_bytes(int64_t n, int restart, bool flexible);
// z = B^-1 v: the one-level preconditioner of P, combined with its coarse level if it has one
void precond_apply(mx_precond *P, const void *vin, void *zout, hipStream_t st);
// the one-level part alone: restriction, block sweeps, prolongation (through P's apply hook if
// it has one; precond_apply_direct launches them here in any case)
void precond_apply_level1(mx_precond *P, const void *vin, void *zout, hipStream_t st);
void precond_apply_direct(mx_precond *P, const void *vin, void *zout, hipStream_t st);
// batched one-level applications (precond.hip): bytes of one sweep job, writing P's job into a
// device array of jobs, and one launch per sweep direction over up to 16 preconditioners
size_t batch_job_bytes();
void batch_job_write(mx_precond *P, void *jobs, int slot);
constexpr int kMaxBatchJobs = 16;
void batch_apply(int njobs, const int *slots, mx_precond *const *Ps, const void *const *vin,
                 void *const *zout, const void *jobs_dev, int *bctrl, int grid_cap, hipStream_t st);
// coarse level (Sec. 3.2, 3.3): R^0 and A^0 = R^0 A R^0^T on the host (host_coarse.cpp)
void build_restriction(const Mesh &fine, const Mesh &coarse, int ratio, int bc, HostCSR &R0,
                       HostCSR &R0T);
// any coarse box mesh of the same box: each fine DOF by an nq-point Gauss rule along the edge
void build_restriction_quad(const Mesh &fine, const Mesh &coarse, int bc, int nq, HostCSR &R0,
                            HostCSR &R0T);
// the coarse mesh of a coarse level: cn cubes per axis; nq = 0 for the nested mesh of a common
// ratio (exact midpoint values), else the quadrature points per fine edge
struct CoarseSpec {
  int cn[3] = {0, 0, 0};
  int nq = 0;
  bool operator==(const CoarseSpec &o) const {
    return cn[0] == o.cn[0] && cn[1] == o.cn[1] && cn[2] == o.cn[2] && nq == o.nq;
  }
};
// validates a spec against the fine mesh (and the element order) and builds R^0 and its
// transpose with the order's column count
void coarse_restriction(const Mesh &fine, const CoarseSpec &cs, int order, int64_t ndof, int bc,
                        Mesh &coarse, HostCSR &R0, HostCSR &R0T);
void galerkin_coarse(const HostCSR &A, const HostCSR &R0, const HostCSR &R0T, const Mesh &coarse,
                     int bc, HostCSR &A0);
// host half of a coarse level (R^0, A^0, plan of its factorisation), attached to P but not usable
// until coarse_setup builds its device half (krylov.hip)
void coarse_plan(mx_precond *P, const mx_matrix *A, const mx_mesh *m, const CoarseSpec &cs,
                 int combine);
bool coarse_incomplete(const mx_precond *P);
// attaches a coarse level to the materialised one-level P built from A, or completes a planned one
void coarse_setup(mx_ctx *ctx, mx_precond *P, const mx_matrix *A, const mx_mesh *m,
                  const CoarseSpec &cs, int combine, hipStream_t st);
// host copies of R^0 and A^0 (sizes when the arrays are NULL)
void coarse_export(const mx_precond *P, int64_t *n_coarse, int64_t *nnz_r, int64_t *nnz_a,
                   int64_t *r_rowptr, int32_t *r_col, double *r_val, int64_t *a_rowptr,
                   int32_t *a_col, double *a_val);
int precond_check(mx_precond *P, hipStream_t st = nullptr);
// throws the recorded device error of P, if any (see mx_precond::failed)
void precond_refuse_failed(const mx_precond *P);
void precond_autotune(mx_ctx *ctx, mx_precond *P, hipStream_t st, int32_t *best_grid, double *best_ms);
void precond_tune_factor(mx_ctx *ctx, const mx_matrix *A, const mx_mesh *mh, const mx_partition *ph,
                         const mx_precond_opts *opts, hipStream_t st, int32_t *best_schedule,
                         int32_t *best_width, double *best_ms, double *ms_each);
void precond_export_diag(const mx_precond *P, int l, double *d);
void precond_timing(mx_precond *P, int enable, int64_t *launches, double *ms_fwd, double *ms_bwd);
void spmv_run(const mx_matrix *A, const void *x, void *y, bool c64, hipStream_t st);
void matrix_upload(mx_matrix *A);
// noalloc: the Krylov workspace is the fixed per-device scratch array (at most
// kNoAllocScratchBytes; larger requests fail with MX_EINVAL) instead of the context's workspace
// D (nullable): weighted GMRES in <v, w>_D = w^H D v (Sec. 5.2) instead of the Euclidean one
void gmres_run(mx_ctx *ctx, const mx_matrix *A, mx_precond *P, const void *b_dev, void *x_dev,
               const mx_gmres_opts *o, mx_gmres_stats *stats, double *hist, hipStream_t st,
               bool noalloc = false, const mx_matrix *D = nullptr);
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
// takes the device address of the GMRES scratch array on `device` (must be current); idempotent
void noalloc_scratch_init(int device);
void selftest_run(double *e64, double *e32);
}  // namespace mx
