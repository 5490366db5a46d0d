// Definitions of the opaque C-ABI handles.
#pragma once

#include <hip/hip_runtime.h>

#include <memory>
#include <string>
#include <vector>

#include "mx_internal.hpp"

#define MX_HIP(call)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      ::mx::fail(e_ == hipErrorOutOfMemory ? MX_ENOMEM : MX_EDEVICE,                      \
                 std::string(#call) + ": " + hipGetErrorString(e_));                      \
  } while (0)

namespace mx {

// Owning device buffer.
struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  ~DevBuf() { release(); }
  void alloc(size_t n) {
    release();
    if (n == 0) n = 16;
    MX_HIP(hipMalloc(&p, n));
    bytes = n;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  template <class T>
  T *as() const { return (T *)p; }
  template <class T>
  void upload(const std::vector<T> &v) {
    alloc(v.size() * sizeof(T));
    if (!v.empty()) MX_HIP(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
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

struct mx_ctx {
  int device = 0;
  int cus = 256;
  mx::Workspace krylov, tmp;
  double *pinned = nullptr;  // small host-visible status area
};

struct mx_mesh {
  mx::Mesh m;
};

struct mx_partition {
  mx::Partition p;
};

struct mx_matrix {
  mx::HostCSR h;
  double k = 0, xi = 0;
  int bc = MX_BC_IMPEDANCE;
  int device = 0;
  mx::DevBuf rowptr, col, val, val32;
};

struct mx_precond {
  int kind = MX_ORAS, prec = MX_C128, nsub = 0, device = 0, sub_begin = 0;
  int64_t E = 0;
  int max_nb = 0;
  int64_t vec_total = 0, blocks_total = 0, tiles_total = 0;
  std::vector<mx::Skyline> sky;
  std::vector<int64_t> sub_vec_base, sub_tile_base;
  std::vector<int32_t> sub_brow_base, sub_nb;
  std::vector<int32_t> panel_pref, update_pref;  // [max_nb][nsub+1]
  // device
  mx::DevBuf d_sub_nb, d_sub_brow_base, d_sub_tile_base, d_sub_vec_base;
  mx::DevBuf d_brow_off, d_bfirst, d_blast;
  mx::DevBuf pool;
  mx::DevBuf d_r, d_y, d_z;                 // local vectors (factor precision)
  mx::DevBuf d_glob, d_src, d_sum_ptr, d_sum_idx;
  mx::DevBuf d_flags, d_ctrl, d_sched_sub, d_sched_blk;
  mx::DevBuf d_panel_pref, d_update_pref;
  int n_items = 0, trsv_grid = 0;
  mx_precond_info info{};
  // optional per-launch timing of the sweep kernel
  bool timing = false;
  std::vector<hipEvent_t> ev_start, ev_mid, ev_stop;
  size_t n_timed = 0;
  ~mx_precond() {
    for (auto e : ev_start) (void)hipEventDestroy(e);
    for (auto e : ev_mid) (void)hipEventDestroy(e);
    for (auto e : ev_stop) (void)hipEventDestroy(e);
  }
};

namespace mx {
// implemented in precond.hip / krylov.hip
void precond_setup(mx_ctx *ctx, const mx_matrix *A, const mx_mesh *m, const mx_partition *p,
                   const mx_precond_opts *opts, mx_precond *P);
void precond_apply(mx_precond *P, const void *vin, void *zout, hipStream_t st);
int precond_check(mx_precond *P);
void precond_autotune(mx_ctx *ctx, mx_precond *P, hipStream_t st, int32_t *best_grid, double *best_ms);
void precond_timing(mx_precond *P, int enable, int64_t *launches, double *ms_fwd, double *ms_bwd);
void spmv_run(const mx_matrix *A, const void *x, void *y, bool c64, hipStream_t st);
void matrix_upload(mx_matrix *A);
void gmres_run(mx_ctx *ctx, const mx_matrix *A, mx_precond *P, const void *b_dev, void *x_dev,
               const mx_gmres_opts *o, mx_gmres_stats *stats, double *hist, hipStream_t st);
void selftest_run(double *e64, double *e32);
}  // namespace mx
