// extern "C" entry points of libmx: argument checks, error capture, handle lifetimes.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "objects.hpp"

namespace mx {
thread_local hipStream_t t_alloc_stream = nullptr;
thread_local int t_alloc_scoped = 0;
static thread_local std::string g_last_error;
void set_error(int code, const std::string &msg) {
  (void)code;
  g_last_error = msg;
}
[[noreturn]] void fail(int code, const std::string &msg) { throw Error{code, msg}; }
uint64_t next_object_id() {
  static std::atomic<uint64_t> counter{1};
  return counter.fetch_add(1);
}
}  // namespace mx

using mx::Error;

#define MX_GUARD(...)                                               \
  try {                                                             \
    __VA_ARGS__;                                                    \
    return MX_OK;                                                   \
  } catch (const Error &e) {                                        \
    mx::set_error(e.code, e.msg);                                   \
    return e.code;                                                  \
  } catch (const std::bad_alloc &) {                                \
    mx::set_error(MX_ENOMEM, "host allocation failed");             \
    return MX_ENOMEM;                                               \
  } catch (const std::exception &e) {                               \
    mx::set_error(MX_EINVAL, e.what());                             \
    return MX_EINVAL;                                               \
  }

#define MX_REQUIRE(cond, msg) \
  if (!(cond)) mx::fail(MX_EINVAL, msg)

static void bind_device(int dev) { MX_HIP(hipSetDevice(dev)); }

extern "C" {

const char *mx_last_error(void) { return mx::g_last_error.c_str(); }
int mx_version(void) { return 100; }

int mx_ctx_create(int device, mx_ctx **out) {
  MX_GUARD({
    MX_REQUIRE(out, "out is NULL");
    int n = 0;
    MX_HIP(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) mx::fail(MX_EDEVICE, "no such HIP device");
    hipDeviceProp_t prop;
    MX_HIP(hipGetDeviceProperties(&prop, device));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
      mx::fail(MX_EDEVICE, std::string("libmx is built for gfx950, device is ") + prop.gcnArchName);
    bind_device(device);
    auto c = std::make_unique<mx_ctx>();
    c->device = device;
    c->cus = prop.multiProcessorCount;
    mx::noalloc_scratch_init(device);
    MX_HIP(hipHostMalloc((void **)&c->pinned, 4096, hipHostMallocDefault));
    *out = c.release();
  });
}

void mx_ctx_destroy(mx_ctx *ctx) {
  if (!ctx) return;
  if (hipSetDevice(ctx->device) == hipSuccess && hipDeviceSynchronize() == hipSuccess) {
    mx::big_trim(ctx->device);
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, ctx->device) == hipSuccess) (void)hipMemPoolTrimTo(pool, 0);
  }
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  delete ctx;
}

int mx_mesh_box(int nx, int ny, int nz, double lx, double ly, double lz, mx_mesh **out) {
  MX_GUARD({
    MX_REQUIRE(out, "out is NULL");
    MX_REQUIRE(nx >= 1 && ny >= 1 && nz >= 1, "mesh: need at least one cube per axis");
    MX_REQUIRE(lx > 0 && ly > 0 && lz > 0, "mesh: lengths must be positive");
    MX_REQUIRE((double)(nx + 1) * (ny + 1) * (nz + 1) < 2.0e9, "mesh: too many vertices");
    auto m = std::make_unique<mx_mesh>();
    mx::build_mesh(m->m, nx, ny, nz, lx, ly, lz);
    *out = m.release();
  });
}

int mx_mesh_sizes(const mx_mesh *m, int64_t *nv, int64_t *nt, int64_t *ne, int64_t *nbf) {
  MX_GUARD({
    MX_REQUIRE(m, "mesh is NULL");
    if (nv) *nv = m->m.nv;
    if (nt) *nt = m->m.nt;
    if (ne) *ne = m->m.ne;
    if (nbf) *nbf = (int64_t)m->m.bface_vert.size() / 3;
  });
}

int mx_mesh_export(const mx_mesh *m, int32_t *tet_vert, int32_t *edge_vert, int32_t *tet_edge,
                   int8_t *tet_edge_sign, int32_t *bface_vert) {
  MX_GUARD({
    MX_REQUIRE(m, "mesh is NULL");
    const auto &M = m->m;
    if (tet_vert) std::memcpy(tet_vert, M.tet_vert.data(), M.tet_vert.size() * 4);
    if (edge_vert) std::memcpy(edge_vert, M.edge_vert.data(), M.edge_vert.size() * 4);
    if (tet_edge) std::memcpy(tet_edge, M.tet_edge.data(), M.tet_edge.size() * 4);
    if (tet_edge_sign) std::memcpy(tet_edge_sign, M.tet_sign.data(), M.tet_sign.size());
    if (bface_vert) std::memcpy(bface_vert, M.bface_vert.data(), M.bface_vert.size() * 4);
  });
}

void mx_mesh_destroy(mx_mesh *m) { delete m; }

int mx_matrix_assemble(mx_ctx *ctx, const mx_mesh *m, double k, double xi, int bc, mx_matrix **out) {
  MX_GUARD({
    MX_REQUIRE(m && out, "NULL argument");
    MX_REQUIRE(bc == MX_BC_PEC || bc == MX_BC_IMPEDANCE, "unknown boundary condition");
    MX_REQUIRE(std::isfinite(k) && std::isfinite(xi) && k > 0, "need finite k > 0 and finite xi");
    auto A = std::make_unique<mx_matrix>();
    A->k = k, A->xi = xi, A->bc = bc;
    mx::assemble_global(m->m, k, xi, bc, A->h);
    if (ctx) {
      bind_device(ctx->device);
      A->device = ctx->device;
      mx::matrix_upload(A.get());
    }
    *out = A.release();
  });
}

int mx_matrix_assemble_order(mx_ctx *ctx, const mx_mesh *m, int order, double k, double xi, int bc,
                             mx_matrix **out) {
  MX_GUARD({
    MX_REQUIRE(m && out, "NULL argument");
    MX_REQUIRE(order == 1 || order == 2, "order must be 1 or 2");
    MX_REQUIRE(bc == MX_BC_PEC || bc == MX_BC_IMPEDANCE, "unknown boundary condition");
    MX_REQUIRE(std::isfinite(k) && std::isfinite(xi) && k > 0, "need finite k > 0 and finite xi");
    auto A = std::make_unique<mx_matrix>();
    A->k = k, A->xi = xi, A->bc = bc, A->order = order;
    if (order == 2) mx::assemble_order2(m->m, m->order2(), k, xi, bc, A->h);
    else mx::assemble_global(m->m, k, xi, bc, A->h);
    if (ctx) {
      bind_device(ctx->device);
      A->device = ctx->device;
      mx::matrix_upload(A.get());
    }
    *out = A.release();
  });
}

int mx_weight_assemble_order(mx_ctx *ctx, const mx_mesh *m, int order, double k, int bc,
                             mx_matrix **out) {
  MX_GUARD({
    MX_REQUIRE(m && out, "NULL argument");
    MX_REQUIRE(order == 1 || order == 2, "order must be 1 or 2");
    MX_REQUIRE(bc == MX_BC_PEC || bc == MX_BC_IMPEDANCE, "unknown boundary condition");
    MX_REQUIRE(std::isfinite(k) && k >= 0, "need finite k >= 0");
    auto D = std::make_unique<mx_matrix>();
    D->k = k, D->xi = 0, D->bc = bc, D->weight = true, D->order = order;
    if (order == 2) mx::assemble_order2(m->m, m->order2(), k, 0.0, bc, D->h, true);
    else mx::assemble_global(m->m, k, 0.0, bc, D->h, true);
    if (ctx) {
      bind_device(ctx->device);
      D->device = ctx->device;
      mx::matrix_upload(D.get());
    }
    *out = D.release();
  });
}

int mx_mesh_order2_sizes(const mx_mesh *m, int64_t *n_face, int64_t *n_dof) {
  MX_GUARD({
    MX_REQUIRE(m, "mesh is NULL");
    const mx::Order2 &o = m->order2();
    if (n_face) *n_face = o.F;
    if (n_dof) *n_dof = o.N;
  });
}

int mx_mesh_order2_export(const mx_mesh *m, int32_t *face_vert, int32_t *tet_face,
                          uint8_t *dof_boundary) {
  MX_GUARD({
    MX_REQUIRE(m, "mesh is NULL");
    const mx::Order2 &o = m->order2();
    if (face_vert) std::memcpy(face_vert, o.face_vert.data(), o.face_vert.size() * 4);
    if (tet_face) std::memcpy(tet_face, o.tet_face.data(), o.tet_face.size() * 4);
    if (dof_boundary) std::memcpy(dof_boundary, o.dof_boundary.data(), o.dof_boundary.size());
  });
}

int mx_partition_order2_export(const mx_mesh *m, const mx_partition *p, int kind, int64_t *offsets,
                               int32_t *loc2glob, int32_t *owner) {
  MX_GUARD({
    MX_REQUIRE(m && p && offsets, "NULL argument");
    MX_REQUIRE(kind >= MX_AS && kind <= MX_ORAS, "unknown kind");
    MX_REQUIRE((int64_t)p->p.part0.size() == m->m.nt, "partition and mesh disagree");
    std::vector<std::vector<int32_t>> sets;
    std::vector<int32_t> own;
    mx::order2_sets(m->m, m->order2(), p->p, kind, sets, own);
    int64_t o = 0;
    for (int l = 0; l < p->p.nsub; ++l) {
      offsets[l] = o;
      if (loc2glob) std::memcpy(loc2glob + o, sets[l].data(), sets[l].size() * 4);
      o += (int64_t)sets[l].size();
    }
    offsets[p->p.nsub] = o;
    if (owner) std::memcpy(owner, own.data(), own.size() * 4);
  });
}

int mx_weight_assemble(mx_ctx *ctx, const mx_mesh *m, double k, int bc, mx_matrix **out) {
  MX_GUARD({
    MX_REQUIRE(m && out, "NULL argument");
    MX_REQUIRE(bc == MX_BC_PEC || bc == MX_BC_IMPEDANCE, "unknown boundary condition");
    MX_REQUIRE(std::isfinite(k) && k >= 0, "need finite k >= 0");
    auto D = std::make_unique<mx_matrix>();
    D->k = k, D->xi = 0, D->bc = bc, D->weight = true;
    mx::assemble_global(m->m, k, 0.0, bc, D->h, true);
    if (ctx) {
      bind_device(ctx->device);
      D->device = ctx->device;
      mx::matrix_upload(D.get());
    }
    *out = D.release();
  });
}

int mx_matrix_upload(mx_ctx *ctx, mx_matrix *A) {
  MX_GUARD({
    MX_REQUIRE(ctx && A, "NULL argument");
    MX_REQUIRE(!A->rowptr.p, "matrix already has a device copy");
    bind_device(ctx->device);
    A->device = ctx->device;
    mx::matrix_upload(A);
  });
}

int mx_matrix_sizes(const mx_matrix *A, int64_t *n, int64_t *nnz) {
  MX_GUARD({
    MX_REQUIRE(A, "matrix is NULL");
    if (n) *n = A->h.n;
    if (nnz) *nnz = A->h.nnz();
  });
}

int mx_matrix_export(const mx_matrix *A, int64_t *rowptr, int32_t *col, double *val) {
  MX_GUARD({
    MX_REQUIRE(A, "matrix is NULL");
    if (rowptr) std::memcpy(rowptr, A->h.rowptr.data(), A->h.rowptr.size() * 8);
    if (col) std::memcpy(col, A->h.col.data(), A->h.col.size() * 4);
    if (val) std::memcpy(val, A->h.val.data(), A->h.val.size() * 8);
  });
}

void mx_matrix_destroy(mx_matrix *A) { delete A; }

int mx_spmv(mx_ctx *ctx, const mx_matrix *A, const void *x_dev, void *y_dev, void *stream) {
  MX_GUARD({
    MX_REQUIRE(ctx && A && x_dev && y_dev, "NULL argument");
    MX_REQUIRE(A->rowptr.p, "matrix has no device copy (assembled without a context)");
    MX_REQUIRE(x_dev != y_dev, "x and y must not overlap");
    bind_device(ctx->device);
    mx::spmv_run(A, x_dev, y_dev, false, (hipStream_t)stream);
  });
}

int mx_rhs_gaussian(const mx_mesh *m, int bc, const double center[3], const double pol[3],
                    double sigma, double *f_host) {
  MX_GUARD({
    MX_REQUIRE(m && center && pol && f_host, "NULL argument");
    MX_REQUIRE(sigma > 0, "sigma must be positive");
    mx::rhs_gaussian(m->m, bc, center, pol, sigma, f_host);
  });
}

int mx_partition_box(const mx_mesh *m, int px, int py, int pz, const int32_t *cx,
                     const int32_t *cy, const int32_t *cz, int layers, mx_partition **out) {
  MX_GUARD({
    MX_REQUIRE(m && out, "NULL argument");
    auto p = std::make_unique<mx_partition>();
    mx::build_partition(m->m, px, py, pz, cx, cy, cz, layers, p->p);
    *out = p.release();
  });
}

int mx_partition_sizes(const mx_partition *p, int kind, int32_t *n_sub, int64_t *total) {
  MX_GUARD({
    MX_REQUIRE(p, "partition is NULL");
    MX_REQUIRE(kind >= MX_AS && kind <= MX_ORAS, "unknown kind");
    if (n_sub) *n_sub = p->p.nsub;
    if (total) {
      int64_t t = 0;
      for (const auto &s : p->p.set(kind)) t += (int64_t)s.size();
      *total = t;
    }
  });
}

int mx_partition_export(const mx_partition *p, int kind, int64_t *offsets, int32_t *loc2glob,
                        int32_t *owner, int64_t *n_tet_local) {
  MX_GUARD({
    MX_REQUIRE(p, "partition is NULL");
    MX_REQUIRE(kind >= MX_AS && kind <= MX_ORAS, "unknown kind");
    const auto &sets = p->p.set(kind);
    int64_t o = 0;
    for (int l = 0; l < p->p.nsub; ++l) {
      if (offsets) offsets[l] = o;
      if (loc2glob) std::memcpy(loc2glob + o, sets[l].data(), sets[l].size() * 4);
      if (n_tet_local) n_tet_local[l] = (int64_t)p->p.tets[l].size();
      o += (int64_t)sets[l].size();
    }
    if (offsets) offsets[p->p.nsub] = o;
    if (owner) std::memcpy(owner, p->p.owner.data(), p->p.owner.size() * 4);
  });
}

void mx_partition_destroy(mx_partition *p) { delete p; }

int mx_local_problem(const mx_mesh *m, const mx_matrix *A, const mx_partition *p,
                     const mx_precond_opts *opts, int l, int64_t *n, int64_t *nnz, int64_t *rowptr,
                     int32_t *col, double *val, int32_t *perm, int32_t *first) {
  MX_GUARD({
    MX_REQUIRE(m && A && p && opts && n && nnz, "NULL argument");
    MX_REQUIRE(l >= 0 && l < p->p.nsub, "subdomain out of range");
    MX_REQUIRE(opts->kind >= MX_AS && opts->kind <= MX_ORAS, "unknown kind");
    MX_REQUIRE(A->h.n == m->ndof(A->order), "matrix and mesh disagree");
    MX_REQUIRE((int64_t)p->p.part0.size() == m->m.nt, "partition and mesh disagree");
    const auto &M = m->m;
    mx::LocalCSR a;
    std::vector<int32_t> g2l(A->h.n, -1);
    if (A->order == 2) {
      const mx::Order2 &o2 = m->order2();
      std::vector<std::vector<int32_t>> sets;
      std::vector<int32_t> own;
      mx::order2_sets(M, o2, p->p, opts->kind, sets, own);
      if (opts->kind == MX_ORAS) {
        std::vector<int32_t> tstamp(M.nt, -1);
        mx::local_impedance2(M, o2, A->k, opts->xi_prec, A->bc, p->p.tets[l], sets[l], a, g2l, tstamp);
      } else {
        mx::local_minor(o2.dof_boundary.data(), A->h, A->bc, sets[l], a, g2l);
      }
    } else if (opts->kind == MX_ORAS) {
      const auto &sets = p->p.set(opts->kind);
      mx::KuhnElements ke;
      mx::kuhn_elements(M.lx / M.nx, M.ly / M.ny, M.lz / M.nz, ke);
      std::vector<int32_t> tstamp(M.nt, -1);
      mx::local_impedance(M, ke, A->k, opts->xi_prec, A->bc, p->p.tets[l], sets[l], a, g2l, tstamp);
    } else {
      mx::local_minor(M.edge_on_boundary.data(), A->h, A->bc, p->p.set(opts->kind)[l], a, g2l);
    }
    *n = a.n;
    *nnz = (int64_t)a.col.size();
    if (rowptr) std::memcpy(rowptr, a.rowptr.data(), a.rowptr.size() * 8);
    if (col) std::memcpy(col, a.col.data(), a.col.size() * 4);
    if (val) std::memcpy(val, a.val.data(), a.val.size() * 8);
    if (perm || first) {
      mx::Skyline s;
      mx::build_skyline(a, s);
      if (perm) std::memcpy(perm, s.perm.data(), s.perm.size() * 4);
      if (first) std::memcpy(first, s.first.data(), s.first.size() * 4);
    }
  });
}

int mx_precond_setup(mx_ctx *ctx, const mx_matrix *A, const mx_mesh *m, const mx_partition *p,
                     const mx_precond_opts *opts, mx_precond **out) {
  MX_GUARD({
    MX_REQUIRE(ctx && A && m && p && opts && out, "NULL argument");
    bind_device(ctx->device);
    auto P = std::make_unique<mx_precond>();
    mx::precond_setup(ctx, A, m, p, opts, P.get(), nullptr);
    *out = P.release();
  });
}

int mx_precond_plan(mx_ctx *ctx, const mx_matrix *A, const mx_mesh *m, const mx_partition *p,
                    const mx_precond_opts *opts, mx_precond **out, uint64_t *device_bytes) {
  MX_GUARD({
    MX_REQUIRE(A && m && p && opts && out, "NULL argument");
    if (ctx) bind_device(ctx->device);
    auto P = std::make_unique<mx_precond>();
    P->plan = std::make_unique<mx::PrecondPlan>();
    mx::precond_plan(ctx, A, m, p, opts, P.get(), *P->plan);
    if (device_bytes) *device_bytes = P->plan->device_bytes;
    *out = P.release();
  });
}

int mx_precond_stage(mx_ctx *ctx, mx_precond *P) {
  MX_GUARD({
    MX_REQUIRE(ctx && P, "NULL argument");
    MX_REQUIRE(P->plan, "preconditioner is already materialised");
    MX_REQUIRE(!P->staged, "preconditioner is already staged");
    MX_REQUIRE(P->device < 0 || ctx->device == P->device, "preconditioner was planned for another device");
    bind_device(ctx->device);
    P->device = ctx->device;
    mx::set_sweep_grid(P, ctx->cus);
    mx::precond_stage(P, *P->plan);
  });
}

int mx_precond_materialize(mx_ctx *ctx, mx_precond *P, void *stream) {
  MX_GUARD({
    MX_REQUIRE(ctx && P, "NULL argument");
    MX_REQUIRE(P->plan, "preconditioner is already materialised");
    MX_REQUIRE(P->device < 0 || ctx->device == P->device, "preconditioner was planned for another device");
    bind_device(ctx->device);
    P->device = ctx->device;
    mx::set_sweep_grid(P, ctx->cus);
    mx::precond_materialize(P, *P->plan, (hipStream_t)stream);
    P->plan.reset();
  });
}

int mx_precond_apply(mx_ctx *ctx, mx_precond *P, const void *v_dev, void *z_dev, void *stream) {
  MX_GUARD({
    MX_REQUIRE(ctx && P && v_dev && z_dev, "NULL argument");
    MX_REQUIRE(!P->plan, "preconditioner is planned but not materialised");
    MX_REQUIRE(v_dev != z_dev, "v and z must be distinct");
    MX_REQUIRE(!mx::coarse_incomplete(P), "coarse level planned but not built (mx_precond_add_coarse)");
    mx::precond_refuse_failed(P);
    bind_device(ctx->device);
    mx::precond_apply(P, v_dev, z_dev, (hipStream_t)stream);
  });
}

int mx_precond_get_info(const mx_precond *P, mx_precond_info *info) {
  MX_GUARD({
    MX_REQUIRE(P && info, "NULL argument");
    *info = P->info;
  });
}

int mx_precond_export_perm(const mx_precond *P, int l, int64_t n, int32_t *perm, int32_t *first) {
  MX_GUARD({
    MX_REQUIRE(P, "NULL argument");
    MX_REQUIRE(l >= 0 && l < P->nsub, "subdomain out of range");
    const auto &s = P->sky[l];
    MX_REQUIRE(n == (int64_t)s.perm.size(), "n differs from the subdomain's DOF count");
    if (perm) std::memcpy(perm, s.perm.data(), s.perm.size() * 4);
    if (first) std::memcpy(first, s.first.data(), s.first.size() * 4);
  });
}

int mx_precond_export_diag(const mx_precond *P, int l, int64_t n, double *d) {
  MX_GUARD({
    MX_REQUIRE(P && d, "NULL argument");
    MX_REQUIRE(!P->plan, "preconditioner is planned but not materialised");
    MX_REQUIRE(l >= 0 && l < P->nsub, "subdomain out of range");
    const auto &s = P->sky[l];
    MX_REQUIRE(n == (int64_t)s.perm.size(), "n differs from the subdomain's DOF count");
    bind_device(P->device);
    mx::precond_export_diag(P, l, d);
  });
}

int mx_precond_sweep_timing(mx_precond *P, int enable, int64_t *launches, double *ms_forward,
                            double *ms_backward) {
  MX_GUARD({
    MX_REQUIRE(P, "NULL argument");
    MX_REQUIRE(!P->plan, "preconditioner is planned but not materialised");
    bind_device(P->device);
    mx::precond_timing(P, enable, launches, ms_forward, ms_backward);
  });
}

int mx_precond_autotune(mx_ctx *ctx, mx_precond *P, void *stream, int32_t *best_grid,
                        double *best_ms) {
  MX_GUARD({
    MX_REQUIRE(ctx && P, "NULL argument");
    MX_REQUIRE(!P->plan, "preconditioner is planned but not materialised");
    mx::precond_refuse_failed(P);
    bind_device(ctx->device);
    mx::precond_autotune(ctx, P, (hipStream_t)stream, best_grid, best_ms);
  });
}

int mx_precond_tune_factor(mx_ctx *ctx, const mx_matrix *A, const mx_mesh *m, const mx_partition *p,
                           const mx_precond_opts *opts, void *stream, int32_t *best_schedule,
                           int32_t *best_width, double *best_ms, double *ms_each) {
  MX_GUARD({
    MX_REQUIRE(ctx && A && m && p && opts, "NULL argument");
    bind_device(ctx->device);
    mx::precond_tune_factor(ctx, A, m, p, opts, (hipStream_t)stream, best_schedule, best_width,
                            best_ms, ms_each);
  });
}

int mx_precond_check(mx_precond *P) {
  MX_GUARD({
    MX_REQUIRE(P, "NULL argument");
    MX_REQUIRE(!P->plan, "preconditioner is planned but not materialised");
    bind_device(P->device);
    MX_HIP(hipDeviceSynchronize());
    mx::precond_check(P);
  });
}

void mx_precond_destroy(mx_precond *P) { delete P; }

int mx_gmres(mx_ctx *ctx, const mx_matrix *A, mx_precond *P, const void *b_dev, void *x_dev,
             const mx_gmres_opts *opts, mx_gmres_stats *stats, double *res_hist, void *stream) {
  MX_GUARD({
    MX_REQUIRE(ctx && A && b_dev && x_dev && opts && stats, "NULL argument");
    MX_REQUIRE(b_dev != x_dev, "b and x must be distinct");
    MX_REQUIRE(A->rowptr.p, "matrix has no device copy");
    MX_REQUIRE(!P || P->E == A->h.n, "preconditioner and matrix sizes differ");
    MX_REQUIRE(!P || !P->plan, "preconditioner is planned but not materialised");
    MX_REQUIRE(!P || !mx::coarse_incomplete(P), "coarse level planned but not built (mx_precond_add_coarse)");
    if (P) mx::precond_refuse_failed(P);
    bind_device(ctx->device);
    mx::gmres_run(ctx, A, P, b_dev, x_dev, opts, stats, res_hist, (hipStream_t)stream);
  });
}

// the nested coarse mesh of a common ratio (exact midpoint values of eq:restriction)
static mx::CoarseSpec ratio_spec(const mx_mesh *m, int ratio) {
  MX_REQUIRE(ratio >= 1 && m->m.nx % ratio == 0 && m->m.ny % ratio == 0 && m->m.nz % ratio == 0,
             "the coarse ratio must divide the cube count of every axis");
  mx::CoarseSpec cs;
  cs.cn[0] = m->m.nx / ratio, cs.cn[1] = m->m.ny / ratio, cs.cn[2] = m->m.nz / ratio;
  cs.nq = 0;
  return cs;
}

static mx::CoarseSpec box_spec(int cnx, int cny, int cnz, int nq) {
  MX_REQUIRE(cnx >= 1 && cny >= 1 && cnz >= 1, "coarse cube counts must be >= 1");
  MX_REQUIRE(nq >= 1 && nq <= 64, "quadrature points per fine edge must be 1 .. 64");
  mx::CoarseSpec cs;
  cs.cn[0] = cnx, cs.cn[1] = cny, cs.cn[2] = cnz;
  cs.nq = nq;
  return cs;
}

static int add_coarse(mx_ctx *ctx, mx_precond *P, const mx_matrix *A, const mx_mesh *m,
                      const mx::CoarseSpec &cs, int combine, void *stream) {
  MX_REQUIRE(!P->plan, "preconditioner is planned but not materialised");
  mx::precond_refuse_failed(P);
  bind_device(ctx->device);
  mx::coarse_setup(ctx, P, A, m, cs, combine, (hipStream_t)stream);
  return MX_OK;
}

int mx_precond_add_coarse(mx_ctx *ctx, mx_precond *P, const mx_matrix *A, const mx_mesh *m,
                          int ratio, int combine, void *stream) {
  MX_GUARD({
    MX_REQUIRE(ctx && P && A && m, "NULL argument");
    add_coarse(ctx, P, A, m, ratio_spec(m, ratio), combine, stream);
  });
}

int mx_precond_add_coarse_box(mx_ctx *ctx, mx_precond *P, const mx_matrix *A, const mx_mesh *m,
                              int cnx, int cny, int cnz, int nq, int combine, void *stream) {
  MX_GUARD({
    MX_REQUIRE(ctx && P && A && m, "NULL argument");
    add_coarse(ctx, P, A, m, box_spec(cnx, cny, cnz, nq), combine, stream);
  });
}

int mx_precond_plan_coarse(mx_precond *P, const mx_matrix *A, const mx_mesh *m, int ratio,
                           int combine) {
  MX_GUARD({
    MX_REQUIRE(P && A && m, "NULL argument");
    mx::coarse_plan(P, A, m, ratio_spec(m, ratio), combine);
  });
}

int mx_precond_plan_coarse_box(mx_precond *P, const mx_matrix *A, const mx_mesh *m, int cnx,
                               int cny, int cnz, int nq, int combine) {
  MX_GUARD({
    MX_REQUIRE(P && A && m, "NULL argument");
    mx::coarse_plan(P, A, m, box_spec(cnx, cny, cnz, nq), combine);
  });
}

static void coarse_operators(const mx_mesh *m, const mx_matrix *A, const mx::CoarseSpec &cs,
                             int64_t *n_coarse, int64_t *nnz_r, int64_t *nnz_a, int64_t *r_rowptr,
                             int32_t *r_col, double *r_val, int64_t *a_rowptr, int32_t *a_col,
                             double *a_val) {
  MX_REQUIRE(A->h.n == m->ndof(A->order), "matrix and mesh sizes differ");
  mx::Mesh cm;
  mx::HostCSR R0, R0T, A0;
  mx::coarse_restriction(m->m, cs, A->order, A->h.n, A->bc, cm, R0, R0T);
  mx::galerkin_coarse(A->h, R0, R0T, cm, A->bc, A0);
  const bool sizes_only = !r_rowptr && !r_col && !r_val && !a_rowptr && !a_col && !a_val;
  if (!sizes_only) {
    MX_REQUIRE(*n_coarse == R0.n && *nnz_r == R0.nnz() && *nnz_a == A0.nnz(),
               "buffer sizes differ from the coarse operators' (query them first)");
    if (r_rowptr) std::copy(R0.rowptr.begin(), R0.rowptr.end(), r_rowptr);
    if (r_col) std::copy(R0.col.begin(), R0.col.end(), r_col);
    if (r_val)
      for (int64_t q = 0; q < R0.nnz(); ++q) r_val[q] = R0.val[2 * q];
    if (a_rowptr) std::copy(A0.rowptr.begin(), A0.rowptr.end(), a_rowptr);
    if (a_col) std::copy(A0.col.begin(), A0.col.end(), a_col);
    if (a_val) std::copy(A0.val.begin(), A0.val.end(), a_val);
  }
  *n_coarse = R0.n;
  *nnz_r = R0.nnz();
  *nnz_a = A0.nnz();
}

int mx_coarse_operators(const mx_mesh *m, const mx_matrix *A, int ratio, int64_t *n_coarse,
                        int64_t *nnz_r, int64_t *nnz_a, int64_t *r_rowptr, int32_t *r_col,
                        double *r_val, int64_t *a_rowptr, int32_t *a_col, double *a_val) {
  MX_GUARD({
    MX_REQUIRE(m && A && n_coarse && nnz_r && nnz_a, "NULL argument");
    coarse_operators(m, A, ratio_spec(m, ratio), n_coarse, nnz_r, nnz_a, r_rowptr, r_col, r_val,
                     a_rowptr, a_col, a_val);
  });
}

int mx_coarse_operators_box(const mx_mesh *m, const mx_matrix *A, int cnx, int cny, int cnz, int nq,
                            int64_t *n_coarse, int64_t *nnz_r, int64_t *nnz_a, int64_t *r_rowptr,
                            int32_t *r_col, double *r_val, int64_t *a_rowptr, int32_t *a_col,
                            double *a_val) {
  MX_GUARD({
    MX_REQUIRE(m && A && n_coarse && nnz_r && nnz_a, "NULL argument");
    coarse_operators(m, A, box_spec(cnx, cny, cnz, nq), n_coarse, nnz_r, nnz_a, r_rowptr, r_col,
                     r_val, a_rowptr, a_col, a_val);
  });
}

int mx_precond_coarse_export(const mx_precond *P, int64_t *n_coarse, int64_t *nnz_r, int64_t *nnz_a,
                             int64_t *r_rowptr, int32_t *r_col, double *r_val, int64_t *a_rowptr,
                             int32_t *a_col, double *a_val) {
  MX_GUARD({
    MX_REQUIRE(P, "NULL argument");
    mx::coarse_export(P, n_coarse, nnz_r, nnz_a, r_rowptr, r_col, r_val, a_rowptr, a_col, a_val);
  });
}

int mx_gmres_noalloc(mx_ctx *ctx, const mx_matrix *A, mx_precond *P, const void *b_dev, void *x_dev,
                     const mx_gmres_opts *opts, mx_gmres_stats *stats, double *res_hist, void *stream) {
  MX_GUARD({
    MX_REQUIRE(ctx && A && b_dev && x_dev && opts && stats, "NULL argument");
    MX_REQUIRE(b_dev != x_dev, "b and x must be distinct");
    MX_REQUIRE(A->rowptr.p, "matrix has no device copy");
    MX_REQUIRE(!P || P->E == A->h.n, "preconditioner and matrix sizes differ");
    MX_REQUIRE(!P || !P->plan, "preconditioner is planned but not materialised");
    MX_REQUIRE(!P || !mx::coarse_incomplete(P), "coarse level planned but not built (mx_precond_add_coarse)");
    if (P) mx::precond_refuse_failed(P);
    bind_device(ctx->device);
    mx::gmres_run(ctx, A, P, b_dev, x_dev, opts, stats, res_hist, (hipStream_t)stream, true);
  });
}

int mx_gmres_weighted(mx_ctx *ctx, const mx_matrix *A, mx_precond *P, const mx_matrix *D,
                      const void *b_dev, void *x_dev, const mx_gmres_opts *opts,
                      mx_gmres_stats *stats, double *res_hist, void *stream) {
  MX_GUARD({
    MX_REQUIRE(ctx && A && b_dev && x_dev && opts && stats, "NULL argument");
    MX_REQUIRE(b_dev != x_dev, "b and x must be distinct");
    MX_REQUIRE(A->rowptr.p, "matrix has no device copy");
    MX_REQUIRE(!D || (D->rowptr.p && D->h.n == A->h.n && D->order == A->order),
               "weight needs a device copy of A's size and element order");
    MX_REQUIRE(!P || P->E == A->h.n, "preconditioner and matrix sizes differ");
    MX_REQUIRE(!P || !P->plan, "preconditioner is planned but not materialised");
    MX_REQUIRE(!P || !mx::coarse_incomplete(P), "coarse level planned but not built (mx_precond_add_coarse)");
    if (P) mx::precond_refuse_failed(P);
    bind_device(ctx->device);
    mx::gmres_run(ctx, A, P, b_dev, x_dev, opts, stats, res_hist, (hipStream_t)stream, false, D);
  });
}

int mx_selftest(mx_ctx *ctx, double *err64, double *err32) {
  MX_GUARD({
    MX_REQUIRE(ctx && err64 && err32, "NULL argument");
    bind_device(ctx->device);
    mx::selftest_run(err64, err32);
  });
}

int mx_selftest_host(int64_t n_items, int64_t fail_item, int fail_code, int64_t *items_run) {
  MX_GUARD({
    MX_REQUIRE(n_items >= 0 && items_run, "bad arguments");
    MX_REQUIRE(fail_code == MX_EINVAL || fail_code == MX_ENOMEM, "fail_code must be MX_EINVAL or MX_ENOMEM");
    std::vector<std::atomic<int>> seen(n_items);
    for (auto &x : seen) x.store(0);
    std::atomic<int64_t> ran(0);
    auto item = [&](int64_t i) {
      if (i == fail_item) {
        if (fail_code == MX_ENOMEM) throw std::bad_alloc();
        mx::fail(MX_EINVAL, "planted failure of item " + std::to_string(i));
      }
      seen[i].fetch_add(1);
      ran.fetch_add(1);
    };
    *items_run = 0;
    try {
      mx::parallel_items(n_items, [&](auto next) {
        for (int64_t i; (i = next()) >= 0;) item(i);
      });
      mx::parallel_for(n_items, [&](int64_t a, int64_t b) {
        for (int64_t i = a; i < b; ++i) item(i);
      }, 1);
    } catch (...) {
      *items_run = ran.load();
      throw;
    }
    *items_run = ran.load();
    for (auto &x : seen)
      if (x.load() != 2) mx::fail(MX_EINVAL, "host thread pool: an item did not run exactly once per pass");
  });
}

}  // extern "C"
