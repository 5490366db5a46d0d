// Complex CSR SpMV and right-preconditioned restarted (F)GMRES on gfx950, FP64 throughout.
//
// GMRES is the minimal-residual Krylov iteration of Sec. 5.2 with the Euclidean inner product,
// right preconditioned and stopped on the relative residual as in Sec. 6.1.  Orthogonalisation:
// classical Gram-Schmidt applied twice with deterministic blocked reductions (fixed row blocks,
// fixed reduction order); least squares: complex Givens rotations updated on the device; the host
// reads one small status record per iteration to decide whether to stop.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <mutex>
#include <random>
#include <string>

#include "device_common.hpp"
#include "objects.hpp"

namespace mx {

// ---- SpMV: 8 lanes per row --------------------------------------------------------------------------
// About 16 entries per row: eight lanes take two entries each per pass, with both entries' loads
// in flight together, and fold with three shuffles.  Measured at 64^3: 204 us with 16 lanes per
// row, 171 us with 8 lanes one entry at a time, 149 us like this (4.6 TB/s); 32 lanes per row and
// nontemporal loads of the values were slower.
template <typename TV>
__global__ __launch_bounds__(256) void k_spmv(int64_t n, const int64_t *__restrict__ rowptr,
                                              const int32_t *__restrict__ col,
                                              const cx<TV> *__restrict__ val,
                                              const cx<double> *__restrict__ x,
                                              cx<double> *__restrict__ y) {
  const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 3;
  const int sub = threadIdx.x & 7;
  cx<double> s = {0, 0};
  if (row < n) {
    const int64_t q1 = rowptr[row + 1];
    int64_t q = rowptr[row] + sub;
    for (; q + 8 < q1; q += 16) {
      const cx<TV> a0 = val[q], a1 = val[q + 8];
      const int c0 = col[q], c1 = col[q + 8];
      const cx<double> x0 = x[c0], x1 = x[c1];
      cfma(s, ccast<double>(a0), x0);
      cfma(s, ccast<double>(a1), x1);
    }
    if (q < q1) cfma(s, ccast<double>(val[q]), x[col[q]]);
  }
#pragma unroll
  for (int o = 4; o >= 1; o >>= 1) s = cadd(s, shfl_xor_c(s, o));
  if (row < n && sub == 0) y[row] = s;
}

// ---- vector kernels ----------------------------------------------------------------------------------
__global__ void k_sub(int64_t n, const cx<double> *b, const cx<double> *y, cx<double> *r) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) r[i] = csub(b[i], y[i]);
}
__global__ void k_add(int64_t n, cx<double> *x, const cx<double> *z) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = cadd(x[i], z[i]);
}
// dst = src / *nrm  (zeros when *nrm == 0)
__global__ void k_scale(int64_t n, const cx<double> *src, const double *nrm, cx<double> *dst) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double d = *nrm;
  double s = d > 0 ? 1.0 / d : 0.0;
  dst[i] = {src[i].re * s, src[i].im * s};
}
// w -= sum_q V_q h_q
__global__ void k_update(int64_t n, const cx<double> *__restrict__ V, int64_t ldv, int nv,
                         const cx<double> *__restrict__ h, cx<double> *__restrict__ w) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  cx<double> acc = w[i];
  for (int q = 0; q < nv; ++q) {
    cx<double> v = V[q * ldv + i], hq = h[q];
    acc.re -= v.re * hq.re - v.im * hq.im;
    acc.im -= v.re * hq.im + v.im * hq.re;
  }
  w[i] = acc;
}
// out = sum_q V_q y_q
__global__ void k_combine(int64_t n, const cx<double> *__restrict__ V, int64_t ldv, int nv,
                          const cx<double> *__restrict__ y, cx<double> *__restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  cx<double> acc = {0, 0};
  for (int q = 0; q < nv; ++q) cfma(acc, V[q * ldv + i], y[q]);
  out[i] = acc;
}

// Block sum of 4 complex values over 256 threads; result valid in thread 0.
template <int C>
__device__ inline void block_sum(cx<double> v[C], cx<double> (*red)[C]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < C; ++c)
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v[c] = cadd(v[c], shfl_xor_c(v[c], o));
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int c = 0; c < C; ++c) red[w][c] = v[c];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int c = 0; c < C; ++c) v[c] = cadd(cadd(red[0][c], red[1][c]), cadd(red[2][c], red[3][c]));
}

// partial[q * G + b] = sum_{i in block b} conj(V_q[i]) w[i], q < nv (mode 0), or
// partial[b] = sum |w_i|^2 (mode 1, nv ignored).  Block b covers a fixed row range; eight basis
// vectors per pass over it, so w is read once per eight.
constexpr int kDotVecs = 8;
// blocks of the partial dot products: rows split into at most 1024 ranges of at least 1024
static inline int dot_blocks(int64_t n) {
  return (int)std::max<int64_t>(1, std::min<int64_t>(1024, (n + 1023) / 1024));
}
__global__ __launch_bounds__(256) void k_dot_partial(int64_t n, const cx<double> *__restrict__ V,
                                                     int64_t ldv, int nv,
                                                     const cx<double> *__restrict__ w,
                                                     cx<double> *__restrict__ partial, int mode) {
  __shared__ cx<double> red[4][kDotVecs];
  const int G = gridDim.x, b = blockIdx.x;
  const int64_t chunk = (n + G - 1) / G;
  const int64_t i0 = b * chunk, i1 = std::min(n, i0 + chunk);
  if (mode == 1) {
    cx<double> v[1] = {{0, 0}};
    for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) v[0].re += w[i].re * w[i].re + w[i].im * w[i].im;
    block_sum<1>(v, reinterpret_cast<cx<double>(*)[1]>(red));
    if (threadIdx.x == 0) partial[b] = v[0];
    return;
  }
  for (int q0 = 0; q0 < nv; q0 += kDotVecs) {
    cx<double> v[kDotVecs];
#pragma unroll
    for (int c = 0; c < kDotVecs; ++c) v[c] = {0, 0};
    for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) {
      const cx<double> wi = w[i];
#pragma unroll
      for (int c = 0; c < kDotVecs; ++c)
        if (q0 + c < nv) {
          const cx<double> a = V[(q0 + c) * ldv + i];
          v[c].re += a.re * wi.re + a.im * wi.im;
          v[c].im += a.re * wi.im - a.im * wi.re;
        }
    }
    block_sum<kDotVecs>(v, red);
    if (threadIdx.x == 0)
#pragma unroll
      for (int c = 0; c < kDotVecs; ++c)
        if (q0 + c < nv) partial[(q0 + c) * G + b] = v[c];
  }
}

// One block per q: fixed-order tree over the G partials.  mode 0: cur = sum = total;
// mode 1: cur = total, sum += total; mode 2: cur[q] = sqrt(total.re) (norm).
__global__ __launch_bounds__(256) void k_reduce(int G, const cx<double> *__restrict__ partial,
                                                cx<double> *cur, cx<double> *sum, double *nrm,
                                                int mode) {
  __shared__ cx<double> s[256];
  const int q = blockIdx.x;
  cx<double> acc = {0, 0};
  for (int b = threadIdx.x; b < G; b += 256) acc = cadd(acc, partial[(int64_t)q * G + b]);
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o >= 1; o >>= 1) {
    if (threadIdx.x < o) s[threadIdx.x] = cadd(s[threadIdx.x], s[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    cx<double> t = s[0];
    if (mode == 0) cur[q] = t, sum[q] = t;
    else if (mode == 1) cur[q] = t, sum[q] = cadd(sum[q], t);
    else *nrm = sqrt(t.re);
  }
}

struct GmresStatus {
  double est;     // |g_{j+1}|
  double hn;      // h_{j+1,j}
  double beta;    // last norm computed by k_reduce mode 2 (copied)
  int abort, pivot;
};

__device__ inline void givens(cx<double> a, cx<double> b, double &c, cx<double> &s, cx<double> &rho) {
  const double aa = hypot(a.re, a.im);
  if (aa == 0.0) {
    c = 0.0, s = {1.0, 0.0}, rho = b;
    return;
  }
  const double r = sqrt(aa * aa + b.re * b.re + b.im * b.im);
  const cx<double> ph = {a.re / aa, a.im / aa};
  c = aa / r;
  s = cmul(ph, cx<double>{b.re / r, -b.im / r});
  rho = {ph.re * r, ph.im * r};
}
// (x, y) -> (c x + s y, -conj(s) x + c y)
__device__ inline void rot(double c, cx<double> s, cx<double> &x, cx<double> &y) {
  const cx<double> nx = cadd(cx<double>{c * x.re, c * x.im}, cmul(s, y));
  const cx<double> ny = csub(cx<double>{c * y.re, c * y.im}, cmul(cx<double>{s.re, -s.im}, x));
  x = nx, y = ny;
}

// Column j of the Hessenberg matrix: h (j+1 entries) and hn = ||w||; previous rotations, new
// rotation, right-hand side g; status for the host.
__global__ void k_givens(int j, int ldh, const cx<double> *h, const double *hn_ptr, cx<double> *H,
                         double *cs, cx<double> *sn, cx<double> *g, GmresStatus *st,
                         const int *pctrl) {
  if (threadIdx.x != 0) return;
  cx<double> *col = H + (int64_t)j * ldh;
  for (int i = 0; i <= j; ++i) col[i] = h[i];
  const double hn = *hn_ptr;
  col[j + 1] = {hn, 0.0};
  for (int i = 0; i < j; ++i) rot(cs[i], sn[i], col[i], col[i + 1]);
  double c;
  cx<double> s, rho;
  givens(col[j], col[j + 1], c, s, rho);
  cs[j] = c, sn[j] = s;
  col[j] = rho;
  col[j + 1] = {0.0, 0.0};
  rot(c, s, g[j], g[j + 1]);
  st->est = hypot(g[j + 1].re, g[j + 1].im);
  st->hn = hn;
  st->abort = pctrl ? pctrl[2] : 0;
  st->pivot = pctrl ? pctrl[3] : 0;
}

__global__ void k_init_g(int m, const double *beta, cx<double> *g, GmresStatus *st) {
  for (int i = threadIdx.x; i <= m; i += blockDim.x) g[i] = {0.0, 0.0};
  __syncthreads();
  if (threadIdx.x == 0) {
    g[0] = {*beta, 0.0};
    st->beta = *beta;
  }
}

__global__ void k_copy_beta(const double *beta, GmresStatus *st) {
  if (threadIdx.x == 0) st->beta = *beta;
}

// Back substitution H(0:k,0:k) y = g(0:k).
__global__ void k_trisolve(int k, int ldh, const cx<double> *H, const cx<double> *g, cx<double> *y) {
  if (threadIdx.x != 0) return;
  for (int i = k - 1; i >= 0; --i) {
    cx<double> acc = g[i];
    for (int q = i + 1; q < k; ++q) acc = csub(acc, cmul(H[(int64_t)q * ldh + i], y[q]));
    y[i] = cdiv(acc, H[(int64_t)i * ldh + i]);
  }
}

// ---- host driver ---------------------------------------------------------------------------------
static inline unsigned nblk(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

void spmv_run(const mx_matrix *A, const void *x, void *y, bool c64, hipStream_t st) {
  const int64_t n = A->h.n;
  if (n == 0) return;
  if (c64)
    k_spmv<float><<<nblk(n * 8), 256, 0, st>>>(n, A->rowptr.as<int64_t>(), A->col.as<int32_t>(),
                                                 A->val32.as<cx<float>>(), (const cx<double> *)x,
                                                 (cx<double> *)y);
  else
    k_spmv<double><<<nblk(n * 8), 256, 0, st>>>(n, A->rowptr.as<int64_t>(), A->col.as<int32_t>(),
                                                  A->val.as<cx<double>>(), (const cx<double> *)x,
                                                  (cx<double> *)y);
  MX_HIP(hipGetLastError());
}

size_t matrix_device_bytes(const mx_matrix *A) {
  return 8 * (size_t)(A->h.n + 1) + (4 + 16 + 8) * (size_t)A->h.nnz() + 4096;
}

size_t gmres_device_bytes(int64_t n, int restart, bool flexible) {
  const size_t vb = ((size_t)n * 16 + 255) & ~(size_t)255;
  const int G = dot_blocks(n);
  return vb * (restart + 1 + (flexible ? restart : 0) + 4) + (size_t)G * (restart + 1) * 16 +
         (size_t)(restart + 1) * restart * 16 + 64 * (size_t)(restart + 1) + 8192;
}

__global__ void k_narrow(int64_t n, const double *__restrict__ in, float *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (float)in[i];
}

// Outside an allocation scope the copies run on a stream of their own that does not synchronise
// with other streams, so a host thread can upload the next matrix while the device works on
// something else; the buffers are then allocated unscoped, since they outlive that stream.
// Inside a scope (a setup on a caller's stream) allocations and copies use the scope's stream.
// Either way the call returns when the copy is complete.  The complex64 copy of the values is made
// on the device.
void matrix_upload(mx_matrix *A) {
  const bool scoped = t_alloc_scoped != 0;
  const hipStream_t prev = t_alloc_stream;
  hipStream_t own = nullptr;
  if (!scoped) {
    MX_HIP(hipStreamCreateWithFlags(&own, hipStreamNonBlocking));
    t_alloc_stream = own;
  }
  auto restore = [&]() {
    t_alloc_stream = prev;
    if (own) {
      (void)hipStreamSynchronize(own);
      (void)hipStreamDestroy(own);
      own = nullptr;
    }
  };
  try {
    const hipStream_t s = t_alloc_stream;
    A->rowptr.upload(A->h.rowptr);
    A->col.upload(A->h.col);
    A->val.upload(A->h.val);
    const int64_t nv = (int64_t)A->h.val.size();
    A->val32.alloc((size_t)nv * sizeof(float));
    if (nv > 0) k_narrow<<<(unsigned)((nv + 255) / 256), 256, 0, s>>>(nv, A->val.as<double>(), A->val32.as<float>());
    MX_HIP(hipGetLastError());
    MX_HIP(hipStreamSynchronize(s));
  } catch (...) {
    restore();
    throw;
  }
  restore();
}

// ---- two-level preconditioners (Sec. 3.2, 3.3, 6.3) -------------------------------------------------
// The coarse problem A^0 = R^0 A R^0^T is factored and solved by the same batched LDL^T and block
// sweeps as the local problems: it is the single subdomain of a one-level AS preconditioner on
// the coarse mesh whose matrix is A^0 (its minor over every coarse edge is A^0 itself), so
// G v = R^0^T (A^0)^-1 R^0 v is an SpMV, that application, and an SpMV.
struct CoarseLevel {
  CoarseSpec spec;
  int combine = MX_COARSE_ADDITIVE;
  mx_mesh mesh;                    // coarse box mesh
  mx_partition part;               // one subdomain, no overlap
  mx_matrix R0, R0T, A0;           // restriction (coarse x fine), its transpose, coarse matrix
  std::unique_ptr<mx_precond> P0;  // factored coarse problem
  std::unique_ptr<PrecondPlan> plan0;  // host half of P0 until the device half is built
  bool ready = false;              // device half built (R^0 uploaded, A^0 factored)
  const mx_matrix *A = nullptr;    // fine matrix the preconditioner is built for (borrowed)
  DevBuf c, y, g, t, s, u;         // coarse vectors c, y; fine vectors g = G v, t, s, u
};

void coarse_free(CoarseLevel *c) { delete c; }

// z = s - w + g
__global__ void k_hybrid_finish(int64_t n, const cx<double> *s, const cx<double> *w,
                                const cx<double> *g, cx<double> *z) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) z[i] = cadd(csub(s[i], w[i]), g[i]);
}

static void coarse_correction(CoarseLevel &C, const void *in, cx<double> *out, hipStream_t st) {
  spmv_run(&C.R0, in, C.c.p, false, st);                 // c = R^0 in
  precond_apply_level1(C.P0.get(), C.c.p, C.y.p, st);   // y = (A^0)^-1 c
  spmv_run(&C.R0T, C.y.p, out, false, st);               // out = R^0^T y
}

void precond_apply(mx_precond *P, const void *vin, void *zout, hipStream_t st) {
  if (!P->coarse) {
    precond_apply_level1(P, vin, zout, st);
    return;
  }
  CoarseLevel &C = *P->coarse;
  const int64_t n = P->E;
  cx<double> *z = (cx<double> *)zout, *g = C.g.as<cx<double>>();
  const cx<double> *v = (const cx<double> *)vin;
  coarse_correction(C, vin, g, st);  // g = G v
  if (C.combine == MX_COARSE_ADDITIVE) {  // B1 v + G v (eq:defAS, eq:RAS2)
    precond_apply_level1(P, vin, zout, st);
    k_add<<<nblk(n), 256, 0, st>>>(n, z, g);
  } else {
    cx<double> *t = C.t.as<cx<double>>(), *u = C.u.as<cx<double>>();
    spmv_run(C.A, g, u, false, st);
    k_sub<<<nblk(n), 256, 0, st>>>(n, v, u, t);  // t = (I - A G) v
    if (C.combine == MX_COARSE_DEFLATION) {     // B1 (I - A G) v + G v (eq:ADEF1ras)
      precond_apply_level1(P, t, zout, st);
      k_add<<<nblk(n), 256, 0, st>>>(n, z, g);
    } else {                                    // (I - G A) B1 (I - A G) v + G v (eq:HRAS)
      cx<double> *s = C.s.as<cx<double>>();
      precond_apply_level1(P, t, s, st);
      spmv_run(C.A, s, u, false, st);
      coarse_correction(C, u, t, st);           // t = G A s
      k_hybrid_finish<<<nblk(n), 256, 0, st>>>(n, s, t, g, z);
    }
  }
  MX_HIP(hipGetLastError());
}

// Host half: coarse mesh, R^0, A^0 = R^0 A R^0^T, and the plan of the coarse factorisation.
void coarse_plan(mx_precond *P, const mx_matrix *A, const mx_mesh *mh, const CoarseSpec &cs,
                 int combine) {
  const Mesh &m = mh->m;
  if (P->coarse) fail(MX_EINVAL, "preconditioner already has a coarse level");
  if (P->share) fail(MX_EINVAL, "a resident share cannot have a coarse level");
  if (combine < MX_COARSE_ADDITIVE || combine > MX_COARSE_DEFLATION) fail(MX_EINVAL, "unknown coarse combination");
  if (A->h.n != P->E || A->order != P->order || mh->ndof(P->order) != P->E)
    fail(MX_EINVAL, "matrix, mesh and preconditioner sizes differ");
  if (A->weight || A->k != P->k || A->xi != P->xi_prec || A->bc != P->bc)
    fail(MX_EINVAL, "the matrix is not the one the preconditioner was built for (k, xi_prec, bc)");
  auto C = std::make_unique<CoarseLevel>();
  C->spec = cs;
  C->combine = combine;
  C->A = A;
  coarse_restriction(m, cs, A->order, P->E, A->bc, C->mesh.m, C->R0.h, C->R0T.h);
  galerkin_coarse(A->h, C->R0.h, C->R0T.h, C->mesh.m, A->bc, C->A0.h);
  for (mx_matrix *X : {&C->R0, &C->R0T, &C->A0}) X->k = A->k, X->xi = A->xi, X->bc = A->bc;
  build_partition(C->mesh.m, 1, 1, 1, nullptr, nullptr, nullptr, 0, C->part.p);
  mx_precond_opts o{};
  o.kind = MX_AS;
  o.xi_prec = A->xi;
  o.precision = P->prec;
  C->P0 = std::make_unique<mx_precond>();
  C->plan0 = std::make_unique<PrecondPlan>();
  precond_plan(nullptr, &C->A0, &C->mesh, &C->part, &o, C->P0.get(), *C->plan0);
  P->coarse = C.release();
}

// Device half: uploads of R^0 and its transpose, factorisation of A^0, work vectors.
void coarse_materialize(mx_ctx *ctx, mx_precond *P, hipStream_t st) {
  if (!P->coarse) fail(MX_EINVAL, "preconditioner has no coarse level");
  CoarseLevel &C = *P->coarse;
  if (C.ready) fail(MX_EINVAL, "coarse level already built");
  if (!C.A->rowptr.p) fail(MX_EINVAL, "matrix has no device copy");
  AllocScope scope(st);
  for (mx_matrix *X : {&C.R0, &C.R0T, &C.A0}) X->device = ctx->device;
  matrix_upload(&C.R0);
  matrix_upload(&C.R0T);
  C.P0->device = ctx->device;
  set_sweep_grid(C.P0.get(), ctx->cus);
  precond_materialize(C.P0.get(), *C.plan0, st);
  C.plan0.reset();
  const int64_t nc = C.mesh.m.ne, E = P->E;
  C.c.alloc((size_t)nc * 16);
  C.y.alloc((size_t)nc * 16);
  C.g.alloc((size_t)E * 16);
  if (C.combine != MX_COARSE_ADDITIVE) {
    C.t.alloc((size_t)E * 16);
    C.u.alloc((size_t)E * 16);
    if (C.combine == MX_COARSE_HYBRID) C.s.alloc((size_t)E * 16);
  }
  MX_HIP(hipStreamSynchronize(st));
  C.ready = true;
}

void coarse_setup(mx_ctx *ctx, mx_precond *P, const mx_matrix *A, const mx_mesh *mh,
                  const CoarseSpec &cs, int combine, hipStream_t st) {
  if (P->coarse) {  // planned earlier: the arguments must be the same
    const CoarseLevel &C = *P->coarse;
    if (C.ready) fail(MX_EINVAL, "preconditioner already has a coarse level");
    if (C.A != A || !(C.spec == cs) || C.combine != combine || C.mesh.m.ne == 0 ||
        mh->ndof(P->order) != P->E)
      fail(MX_EINVAL, "arguments differ from those the coarse level was planned with");
  } else {
    coarse_plan(P, A, mh, cs, combine);
  }
  try {
    coarse_materialize(ctx, P, st);
  } catch (...) {
    if (!P->coarse->ready) {  // leave P one-level and usable
      coarse_free(P->coarse);
      P->coarse = nullptr;
    }
    throw;
  }
}

bool coarse_incomplete(const mx_precond *P) { return P->coarse && !P->coarse->ready; }

void coarse_export(const mx_precond *P, int64_t *n_coarse, int64_t *nnz_r, int64_t *nnz_a,
                   int64_t *r_rowptr, int32_t *r_col, double *r_val, int64_t *a_rowptr,
                   int32_t *a_col, double *a_val) {
  if (!P->coarse) fail(MX_EINVAL, "preconditioner has no coarse level");
  const CoarseLevel &C = *P->coarse;
  if (n_coarse) *n_coarse = C.R0.h.n;
  if (nnz_r) *nnz_r = C.R0.h.nnz();
  if (nnz_a) *nnz_a = C.A0.h.nnz();
  const HostCSR &R = C.R0.h, &A0 = C.A0.h;
  if (r_rowptr) std::copy(R.rowptr.begin(), R.rowptr.end(), r_rowptr);
  if (r_col) std::copy(R.col.begin(), R.col.end(), r_col);
  if (r_val)
    for (int64_t q = 0; q < R.nnz(); ++q) r_val[q] = R.val[2 * q];
  if (a_rowptr) std::copy(A0.rowptr.begin(), A0.rowptr.end(), a_rowptr);
  if (a_col) std::copy(A0.col.begin(), A0.col.end(), a_col);
  if (a_val) std::copy(A0.val.begin(), A0.val.end(), a_val);
}

// ---- fixed device scratch for GMRES without allocation -------------------------------------------
// One array per device, held by the code object until the process ends.  In host code `scratch`
// only stands for the symbol; its device address (one per GPU) comes from hipGetSymbolAddress,
// taken once per device when a context is created there, and only that address is handed to
// kernels and copies.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

void noalloc_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) fail(MX_EDEVICE, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return;
  int cur = 0;
  MX_HIP(hipGetDevice(&cur));
  if (cur != device) fail(MX_EDEVICE, "scratch set-up needs its device current");
  void *ptr = nullptr;
  MX_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  if (!ptr) fail(MX_EDEVICE, "no device address for the GMRES scratch array");
  g_scratch_ptr[device] = ptr;
}

static void *noalloc_scratch(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  void *p = (device >= 0 && device < kMaxDevices) ? g_scratch_ptr[device] : nullptr;
  if (!p) fail(MX_EDEVICE, "GMRES scratch not set up on this device (create a context first)");
  return p;
}

void gmres_run(mx_ctx *ctx, const mx_matrix *A, mx_precond *P, const void *b_dev, void *x_dev,
               const mx_gmres_opts *o, mx_gmres_stats *stats, double *hist, hipStream_t st,
               bool noalloc, const mx_matrix *D) {
  const auto t0 = std::chrono::steady_clock::now();
  const int64_t n = A->h.n;
  const int m = o->restart;
  if (m < 1 || o->max_iters < 0 || o->fixed_iters < 0 || !(o->rtol >= 0)) fail(MX_EINVAL, "bad GMRES options");
  const bool flex = o->flexible != 0, c64 = o->spmv_c64 != 0;
  const int G = dot_blocks(n);
  // workspace layout (bytes, 256-aligned)
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t vb = al((size_t)n * 16);
  size_t off = 0;
  const size_t oV = off; off += vb * (m + 1);
  const size_t oZ = off; off += flex ? vb * m : 0;
  const size_t oW = off; off += vb;
  const size_t oR = off; off += vb;
  const size_t oT = off; off += vb;
  const size_t oU = off; off += vb;
  const size_t oP = off; off += al((size_t)G * (m + 1) * 16);
  const size_t oH = off; off += al((size_t)(m + 1) * m * 16);
  const size_t oG = off; off += al((size_t)(m + 1) * 16);
  const size_t oC = off; off += al((size_t)m * 8);
  const size_t oS = off; off += al((size_t)m * 16);
  const size_t oh1 = off; off += al((size_t)(m + 1) * 16);
  const size_t oh2 = off; off += al((size_t)(m + 1) * 16);
  const size_t oY = off; off += al((size_t)(m + 1) * 16);
  const size_t oN = off; off += 256;
  const size_t oST = off; off += 256;
  char *ws = nullptr;
  if (noalloc) {
    if (off > kNoAllocScratchBytes)
      fail(MX_EINVAL, "GMRES without allocation needs " + std::to_string(off) +
                          " bytes of workspace; its fixed scratch holds " +
                          std::to_string(kNoAllocScratchBytes) +
                          " (fewer unknowns or a shorter restart, or use mx_gmres)");
    ws = (char *)noalloc_scratch(ctx->device);
  } else {
    ws = (char *)ctx->krylov.get(off);
  }
  cx<double> *V = (cx<double> *)(ws + oV), *Z = flex ? (cx<double> *)(ws + oZ) : nullptr;
  cx<double> *w = (cx<double> *)(ws + oW), *r = (cx<double> *)(ws + oR);
  cx<double> *tmp = (cx<double> *)(ws + oT), *u = (cx<double> *)(ws + oU);
  cx<double> *part = (cx<double> *)(ws + oP), *H = (cx<double> *)(ws + oH);
  cx<double> *g = (cx<double> *)(ws + oG), *sn = (cx<double> *)(ws + oS);
  double *cs = (double *)(ws + oC);
  cx<double> *h1 = (cx<double> *)(ws + oh1), *h2 = (cx<double> *)(ws + oh2), *y = (cx<double> *)(ws + oY);
  double *nrm = (double *)(ws + oN);
  GmresStatus *dst = (GmresStatus *)(ws + oST);
  GmresStatus *hst = (GmresStatus *)ctx->pinned;
  const int64_t ldv = (int64_t)(vb / 16);
  const int *pctrl = P ? P->d_ctrl.as<int>() : nullptr;
  // graph replay of the Arnoldi steps: not while the preconditioner's applications are routed
  // elsewhere or its sweeps are timed on the host side
  // (graph instantiation may allocate, so the no-allocation entry point never captures)
  const bool use_graph = o->graph != 0 && !noalloc && !(P && (P->apply_hook || P->timing));
  if (use_graph) {
    GraphCache &gc = ctx->graphs;
    const uint64_t pid = P ? P->id : 0, did = D ? D->id : 0;
    const void *pc = P ? (const void *)P->coarse : nullptr;  // a coarse level added later
    if (gc.a_id != A->id || gc.p_id != pid || gc.d_id != did || gc.ws != (const void *)ws ||
        gc.coarse != pc || gc.n != n || gc.m != m || gc.flex != flex || gc.c64 != c64 ||
        (int)gc.steps.size() != m) {
      gc.clear();
      gc.a_id = A->id, gc.p_id = pid, gc.d_id = did, gc.ws = ws, gc.coarse = pc, gc.n = n, gc.m = m;
      gc.flex = flex, gc.c64 = c64;
      gc.steps.assign(m, nullptr);
    }
  }
  const cx<double> *b = (const cx<double> *)b_dev;
  cx<double> *x = (cx<double> *)x_dev;

  // ||vec|| (Euclidean) or ||vec||_D = sqrt(vec^H (D vec)), with D vec formed in `scratch`
  auto norm_of = [&](const cx<double> *vec, cx<double> *scratch) {
    if (D) {
      spmv_run(D, vec, scratch, false, st);
      k_dot_partial<<<G, 256, 0, st>>>(n, vec, ldv, 1, scratch, part, 0);
    } else {
      k_dot_partial<<<G, 256, 0, st>>>(n, nullptr, 0, 0, vec, part, 1);
    }
    k_reduce<<<1, 256, 0, st>>>(G, part, nullptr, nullptr, nrm, 2);
  };
  // partial sums of h_q = <w, v_q> = v_q^H w, or v_q^H (D w) with D w formed in `scratch`
  auto dots = [&](int nv, const cx<double> *w, cx<double> *scratch) {
    const cx<double> *x = w;
    if (D) {
      spmv_run(D, w, scratch, false, st);
      x = scratch;
    }
    k_dot_partial<<<G, 256, 0, st>>>(n, V, ldv, nv, x, part, 0);
  };
  // Arnoldi steps are enqueued one ahead of the host: step j+1 is queued before the status of
  // step j is read, so the device never waits for the host between steps. The status of step j
  // lands in its own pinned slot (two alternate) and is read after that step's event.  A step
  // queued past the one that ends the cycle only touches column j+1 of H, g[j+1..j+2], V[j+2]
  // and the scratch vectors, none of which the cycle's update reads.
  struct Events {
    hipEvent_t e[2] = {nullptr, nullptr};
    ~Events() {
      for (auto x : e)
        if (x) (void)hipEventDestroy(x);
    }
  } ev;
  for (auto &x : ev.e) MX_HIP(hipEventCreateWithFlags(&x, hipEventDisableTiming));
  auto read_status = [&](int slot) -> const GmresStatus & {
    MX_HIP(hipEventSynchronize(ev.e[slot]));
    const GmresStatus &s = hst[slot];
    if (P && (s.pivot || s.abort)) {
      P->failed = s.pivot ? MX_EPIVOT : MX_ESTALL;
      precond_refuse_failed(P);
    }
    return s;
  };
  auto residual = [&]() {  // r = b - A x, beta -> status
    spmv_run(A, x, tmp, false, st);
    k_sub<<<nblk(n), 256, 0, st>>>(n, b, tmp, r);
    norm_of(r, tmp);
    k_copy_beta<<<1, 64, 0, st>>>(nrm, dst);
    hst->pivot = hst->abort = 0;
    MX_HIP(hipMemcpyAsync(hst, dst, sizeof(GmresStatus), hipMemcpyDeviceToHost, st));
    MX_HIP(hipStreamSynchronize(st));
    return hst->beta;
  };
  auto apply_prec = [&](const cx<double> *in, cx<double> *out) {
    if (P) precond_apply(P, in, out, st);
    else MX_HIP(hipMemcpyAsync(out, in, n * 16, hipMemcpyDeviceToDevice, st));
  };
  MX_HIP(hipMemsetAsync(dst, 0, sizeof(GmresStatus), st));
  const double beta0 = residual();
  int total = 0, cycles = 0;
  const int limit = o->fixed_iters > 0 ? o->fixed_iters : o->max_iters;
  if (hist) hist[0] = 1.0;
  double est = 1.0, beta = beta0;
  double last = beta0, rate = 1.0;  // last residual estimate and its last contraction factor
  bool converged = false;
  if (!std::isfinite(beta0)) fail(MX_ENAN, "non-finite initial residual");
  if (beta0 == 0.0) {
    converged = true;
  } else {
    while (true) {
      if (o->fixed_iters == 0 && beta <= o->rtol * beta0) {
        converged = true;
        break;
      }
      if (total >= limit) {
        converged = o->fixed_iters > 0;
        break;
      }
      ++cycles;
      k_scale<<<nblk(n), 256, 0, st>>>(n, r, nrm, V);
      k_init_g<<<1, 64, 0, st>>>(m, nrm, g, dst);
      int jend = 0;
      auto step_body = [&](int j) {
        cx<double> *z = flex ? Z + (int64_t)j * ldv : tmp;
        apply_prec(V + (int64_t)j * ldv, z);
        spmv_run(A, z, w, c64, st);
        const int nv = j + 1;
        dots(nv, w, u);
        k_reduce<<<nv, 256, 0, st>>>(G, part, h2, h1, nullptr, 0);
        k_update<<<nblk(n), 256, 0, st>>>(n, V, ldv, nv, h2, w);
        dots(nv, w, u);
        k_reduce<<<nv, 256, 0, st>>>(G, part, h2, h1, nullptr, 1);
        k_update<<<nblk(n), 256, 0, st>>>(n, V, ldv, nv, h2, w);
        norm_of(w, u);
        k_givens<<<1, 64, 0, st>>>(j, m + 1, h1, nrm, H, cs, sn, g, dst, pctrl);
        k_scale<<<nblk(n), 256, 0, st>>>(n, w, nrm, V + (int64_t)(j + 1) * ldv);
        MX_HIP(hipGetLastError());
        MX_HIP(hipMemcpyAsync(hst + (j & 1), dst, sizeof(GmresStatus), hipMemcpyDeviceToHost, st));
      };
      // With graphs, step j is captured the first time it runs for this key and replayed after.
      auto arnoldi_step = [&](int j) {
        if (use_graph) {
          hipGraphExec_t &ex = ctx->graphs.steps[j];
          if (!ex) {  // captured on the context's own stream, launched on st
            if (!ctx->capture) MX_HIP(hipStreamCreateWithFlags(&ctx->capture, hipStreamNonBlocking));
            const hipStream_t run_st = st;
            st = ctx->capture;
            hipGraph_t gr = nullptr;
            MX_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
            try {
              step_body(j);
            } catch (...) {
              (void)hipStreamEndCapture(st, &gr);
              if (gr) (void)hipGraphDestroy(gr);
              (void)hipGetLastError();
              st = run_st;
              throw;
            }
            const hipError_t ec = hipStreamEndCapture(st, &gr);
            st = run_st;
            if (ec != hipSuccess) {
              if (gr) (void)hipGraphDestroy(gr);
              (void)hipGetLastError();
              fail(MX_EDEVICE, std::string("graph capture: ") + hipGetErrorString(ec));
            }
            const hipError_t e = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
            (void)hipGraphDestroy(gr);
            if (e != hipSuccess) {
              ex = nullptr;
              (void)hipGetLastError();
              fail(MX_EDEVICE, std::string("graph instantiation: ") + hipGetErrorString(e));
            }
          }
          MX_HIP(hipGraphLaunch(ex, st));
        } else {
          step_body(j);
        }
        MX_HIP(hipEventRecord(ev.e[j & 1], st));
      };
      const int total0 = total;
      arnoldi_step(0);
      for (int j = 0; j < m; ++j) {
        // Step j+1 is queued before step j's status only if it is inside the cycle and the
        // iteration limit and, with a tolerance, if the residual estimate two steps on, at the
        // last contraction rate, is still above it (so the step is almost surely needed; a
        // wasted step costs a whole preconditioner application on large problems).
        const bool inside = j + 1 < m && total0 + j + 2 <= limit;
        const double pred = last * rate * rate;
        const bool queued = inside && (o->fixed_iters > 0 || pred > o->rtol * beta0);
        if (queued) arnoldi_step(j + 1);
        const GmresStatus &s = read_status(j & 1);
        ++total;
        jend = j + 1;
        est = s.est / beta0;
        if (hist) hist[total] = est;
        if (!std::isfinite(s.est) || !std::isfinite(s.hn)) fail(MX_ENAN, "non-finite Arnoldi value");
        if (s.est > 0.0 && last > 0.0) rate = std::min(1.0, s.est / last);
        last = s.est;
        if (o->fixed_iters == 0 && s.est <= o->rtol * beta0) break;
        if (!inside || s.hn == 0.0) break;
        if (!queued) arnoldi_step(j + 1);
      }
      k_trisolve<<<1, 64, 0, st>>>(jend, m + 1, H, g, y);
      if (flex) {
        k_combine<<<nblk(n), 256, 0, st>>>(n, Z, ldv, jend, y, u);
        k_add<<<nblk(n), 256, 0, st>>>(n, x, u);
      } else {
        k_combine<<<nblk(n), 256, 0, st>>>(n, V, ldv, jend, y, u);
        apply_prec(u, tmp);
        k_add<<<nblk(n), 256, 0, st>>>(n, x, tmp);
      }
      beta = residual();
      last = beta;
      if (!std::isfinite(beta)) fail(MX_ENAN, "non-finite residual");
      if (P) precond_check(P, st);
    }
  }
  stats->iters = total;
  stats->cycles = cycles;
  stats->converged = converged ? 1 : 0;
  stats->relres_true = beta0 > 0 ? beta / beta0 : 0.0;
  stats->relres_est = est;
  stats->t_solve = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

// ---- self-test of the matrix-core tile product ----------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_selftest_mfma(const cx<T> *A, const cx<T> *B, const cx<T> *s,
                                                       cx<T> *out) {
  const int w = threadIdx.x >> 6;
  const int r0 = (w >> 1) * 32, c0 = (w & 1) * 32;
  typename Mfma<T>::acc_t acc[2][2][2];
  tile_nt_quadrant<T, true, false>(A, B, s, r0, c0, acc);
  for (int rb = 0; rb < 2; ++rb)
    for (int cb = 0; cb < 2; ++cb)
      for (int q = 0; q < 4; ++q)
        out[acc_row<T>(r0, rb, q) * kTile + acc_col(c0, cb)] = {acc[rb][cb][0][q], acc[rb][cb][1][q]};
}
template <typename T>
__global__ void k_selftest_ref(const cx<T> *A, const cx<T> *B, const cx<T> *s, cx<T> *out) {
  const int i = blockIdx.x, j = threadIdx.x;
  cx<double> acc = {0, 0};
  for (int k = 0; k < kTile; ++k)
    cfma(acc, ccast<double>(A[i * kTile + k]), cmul(ccast<double>(s[k]), ccast<double>(B[j * kTile + k])));
  out[i * kTile + j] = ccast<T>(acc);
}

template <typename T>
static double selftest_t() {
  std::mt19937_64 rng(12345);
  std::normal_distribution<double> nd;
  std::vector<T> h(2 * (2 * kTileElems + kTile));
  for (auto &x : h) x = (T)nd(rng);
  DevBuf d_in, d_a, d_b;
  d_in.upload(h);
  d_a.alloc(kTileElems * 2 * sizeof(T));
  d_b.alloc(kTileElems * 2 * sizeof(T));
  const cx<T> *A = d_in.as<cx<T>>(), *B = A + kTileElems, *s = B + kTileElems;
  k_selftest_mfma<T><<<1, 256>>>(A, B, s, d_a.as<cx<T>>());
  k_selftest_ref<T><<<kTile, kTile>>>(A, B, s, d_b.as<cx<T>>());
  MX_HIP(hipGetLastError());
  MX_HIP(hipDeviceSynchronize());
  std::vector<T> ra(2 * kTileElems), rb(2 * kTileElems);
  MX_HIP(hipMemcpy(ra.data(), d_a.p, ra.size() * sizeof(T), hipMemcpyDeviceToHost));
  MX_HIP(hipMemcpy(rb.data(), d_b.p, rb.size() * sizeof(T), hipMemcpyDeviceToHost));
  double err = 0, mag = 0;
  for (size_t i = 0; i < ra.size(); ++i) {
    err = std::max(err, (double)std::fabs((double)ra[i] - (double)rb[i]));
    mag = std::max(mag, (double)std::fabs((double)rb[i]));
  }
  return err / mag;
}

void selftest_run(double *e64, double *e32) {
  *e64 = selftest_t<double>();
  *e32 = selftest_t<float>();
}

}  // namespace mx
