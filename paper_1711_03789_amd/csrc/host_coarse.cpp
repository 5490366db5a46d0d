// Coarse space of the two-level Schwarz preconditioners (Sec. 3.2, Sec. 3.3): the restriction
// R^0 of eq:restriction from a coarse box mesh, nested or not, and the coarse Galerkin matrix
// A^0 = R^0 A (R^0)^T (eq:minor with l = 0).
//
// A coarse mesh that is not nested (Sec. 6.1: the coarse tetrahedra are not unions of fine
// ones) gives integrands that are only piecewise affine along a fine edge; there the line
// integral is taken with an nq-point Gauss-Legendre rule along the edge, as in the paper's runs,
// which use a fixed number of quadrature points per edge.  The coarse tetrahedron holding a
// quadrature point is read off the Kuhn split as below; a point on a face shared by two coarse
// tetrahedra lies there only when the whole fine edge lies in that face, and then both give the
// same tangential values.
//
// The coarse mesh has the same box and split with r times fewer cubes on every axis; each coarse
// tetrahedron is then a union of fine ones.  A fine edge therefore lies in one closed coarse
// tetrahedron, where every coarse Whitney function is affine, so its degree of freedom (the line
// integral of the tangential component along the edge, unnormalised tangent x_hi - x_lo) is the
// value at the edge midpoint dotted with the tangent.  The coarse tetrahedron holding the
// midpoint is read off the Kuhn split: in coarse-cube coordinates u in [0,1]^3, the tetrahedron
// of axis permutation s holds the points with u_s0 >= u_s1 >= u_s2, where the barycentric
// coordinates are 1 - u_s0, u_s0 - u_s1, u_s1 - u_s2, u_s2.  (On a face shared by two coarse
// tetrahedra the fine edge lies in that face, and both give the same tangential values.)
#include <cmath>

#include "objects.hpp"

namespace mx {

namespace {
const int kLocalEdge[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};

int perm_rank(const int s[3]) {  // rank of the permutation in lexicographic order
  static const int P[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
  for (int p = 0; p < 6; ++p)
    if (P[p][0] == s[0] && P[p][1] == s[1] && P[p][2] == s[2]) return p;
  return -1;
}

struct REnt {
  int32_t col;
  double v;
};
}  // namespace

// R0^T (row j = fine edge j, columns = coarse edges ascending) and R0 from the per-edge lists
// ent[off[j] .. off[j] + cnt[j+1]).
static void restriction_csr(int64_t E, int64_t Ec, const std::vector<int64_t> &cnt,
                            const std::vector<int64_t> &off, const std::vector<REnt> &ent,
                            HostCSR &R0, HostCSR &R0T) {
  R0T.n = E;
  R0T.rowptr.assign(E + 1, 0);
  for (int64_t j = 0; j < E; ++j) R0T.rowptr[j + 1] = R0T.rowptr[j] + cnt[j + 1];
  const int64_t nnz = R0T.rowptr[E];
  R0T.col.resize(nnz);
  R0T.val.resize(2 * nnz);
  for (int64_t j = 0; j < E; ++j)
    for (int64_t q = R0T.rowptr[j], i = 0; q < R0T.rowptr[j + 1]; ++q, ++i) {
      R0T.col[q] = ent[(size_t)off[j] + i].col;
      R0T.val[2 * q] = ent[(size_t)off[j] + i].v;
      R0T.val[2 * q + 1] = 0.0;
    }
  R0.n = Ec;
  R0.rowptr.assign(Ec + 1, 0);
  for (int64_t q = 0; q < nnz; ++q) ++R0.rowptr[R0T.col[q] + 1];
  for (int64_t p = 0; p < Ec; ++p) R0.rowptr[p + 1] += R0.rowptr[p];
  R0.col.resize(nnz);
  R0.val.resize(2 * nnz);
  std::vector<int64_t> fill(R0.rowptr.begin(), R0.rowptr.end() - 1);
  for (int64_t j = 0; j < E; ++j)
    for (int64_t q = R0T.rowptr[j]; q < R0T.rowptr[j + 1]; ++q) {
      const int64_t d = fill[R0T.col[q]]++;
      R0.col[d] = (int32_t)j;
      R0.val[2 * d] = R0T.val[2 * q];
      R0.val[2 * d + 1] = 0.0;
    }
}

// Coarse tetrahedron of the Kuhn split holding the point with coarse-cube index c and local
// coordinates u in [0,1]^3: its vertices v and the barycentric coordinates lam and their
// gradients (coarse spacing H).
static void coarse_tet_at(const Mesh &coarse, const int c[3], const double u[3], const double H[3],
                          int32_t v[4], double lam[4], double grad[4][3]) {
  int s[3] = {0, 1, 2};  // axes by decreasing u (ties: lower axis first)
  for (int a = 0; a < 3; ++a)
    for (int b = a + 1; b < 3; ++b)
      if (u[s[b]] > u[s[a]]) std::swap(s[a], s[b]);
  if (s[0] > s[1] && u[s[0]] == u[s[1]]) std::swap(s[0], s[1]);
  if (s[1] > s[2] && u[s[1]] == u[s[2]]) std::swap(s[1], s[2]);
  if (s[0] > s[1] && u[s[0]] == u[s[1]]) std::swap(s[0], s[1]);
  if (perm_rank(s) < 0) fail(MX_EINVAL, "internal: bad permutation");
  lam[0] = 1.0 - u[s[0]], lam[1] = u[s[0]] - u[s[1]], lam[2] = u[s[1]] - u[s[2]], lam[3] = u[s[2]];
  for (int a = 0; a < 4; ++a)
    for (int d = 0; d < 3; ++d) grad[a][d] = 0.0;
  grad[0][s[0]] = -1.0 / H[s[0]];
  grad[1][s[0]] = 1.0 / H[s[0]];
  grad[1][s[1]] = -1.0 / H[s[1]];
  grad[2][s[1]] = 1.0 / H[s[1]];
  grad[2][s[2]] = -1.0 / H[s[2]];
  grad[3][s[2]] = 1.0 / H[s[2]];
  int p[3] = {c[0], c[1], c[2]};
  v[0] = coarse.vid(p[0], p[1], p[2]);
  for (int k = 0; k < 3; ++k) {
    ++p[s[k]];
    v[k + 1] = coarse.vid(p[0], p[1], p[2]);
  }
}

// Nodes (on [0,1]) and weights (sum 1) of the n-point Gauss-Legendre rule: Newton's method on
// the Legendre polynomial P_n from the usual cosine first guesses, weights 2/((1-x^2) P_n'(x)^2)
// on [-1,1].
static void gauss_legendre01(int n, std::vector<double> &s, std::vector<double> &w) {
  s.assign(n, 0.0);
  w.assign(n, 0.0);
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < n; ++i) {
    double x = std::cos(pi * (i + 0.75) / (n + 0.5)), dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;  // P_0, P_1, then the three-term recurrence up to P_n
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1, p1 = p2;
      }
      if (n == 1) p1 = x, p0 = 1.0;
      dp = n * (x * p1 - p0) / (x * x - 1.0);
      const double dx = p1 / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    double p0 = 1.0, p1 = x;
    for (int k = 2; k <= n; ++k) {
      const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
      p0 = p1, p1 = p2;
    }
    if (n == 1) p1 = x, p0 = 1.0;
    dp = n * (x * p1 - p0) / (x * x - 1.0);
    s[n - 1 - i] = 0.5 * (x + 1.0);
    w[n - 1 - i] = 1.0 / ((1.0 - x * x) * dp * dp);  // 2/((1-x^2)P'^2) on [-1,1], halved on [0,1]
  }
}

void build_restriction_quad(const Mesh &fine, const Mesh &coarse, int bc, int nq, HostCSR &R0,
                            HostCSR &R0T) {
  if (nq < 1 || nq > 64) fail(MX_EINVAL, "quadrature points per fine edge must be 1 .. 64");
  if (fine.lx != coarse.lx || fine.ly != coarse.ly || fine.lz != coarse.lz)
    fail(MX_EINVAL, "coarse mesh is not a mesh of the fine mesh's box");
  const int64_t E = fine.ne, Ec = coarse.ne;
  const int nc[3] = {coarse.nx, coarse.ny, coarse.nz};
  const double H[3] = {coarse.lx / coarse.nx, coarse.ly / coarse.ny, coarse.lz / coarse.nz};
  std::vector<double> gs, gw;
  gauss_legendre01(nq, gs, gw);
  // fine edges in chunks; each chunk packs its edges' merged (coarse edge, value) lists
  const int64_t cs = 4096, nchunk = (E + cs - 1) / cs;
  std::vector<std::vector<REnt>> packed(nchunk);
  std::vector<int64_t> cnt(E + 1, 0);
  parallel_items(nchunk, [&](auto next) {
    std::vector<REnt> acc;
    for (int64_t ch; (ch = next()) >= 0;) {
      auto &out = packed[ch];
      for (int64_t j = ch * cs; j < std::min(E, (ch + 1) * cs); ++j) {
        const int32_t lo = fine.edge_vert[2 * j], hi = fine.edge_vert[2 * j + 1];
        double xl[3], xh[3], t[3];
        fine.xyz(lo, xl);
        fine.xyz(hi, xh);
        for (int d = 0; d < 3; ++d) t[d] = xh[d] - xl[d];
        acc.clear();
        for (int q = 0; q < nq; ++q) {
          int c[3];
          double u[3];
          for (int d = 0; d < 3; ++d) {
            const double y = (xl[d] + gs[q] * t[d]) / H[d];
            c[d] = std::min(std::max((int)std::floor(y), 0), nc[d] - 1);
            u[d] = std::min(std::max(y - c[d], 0.0), 1.0);
          }
          int32_t v[4];
          double lam[4], grad[4][3];
          coarse_tet_at(coarse, c, u, H, v, lam, grad);
          for (int le = 0; le < 6; ++le) {
            const int a = kLocalEdge[le][0], b = kLocalEdge[le][1];
            const int32_t ce = coarse.edge_id(std::min(v[a], v[b]), std::max(v[a], v[b]));
            if (ce < 0) fail(MX_EINVAL, "internal: coarse edge not found");
            if (bc == MX_BC_PEC && coarse.edge_on_boundary[ce]) continue;  // zero tangential trace
            double wt = 0;
            for (int d = 0; d < 3; ++d) wt += (lam[a] * grad[b][d] - lam[b] * grad[a][d]) * t[d];
            if (v[a] > v[b]) wt = -wt;  // global orientation lo -> hi
            acc.push_back({ce, gw[q] * wt});
          }
        }
        // merge by coarse edge, summing in quadrature-point order
        std::stable_sort(acc.begin(), acc.end(), [](const REnt &x, const REnt &y) { return x.col < y.col; });
        int64_t n = 0;
        for (size_t i = 0; i < acc.size();) {
          size_t k = i;
          double sum = 0;
          for (; k < acc.size() && acc[k].col == acc[i].col; ++k) sum += acc[k].v;
          if (sum != 0.0) out.push_back({acc[i].col, sum}), ++n;
          i = k;
        }
        cnt[j + 1] = n;
      }
    }
  });
  std::vector<int64_t> off(E + 1, 0);
  for (int64_t j = 0; j < E; ++j) off[j + 1] = off[j] + cnt[j + 1];
  std::vector<REnt> ent((size_t)off[E]);
  for (int64_t ch = 0; ch < nchunk; ++ch)
    std::copy(packed[ch].begin(), packed[ch].end(), ent.begin() + off[ch * cs]);
  restriction_csr(E, Ec, cnt, off, ent, R0, R0T);
}

void coarse_restriction(const Mesh &fine, const CoarseSpec &cs, int order, int64_t ndof, int bc,
                        Mesh &coarse, HostCSR &R0, HostCSR &R0T) {
  const int n[3] = {fine.nx, fine.ny, fine.nz};
  for (int d = 0; d < 3; ++d)
    if (cs.cn[d] < 1) fail(MX_EINVAL, "coarse cube counts must be >= 1");
  if (cs.nq == 0) {  // nested: one ratio for every axis
    const int r = n[0] / cs.cn[0];
    for (int d = 0; d < 3; ++d)
      if (n[d] % cs.cn[d] || n[d] / cs.cn[d] != r)
        fail(MX_EINVAL, "the coarse ratio must divide the cube count of every axis");
  } else if (order != 1) {
    fail(MX_EINVAL, "order-2 coarse levels need the nested coarse mesh of a common ratio");
  }
  build_mesh(coarse, cs.cn[0], cs.cn[1], cs.cn[2], fine.lx, fine.ly, fine.lz);
  if (cs.nq == 0) build_restriction(fine, coarse, n[0] / cs.cn[0], bc, R0, R0T);
  else build_restriction_quad(fine, coarse, bc, cs.nq, R0, R0T);
  if (ndof > R0T.n) {
    // order 2: the coarse Whitney functions are piecewise lowest-order fields on the fine mesh,
    // so in the hierarchical order-2 basis they have Whitney coefficients only: R^0 keeps its
    // columns and its transpose gains empty rows for the gradient and face functions
    R0T.rowptr.resize(ndof + 1, R0T.rowptr.back());
    R0T.n = ndof;
  }
}

void build_restriction(const Mesh &fine, const Mesh &coarse, int ratio, int bc, HostCSR &R0,
                       HostCSR &R0T) {
  if (ratio < 1 || fine.nx != coarse.nx * ratio || fine.ny != coarse.ny * ratio ||
      fine.nz != coarse.nz * ratio || fine.lx != coarse.lx || fine.ly != coarse.ly ||
      fine.lz != coarse.lz)
    fail(MX_EINVAL, "coarse mesh is not the fine box with ratio times fewer cubes per axis");
  const int64_t E = fine.ne, Ec = coarse.ne;
  const int nc[3] = {coarse.nx, coarse.ny, coarse.nz};
  const double H[3] = {coarse.lx / coarse.nx, coarse.ly / coarse.ny, coarse.lz / coarse.nz};
  // per fine edge: up to six (coarse edge, value) pairs, sorted by coarse edge
  std::vector<int64_t> cnt(E + 1, 0);
  std::vector<REnt> tmp((size_t)E * 6);
  parallel_for(E, [&](int64_t e0, int64_t e1) {
    for (int64_t j = e0; j < e1; ++j) {
      const int32_t lo = fine.edge_vert[2 * j], hi = fine.edge_vert[2 * j + 1];
      int Il[3], Ih[3];
      fine.vijk(lo, Il[0], Il[1], Il[2]);
      fine.vijk(hi, Ih[0], Ih[1], Ih[2]);
      double xl[3], xh[3], t[3], u[3];
      fine.xyz(lo, xl);
      fine.xyz(hi, xh);
      int c[3];
      for (int d = 0; d < 3; ++d) {
        t[d] = xh[d] - xl[d];
        const int twice = Il[d] + Ih[d];  // twice the midpoint in fine-grid units
        c[d] = std::min(twice / (2 * ratio), nc[d] - 1);
        u[d] = (double)(twice - 2 * ratio * c[d]) / (double)(2 * ratio);
      }
      int32_t v[4];
      double lam[4], grad[4][3];
      coarse_tet_at(coarse, c, u, H, v, lam, grad);
      REnt *out = &tmp[(size_t)j * 6];
      int n = 0;
      for (int le = 0; le < 6; ++le) {
        const int a = kLocalEdge[le][0], b = kLocalEdge[le][1];
        const int32_t va = v[a], vb = v[b];
        const int32_t ce = coarse.edge_id(std::min(va, vb), std::max(va, vb));
        if (ce < 0) fail(MX_EINVAL, "internal: coarse edge not found");
        if (bc == MX_BC_PEC && coarse.edge_on_boundary[ce]) continue;  // zero tangential trace
        double w = 0;
        for (int d = 0; d < 3; ++d) w += (lam[a] * grad[b][d] - lam[b] * grad[a][d]) * t[d];
        if (va > vb) w = -w;  // global orientation lo -> hi
        if (w == 0.0) continue;
        out[n++] = {ce, w};
      }
      std::sort(out, out + n, [](const REnt &x, const REnt &y) { return x.col < y.col; });
      cnt[j + 1] = n;
    }
  });
  std::vector<int64_t> off(E + 1);
  for (int64_t j = 0; j <= E; ++j) off[j] = 6 * j;
  restriction_csr(E, Ec, cnt, off, tmp, R0, R0T);
}

// Sparse product of complex CSR matrices, row-parallel: C = X Y (rows of X, columns of Y).
static void spgemm(const HostCSR &X, const HostCSR &Y, int64_t ncol, HostCSR &C) {
  const int64_t n = X.n;
  std::vector<std::vector<int32_t>> rcol(n);
  std::vector<std::vector<double>> rval(n);
  parallel_items(std::max<int64_t>(1, (n + 1023) / 1024), [&](auto next) {
    std::vector<int32_t> pos(ncol, -1), touched;
    std::vector<double> acc;
    for (int64_t blk; (blk = next()) >= 0;) {
      for (int64_t i = blk * 1024; i < std::min(n, (blk + 1) * 1024); ++i) {
        touched.clear();
        acc.clear();
        for (int64_t q = X.rowptr[i]; q < X.rowptr[i + 1]; ++q) {
          const double xr = X.val[2 * q], xi = X.val[2 * q + 1];
          const int32_t k = X.col[q];
          for (int64_t r = Y.rowptr[k]; r < Y.rowptr[k + 1]; ++r) {
            const int32_t c = Y.col[r];
            const double yr = Y.val[2 * r], yi = Y.val[2 * r + 1];
            int32_t s = pos[c];
            if (s < 0) {
              s = pos[c] = (int32_t)touched.size();
              touched.push_back(c);
              acc.push_back(0.0);
              acc.push_back(0.0);
            }
            acc[2 * s] += xr * yr - xi * yi;
            acc[2 * s + 1] += xr * yi + xi * yr;
          }
        }
        std::vector<int32_t> order(touched.size());
        for (size_t a = 0; a < order.size(); ++a) order[a] = (int32_t)a;
        std::sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return touched[a] < touched[b]; });
        rcol[i].resize(order.size());
        rval[i].resize(2 * order.size());
        for (size_t a = 0; a < order.size(); ++a) {
          rcol[i][a] = touched[order[a]];
          rval[i][2 * a] = acc[2 * order[a]];
          rval[i][2 * a + 1] = acc[2 * order[a] + 1];
        }
        for (int32_t c : touched) pos[c] = -1;
      }
    }
  });
  C.n = n;
  C.rowptr.assign(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) C.rowptr[i + 1] = C.rowptr[i] + (int64_t)rcol[i].size();
  C.col.resize(C.rowptr[n]);
  C.val.resize(2 * C.rowptr[n]);
  parallel_for(n, [&](int64_t a, int64_t b) {
    for (int64_t i = a; i < b; ++i) {
      std::copy(rcol[i].begin(), rcol[i].end(), C.col.begin() + C.rowptr[i]);
      std::copy(rval[i].begin(), rval[i].end(), C.val.begin() + 2 * C.rowptr[i]);
    }
  }, 1024);
}

void galerkin_coarse(const HostCSR &A, const HostCSR &R0, const HostCSR &R0T, const Mesh &coarse,
                     int bc, HostCSR &A0) {
  if (A.n != R0T.n) fail(MX_EINVAL, "matrix and restriction sizes differ");
  HostCSR C;
  spgemm(A, R0T, R0.n, C);   // A R0^T   (E x Ec)
  spgemm(R0, C, R0.n, A0);   // R0 A R0^T (Ec x Ec)
  if (bc == MX_BC_PEC) {
    // coarse boundary edges carry no basis function: their rows and columns are empty, and get a
    // unit diagonal so the coarse solve leaves them at zero
    for (int64_t p = 0; p < A0.n; ++p) {
      if (!coarse.edge_on_boundary[p]) continue;
      if (A0.rowptr[p + 1] != A0.rowptr[p]) fail(MX_EINVAL, "internal: constrained coarse row not empty");
    }
    HostCSR B;
    B.n = A0.n;
    B.rowptr.assign(A0.n + 1, 0);
    for (int64_t p = 0; p < A0.n; ++p)
      B.rowptr[p + 1] = B.rowptr[p] + (coarse.edge_on_boundary[p] ? 1 : A0.rowptr[p + 1] - A0.rowptr[p]);
    B.col.resize(B.rowptr[A0.n]);
    B.val.resize(2 * B.rowptr[A0.n]);
    for (int64_t p = 0; p < A0.n; ++p) {
      if (coarse.edge_on_boundary[p]) {
        B.col[B.rowptr[p]] = (int32_t)p;
        B.val[2 * B.rowptr[p]] = 1.0;
        B.val[2 * B.rowptr[p] + 1] = 0.0;
        continue;
      }
      std::copy(A0.col.begin() + A0.rowptr[p], A0.col.begin() + A0.rowptr[p + 1], B.col.begin() + B.rowptr[p]);
      std::copy(A0.val.begin() + 2 * A0.rowptr[p], A0.val.begin() + 2 * A0.rowptr[p + 1],
                B.val.begin() + 2 * B.rowptr[p]);
    }
    A0 = std::move(B);
  }
}

}  // namespace mx
