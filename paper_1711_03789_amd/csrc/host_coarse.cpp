// Coarse space of the two-level Schwarz preconditioners (Sec. 3.2, Sec. 3.3): the restriction
// R^0 of eq:restriction from a nested coarse box mesh, and the coarse Galerkin matrix
// A^0 = R^0 A (R^0)^T (eq:minor with l = 0).
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

#include "mx_internal.hpp"

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
      int s[3] = {0, 1, 2};  // axes by decreasing u (ties: lower axis first)
      for (int a = 0; a < 3; ++a)
        for (int b = a + 1; b < 3; ++b)
          if (u[s[b]] > u[s[a]]) std::swap(s[a], s[b]);
      if (s[0] > s[1] && u[s[0]] == u[s[1]]) std::swap(s[0], s[1]);
      if (s[1] > s[2] && u[s[1]] == u[s[2]]) std::swap(s[1], s[2]);
      if (s[0] > s[1] && u[s[0]] == u[s[1]]) std::swap(s[0], s[1]);
      if (perm_rank(s) < 0) fail(MX_EINVAL, "internal: bad permutation");
      const double lam[4] = {1.0 - u[s[0]], u[s[0]] - u[s[1]], u[s[1]] - u[s[2]], u[s[2]]};
      double grad[4][3] = {};
      grad[0][s[0]] = -1.0 / H[s[0]];
      grad[1][s[0]] = 1.0 / H[s[0]];
      grad[1][s[1]] = -1.0 / H[s[1]];
      grad[2][s[1]] = 1.0 / H[s[1]];
      grad[2][s[2]] = -1.0 / H[s[2]];
      grad[3][s[2]] = 1.0 / H[s[2]];
      int32_t v[4];
      int p[3] = {c[0], c[1], c[2]};
      v[0] = coarse.vid(p[0], p[1], p[2]);
      for (int k = 0; k < 3; ++k) {
        ++p[s[k]];
        v[k + 1] = coarse.vid(p[0], p[1], p[2]);
      }
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
  // R0^T: row j = fine edge j
  R0T.n = E;
  R0T.rowptr.assign(E + 1, 0);
  for (int64_t j = 0; j < E; ++j) R0T.rowptr[j + 1] = R0T.rowptr[j] + cnt[j + 1];
  const int64_t nnz = R0T.rowptr[E];
  R0T.col.resize(nnz);
  R0T.val.resize(2 * nnz);
  for (int64_t j = 0; j < E; ++j)
    for (int64_t q = R0T.rowptr[j], i = 0; q < R0T.rowptr[j + 1]; ++q, ++i) {
      R0T.col[q] = tmp[(size_t)j * 6 + i].col;
      R0T.val[2 * q] = tmp[(size_t)j * 6 + i].v;
      R0T.val[2 * q + 1] = 0.0;
    }
  // R0 = transpose (rows = coarse edges, columns = fine edges ascending)
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
