// Structured Kuhn box mesh, closed-form edge numbering, Whitney element matrices, global
// Galerkin assembly and Gaussian load (host side).
//
// Discretisation: lowest-order Nedelec (Whitney) edge elements on a conforming tetrahedral mesh
// (Sec. 2.2); Galerkin matrix (A)_ij = a(w_j, w_i) of the sesquilinear form eq:Helmholtzvf_intro
// plus the boundary term of the impedance condition eq:imp:
//     A = K - (k^2 + i xi) M - i sign(xi) k M_b.
#include <algorithm>
#include <cmath>
#include <complex>

#include "mx_internal.hpp"

namespace mx {

// The 7 edge directions (v, v + s) of the Kuhn split, in increasing order of the vertex-id
// offset 1 < nx+1 < nx+2 < P < P+1 < P+nx+1 < P+nx+2 (P = (nx+1)(ny+1)), so enumerating them in
// this order for ascending lo lists the edges sorted by (lo, hi).
static const int kDir[7][3] = {{1, 0, 0}, {0, 1, 0}, {1, 1, 0}, {0, 0, 1},
                               {1, 0, 1}, {0, 1, 1}, {1, 1, 1}};
// The 6 axis permutations in lexicographic order.
static const int kPerm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
static const int kLocalEdge[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};

static inline bool dir_valid(const Mesh &m, int i, int j, int k, int d) {
  return i + kDir[d][0] <= m.nx && j + kDir[d][1] <= m.ny && k + kDir[d][2] <= m.nz;
}

int32_t Mesh::edge_id(int32_t lo, int32_t hi) const {
  int i, j, k, i2, j2, k2;
  vijk(lo, i, j, k);
  vijk(hi, i2, j2, k2);
  int s[3] = {i2 - i, j2 - j, k2 - k};
  int rank = 0;
  for (int d = 0; d < 7; ++d) {
    if (!dir_valid(*this, i, j, k, d)) continue;
    if (kDir[d][0] == s[0] && kDir[d][1] == s[1] && kDir[d][2] == s[2]) {
      return (int32_t)(edge_first_[lo] + rank);
    }
    ++rank;
  }
  return -1;
}

void build_mesh(Mesh &m, int nx, int ny, int nz, double lx, double ly, double lz) {
  m.nx = nx, m.ny = ny, m.nz = nz, m.lx = lx, m.ly = ly, m.lz = lz;
  m.nv = (int64_t)(nx + 1) * (ny + 1) * (nz + 1);
  m.nt = 6LL * nx * ny * nz;
  // edges: count valid directions per vertex, prefix sum
  m.edge_first_.assign(m.nv + 1, 0);
  for (int64_t v = 0; v < m.nv; ++v) {
    int i, j, k, c = 0;
    m.vijk(v, i, j, k);
    for (int d = 0; d < 7; ++d) c += dir_valid(m, i, j, k, d);
    m.edge_first_[v + 1] = m.edge_first_[v] + c;
  }
  m.ne = m.edge_first_[m.nv];
  if (m.ne > INT32_MAX || m.nt > INT32_MAX) fail(MX_EINVAL, "mesh too large for int32 ids");
  m.edge_vert.resize(2 * m.ne);
  parallel_for(m.nv, [&](int64_t a, int64_t b) {
    for (int64_t v = a; v < b; ++v) {
      int i, j, k;
      m.vijk(v, i, j, k);
      int64_t e = m.edge_first_[v];
      for (int d = 0; d < 7; ++d) {
        if (!dir_valid(m, i, j, k, d)) continue;
        m.edge_vert[2 * e] = (int32_t)v;
        m.edge_vert[2 * e + 1] = m.vid(i + kDir[d][0], j + kDir[d][1], k + kDir[d][2]);
        ++e;
      }
    }
  });
  // tetrahedra
  m.tet_vert.resize(4 * m.nt);
  m.tet_edge.resize(6 * m.nt);
  m.tet_sign.resize(6 * m.nt);
  int64_t ncube = (int64_t)nx * ny * nz;
  parallel_for(ncube, [&](int64_t a, int64_t b) {
    for (int64_t c = a; c < b; ++c) {
      int ci = (int)(c % nx), cj = (int)((c / nx) % ny), ck = (int)(c / ((int64_t)nx * ny));
      for (int p = 0; p < 6; ++p) {
        int pos[3] = {ci, cj, ck};
        int32_t *tv = &m.tet_vert[4 * (6 * c + p)];
        tv[0] = m.vid(pos[0], pos[1], pos[2]);
        for (int s = 0; s < 3; ++s) {
          pos[kPerm[p][s]] += 1;
          tv[s + 1] = m.vid(pos[0], pos[1], pos[2]);
        }
        for (int e = 0; e < 6; ++e) {
          int32_t va = tv[kLocalEdge[e][0]], vb = tv[kLocalEdge[e][1]];
          int32_t lo = std::min(va, vb), hi = std::max(va, vb);
          m.tet_edge[6 * (6 * c + p) + e] = m.edge_id(lo, hi);
          m.tet_sign[6 * (6 * c + p) + e] = va < vb ? 1 : -1;
        }
      }
    }
  });
  // edge -> tetrahedron incidence, tet ids ascending: counted and filled in parallel (atomic
  // cursors), then each edge's short list is sorted by tet id
  m.et_ptr.assign(m.ne + 1, 0);
  parallel_for(m.nt, [&](int64_t a, int64_t b) {
    for (int64_t t = a; t < b; ++t)
      for (int e = 0; e < 6; ++e)
        __atomic_fetch_add(&m.et_ptr[m.tet_edge[6 * t + e] + 1], (int64_t)1, __ATOMIC_RELAXED);
  });
  for (int64_t e = 0; e < m.ne; ++e) m.et_ptr[e + 1] += m.et_ptr[e];
  m.et_tet.resize(m.et_ptr[m.ne]);
  m.et_loc.resize(m.et_ptr[m.ne]);
  {
    std::vector<int32_t> cursor(m.ne, 0);
    parallel_for(m.nt, [&](int64_t a, int64_t b) {
      for (int64_t t = a; t < b; ++t)
        for (int e = 0; e < 6; ++e) {
          const int32_t g = m.tet_edge[6 * t + e];
          const int64_t q = m.et_ptr[g] + __atomic_fetch_add(&cursor[g], 1, __ATOMIC_RELAXED);
          m.et_tet[q] = (int32_t)t;
          m.et_loc[q] = (int8_t)e;
        }
    });
    parallel_for(m.ne, [&](int64_t a, int64_t b) {
      for (int64_t g = a; g < b; ++g)
        for (int64_t i = m.et_ptr[g] + 1; i < m.et_ptr[g + 1]; ++i) {
          const int32_t t = m.et_tet[i];
          const int8_t l = m.et_loc[i];
          int64_t j = i - 1;
          for (; j >= m.et_ptr[g] && m.et_tet[j] > t; --j) {
            m.et_tet[j + 1] = m.et_tet[j];
            m.et_loc[j + 1] = m.et_loc[j];
          }
          m.et_tet[j + 1] = t;
          m.et_loc[j + 1] = l;
        }
    });
  }
  // boundary triangles: each boundary square (a, a+u, a+w, a+u+w), u < w axes, is split along
  // its diagonal a -> a+u+w into (a, a+u, a+u+w) and (a, a+w, a+u+w)
  m.bface_vert.clear();
  const int n3[3] = {nx, ny, nz};
  for (int normal = 0; normal < 3; ++normal) {
    int u = normal == 0 ? 1 : 0, w = normal == 2 ? 1 : 2;
    for (int side = 0; side < 2; ++side) {
      int fixed = side ? n3[normal] : 0;
      for (int b = 0; b < n3[w]; ++b)
        for (int a = 0; a < n3[u]; ++a) {
          int p[3];
          p[normal] = fixed, p[u] = a, p[w] = b;
          int q1[3] = {p[0], p[1], p[2]}, q2[3] = {p[0], p[1], p[2]}, q3[3] = {p[0], p[1], p[2]};
          q1[u] += 1;
          q2[w] += 1;
          q3[u] += 1, q3[w] += 1;
          int32_t v0 = m.vid(p[0], p[1], p[2]), v1 = m.vid(q1[0], q1[1], q1[2]);
          int32_t v2 = m.vid(q2[0], q2[1], q2[2]), v3 = m.vid(q3[0], q3[1], q3[2]);
          int32_t t1[3] = {v0, v1, v3}, t2[3] = {v0, v2, v3};
          std::sort(t1, t1 + 3);
          std::sort(t2, t2 + 3);
          m.bface_vert.insert(m.bface_vert.end(), t1, t1 + 3);
          m.bface_vert.insert(m.bface_vert.end(), t2, t2 + 3);
        }
    }
  }
  int64_t nbf = (int64_t)m.bface_vert.size() / 3;
  m.bface_edge.resize(3 * nbf);
  m.edge_on_boundary.assign(m.ne, 0);
  m.eb_ptr.assign(m.ne + 1, 0);
  for (int64_t f = 0; f < nbf; ++f) {
    const int32_t *v = &m.bface_vert[3 * f];
    int32_t e3[3] = {m.edge_id(v[0], v[1]), m.edge_id(v[0], v[2]), m.edge_id(v[1], v[2])};
    for (int a = 0; a < 3; ++a) {
      if (e3[a] < 0) fail(MX_EINVAL, "internal: boundary triangle edge missing");
      m.bface_edge[3 * f + a] = e3[a];
      m.edge_on_boundary[e3[a]] = 1;
      m.eb_ptr[e3[a] + 1]++;
    }
  }
  for (int64_t e = 0; e < m.ne; ++e) m.eb_ptr[e + 1] += m.eb_ptr[e];
  m.eb_face.resize(m.eb_ptr[m.ne]);
  {
    std::vector<int64_t> pos(m.eb_ptr.begin(), m.eb_ptr.end() - 1);
    for (int64_t f = 0; f < nbf; ++f)
      for (int a = 0; a < 3; ++a) m.eb_face[pos[m.bface_edge[3 * f + a]]++] = (int32_t)f;
  }
}

// ---- element matrices ----------------------------------------------------------------------------
static inline void cross(const double a[3], const double b[3], double c[3]) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}
static inline double dot(const double a[3], const double b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// Mass-type Whitney integral from gradient dot products G[a][b] and the lambda-product weights
// int lambda_a lambda_b = meas * (1 + delta_ab) * c: for edges (a->b), (c->d),
// int w_ab . w_cd = meas*c*[(1+d_ac)G_bd - (1+d_ad)G_bc - (1+d_bc)G_ad + (1+d_bd)G_ac].
template <int NV>
static double whitney_mass(const double G[NV][NV], int a, int b, int c, int d, double meas,
                           double wc) {
  auto f = [](int x, int y) { return x == y ? 2.0 : 1.0; };
  return meas * wc *
         (f(a, c) * G[b][d] - f(a, d) * G[b][c] - f(b, c) * G[a][d] + f(b, d) * G[a][c]);
}

void tet_element(const double X[4][3], double K[6][6], double M[6][6], double *vol) {
  double c1[3], c2[3], c3[3];
  for (int i = 0; i < 3; ++i) {
    c1[i] = X[1][i] - X[0][i];
    c2[i] = X[2][i] - X[0][i];
    c3[i] = X[3][i] - X[0][i];
  }
  double x23[3], x31[3], x12[3];
  cross(c2, c3, x23);
  cross(c3, c1, x31);
  cross(c1, c2, x12);
  double det = dot(c1, x23);
  double g[4][3];
  for (int i = 0; i < 3; ++i) {
    g[1][i] = x23[i] / det;
    g[2][i] = x31[i] / det;
    g[3][i] = x12[i] / det;
    g[0][i] = -(g[1][i] + g[2][i] + g[3][i]);
  }
  double V = std::fabs(det) / 6.0;
  double G[4][4];
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) G[a][b] = dot(g[a], g[b]);
  double curl[6][3];
  for (int e = 0; e < 6; ++e) {
    cross(g[kLocalEdge[e][0]], g[kLocalEdge[e][1]], curl[e]);
    for (int i = 0; i < 3; ++i) curl[e][i] *= 2.0;
  }
  for (int e = 0; e < 6; ++e)
    for (int f = 0; f < 6; ++f) {
      K[e][f] = V * dot(curl[e], curl[f]);
      M[e][f] = whitney_mass<4>(G, kLocalEdge[e][0], kLocalEdge[e][1], kLocalEdge[f][0],
                                kLocalEdge[f][1], V, 1.0 / 20.0);
    }
  if (vol) *vol = V;
}

void kuhn_elements(double hx, double hy, double hz, KuhnElements &out) {
  const double h[3] = {hx, hy, hz};
  for (int p = 0; p < 6; ++p) {
    double X[4][3] = {{0, 0, 0}};
    double pos[3] = {0, 0, 0};
    for (int s = 0; s < 3; ++s) {
      pos[kPerm[p][s]] += h[kPerm[p][s]];
      for (int i = 0; i < 3; ++i) X[s + 1][i] = pos[i];
    }
    tet_element(X, out.K[p], out.M[p], nullptr);
  }
}

void triangle_mass(const double x0[3], const double x1[3], const double x2[3], double Mb[3][3]) {
  const double *P[3] = {x0, x1, x2};
  double e1[3], e2[3], nn[3];
  for (int i = 0; i < 3; ++i) e1[i] = x1[i] - x0[i], e2[i] = x2[i] - x0[i];
  cross(e1, e2, nn);
  double twoA = std::sqrt(dot(nn, nn));
  double n[3] = {nn[0] / twoA, nn[1] / twoA, nn[2] / twoA};
  // surface gradient of lambda_i = n x (P_{i+2} - P_{i+1}) / (2 area)
  double g[3][3];
  for (int i = 0; i < 3; ++i) {
    const double *a = P[(i + 1) % 3], *b = P[(i + 2) % 3];
    double d[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    cross(n, d, g[i]);
    for (int j = 0; j < 3; ++j) g[i][j] /= twoA;
  }
  double G[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) G[a][b] = dot(g[a], g[b]);
  static const int le[3][2] = {{0, 1}, {0, 2}, {1, 2}};
  for (int e = 0; e < 3; ++e)
    for (int f = 0; f < 3; ++f)
      Mb[e][f] = whitney_mass<3>(G, le[e][0], le[e][1], le[f][0], le[f][1], 0.5 * twoA, 1.0 / 12.0);
}

// ---- global assembly -------------------------------------------------------------------------------
struct Entry {
  int32_t col;
  double re, im;
};

// Sums the contributions of equal columns in arrival order (slot[col] = position of the column's
// entry while a row is built, -1 otherwise) and sorts the distinct columns.
static void merge_entries(std::vector<Entry> &ent, std::vector<int32_t> &slot) {
  size_t w = 0;
  for (size_t r = 0; r < ent.size(); ++r) {
    const int32_t c = ent[r].col;
    if (slot[c] >= 0) {
      ent[slot[c]].re += ent[r].re;
      ent[slot[c]].im += ent[r].im;
    } else {
      slot[c] = (int32_t)w;
      ent[w++] = ent[r];
    }
  }
  ent.resize(w);
  for (const Entry &x : ent) slot[x.col] = -1;
  std::sort(ent.begin(), ent.end(), [](const Entry &a, const Entry &b) { return a.col < b.col; });
}

static double imp_sign(double xi) { return xi >= 0 ? 1.0 : -1.0; }

// Row e of the global matrix: tetrahedra in ascending id, then boundary triangles.  With
// `weight`, row e of the weight D_k = K + k^2 M instead (no boundary term).
static void global_row(const Mesh &m, const KuhnElements &ke, double k, double xi, int bc,
                       bool weight, int64_t e, std::vector<Entry> &ent, std::vector<int32_t> &slot) {
  ent.clear();
  // coefficient -(k^2 + i xi) of M, or +k^2 for the weight
  const double sre = weight ? k * k : -k * k, sim = weight ? 0.0 : -xi;
  for (int64_t q = m.et_ptr[e]; q < m.et_ptr[e + 1]; ++q) {
    int32_t t = m.et_tet[q];
    int a = m.et_loc[q];
    int p = t % 6;
    double sa = m.tet_sign[6 * (int64_t)t + a];
    for (int b = 0; b < 6; ++b) {
      double s = sa * m.tet_sign[6 * (int64_t)t + b];
      ent.push_back({m.tet_edge[6 * (int64_t)t + b], s * (ke.K[p][a][b] + sre * ke.M[p][a][b]),
                     s * sim * ke.M[p][a][b]});
    }
  }
  if (bc == MX_BC_IMPEDANCE && !weight) {
    double cb = -imp_sign(xi) * k;  // coefficient -i sign(xi) k of M_b (purely imaginary)
    for (int64_t q = m.eb_ptr[e]; q < m.eb_ptr[e + 1]; ++q) {
      int32_t f = m.eb_face[q];
      const int32_t *v = &m.bface_vert[3 * (int64_t)f];
      double x0[3], x1[3], x2[3], Mb[3][3];
      m.xyz(v[0], x0), m.xyz(v[1], x1), m.xyz(v[2], x2);
      triangle_mass(x0, x1, x2, Mb);
      int a = 0;
      while (m.bface_edge[3 * (int64_t)f + a] != e) ++a;
      for (int b = 0; b < 3; ++b) ent.push_back({m.bface_edge[3 * (int64_t)f + b], 0.0, cb * Mb[a][b]});
    }
  }
  merge_entries(ent, slot);
  if (bc == MX_BC_PEC) {
    bool row_pec = m.edge_on_boundary[e];
    for (auto &x : ent) {
      if (row_pec || m.edge_on_boundary[x.col]) {
        x.re = (x.col == e && row_pec) ? 1.0 : 0.0;
        x.im = 0.0;
      }
    }
  }
}

void assemble_global(const Mesh &m, double k, double xi, int bc, HostCSR &A, bool weight) {
  KuhnElements ke;
  kuhn_elements(m.lx / m.nx, m.ly / m.ny, m.lz / m.nz, ke);
  A.n = m.ne;
  A.rowptr.assign(m.ne + 1, 0);
  // one pass: each thread assembles a contiguous range of rows into its own buffer, then the
  // buffers are copied into place once the row offsets are known
  const unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  const int64_t chunk = (m.ne + nt - 1) / nt;
  std::vector<std::vector<Entry>> part(nt);
  parallel_for(nt, [&](int64_t t0, int64_t t1) {
    std::vector<Entry> ent;
    std::vector<int32_t> slot(m.ne, -1);
    for (int64_t t = t0; t < t1; ++t) {
      const int64_t a = t * chunk, b = std::min<int64_t>(m.ne, a + chunk);
      std::vector<Entry> &out = part[t];
      out.reserve((size_t)std::max<int64_t>(0, b - a) * 17);  // about 16.3 entries per row
      for (int64_t e = a; e < b; ++e) {
        global_row(m, ke, k, xi, bc, weight, e, ent, slot);
        A.rowptr[e + 1] = (int64_t)ent.size();
        out.insert(out.end(), ent.begin(), ent.end());
      }
    }
  }, 1);
  for (int64_t e = 0; e < m.ne; ++e) A.rowptr[e + 1] += A.rowptr[e];
  A.col.resize(A.rowptr[m.ne]);
  A.val.resize(2 * A.rowptr[m.ne]);
  parallel_for(nt, [&](int64_t t0, int64_t t1) {
    for (int64_t t = t0; t < t1; ++t) {
      const int64_t a = std::min<int64_t>(m.ne, t * chunk);
      std::vector<Entry> &in = part[t];
      int64_t o = A.rowptr[a];
      for (size_t i = 0; i < in.size(); ++i, ++o) {
        A.col[o] = in[i].col;
        A.val[2 * o] = in[i].re;
        A.val[2 * o + 1] = in[i].im;
      }
      std::vector<Entry>().swap(in);
    }
  }, 1);
}

// ---- load vector ------------------------------------------------------------------------------------
void rhs_gaussian(const Mesh &m, int bc, const double c[3], const double pol[3], double sigma,
                  double *f) {
  const double alpha = (5.0 + 3.0 * std::sqrt(5.0)) / 20.0, beta = (5.0 - std::sqrt(5.0)) / 20.0;
  std::fill(f, f + 2 * m.ne, 0.0);
  for (int64_t t = 0; t < m.nt; ++t) {
    double X[4][3];
    for (int a = 0; a < 4; ++a) m.xyz(m.tet_vert[4 * t + a], X[a]);
    double c1[3], c2[3], c3[3], x23[3], x31[3], x12[3];
    for (int i = 0; i < 3; ++i)
      c1[i] = X[1][i] - X[0][i], c2[i] = X[2][i] - X[0][i], c3[i] = X[3][i] - X[0][i];
    cross(c2, c3, x23);
    cross(c3, c1, x31);
    cross(c1, c2, x12);
    double det = dot(c1, x23);
    double g[4][3];
    for (int i = 0; i < 3; ++i) {
      g[1][i] = x23[i] / det, g[2][i] = x31[i] / det, g[3][i] = x12[i] / det;
      g[0][i] = -(g[1][i] + g[2][i] + g[3][i]);
    }
    double w = std::fabs(det) / 6.0 / 4.0;
    double loc[6] = {0, 0, 0, 0, 0, 0};
    for (int q = 0; q < 4; ++q) {
      double lam[4] = {beta, beta, beta, beta};
      lam[q] = alpha;
      double xq[3] = {0, 0, 0};
      for (int a = 0; a < 4; ++a)
        for (int i = 0; i < 3; ++i) xq[i] += lam[a] * X[a][i];
      double r2 = 0;
      for (int i = 0; i < 3; ++i) r2 += (xq[i] - c[i]) * (xq[i] - c[i]);
      double amp = std::exp(-r2 / (2.0 * sigma * sigma));
      for (int e = 0; e < 6; ++e) {
        int a = kLocalEdge[e][0], b = kLocalEdge[e][1];
        double we = 0;
        for (int i = 0; i < 3; ++i) we += (lam[a] * g[b][i] - lam[b] * g[a][i]) * pol[i];
        loc[e] += w * amp * we;
      }
    }
    for (int e = 0; e < 6; ++e) f[2 * (int64_t)m.tet_edge[6 * t + e]] += m.tet_sign[6 * t + e] * loc[e];
  }
  if (bc == MX_BC_PEC)
    for (int64_t e = 0; e < m.ne; ++e)
      if (m.edge_on_boundary[e]) f[2 * e] = f[2 * e + 1] = 0.0;
}

}  // namespace mx
