// Second-order Nedelec elements (first family) on the Kuhn box mesh: hierarchical basis, element
// integrals, global assembly, local DOF sets and ORAS local problems (Sec. 2.2 with order m = 2;
// the paper's order-2 runs are Tables tab:theoryDeltamin and tab:6bis).
//
// Basis, from the global vertex numbering (l = barycentric coordinates):
//   edge i -> j (i < j): Whitney w = l_i grad l_j - l_j grad l_i and gradient g = grad(l_i l_j);
//   face i < j < k:      l_k w_ij and l_j w_ik.
// DOF numbering: the E Whitney functions (the lowest-order numbering, so the lowest-order space
// is the leading block), the E edge gradients, then two per face, faces sorted by vertex triple.
// Along every tetrahedron of the split the vertex ids increase (each step of the path raises one
// coordinate), so a tetrahedron's local vertex order is its global one and its 20 functions
// depend only on its type (one of six) and the cube spacing.  Element integrals are exact:
// every function is a sum of c l^a grad l_m, and int_T l^a = 6 |T| a! / (|a| + 3)!, on a
// triangle 2 |tau| a! / (|a| + 2)!.
#include <array>
#include <cmath>

#include "mx_internal.hpp"

namespace mx {

namespace {
const int kLE[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
const int kLF[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};
const int kPermO2[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

struct Term {
  double c;
  int a[4];
  int m;  // gradient of barycentric m
};
using Fn = std::vector<Term>;

Term term(double c, int i1, int i2, int m) {
  Term t{c, {0, 0, 0, 0}, m};
  if (i1 >= 0) ++t.a[i1];
  if (i2 >= 0) ++t.a[i2];
  return t;
}

// the 20 local functions: 6 Whitney, 6 gradients, 2 per local face
std::vector<Fn> local_functions() {
  std::vector<Fn> f;
  for (auto &e : kLE) f.push_back({term(1, e[0], -1, e[1]), term(-1, e[1], -1, e[0])});
  for (auto &e : kLE) f.push_back({term(1, e[0], -1, e[1]), term(1, e[1], -1, e[0])});
  for (auto &v : kLF) {
    const int i = v[0], j = v[1], k = v[2];
    f.push_back({term(1, k, i, j), term(-1, k, j, i)});
    f.push_back({term(1, j, i, k), term(-1, j, k, i)});
  }
  return f;
}

double fact(int n) {
  double r = 1;
  for (int i = 2; i <= n; ++i) r *= i;
  return r;
}

double int_tet(const int a[4], double vol) {
  return 6.0 * vol * fact(a[0]) * fact(a[1]) * fact(a[2]) * fact(a[3]) / fact(a[0] + a[1] + a[2] + a[3] + 3);
}

double int_tri(const int a[4], double area, int opp) {
  if (a[opp]) return 0.0;
  return 2.0 * area * fact(a[0]) * fact(a[1]) * fact(a[2]) * fact(a[3]) / fact(a[0] + a[1] + a[2] + a[3] + 2);
}

void cross3(const double *x, const double *y, double *z) {
  z[0] = x[1] * y[2] - x[2] * y[1];
  z[1] = x[2] * y[0] - x[0] * y[2];
  z[2] = x[0] * y[1] - x[1] * y[0];
}

// does local function u have a nonzero tangential trace on local face lf (its edges' functions
// and the face's own two)?
bool on_face(int u, int lf) {
  const int opp = lf;  // local face lf leaves out local vertex lf
  if (u < 12) {
    const int e = u % 6;
    return kLE[e][0] != opp && kLE[e][1] != opp;
  }
  return (u - 12) / 2 == lf;
}
}  // namespace

// element matrices of the six Kuhn tetrahedra of a cube with spacing h
static void order2_elements(const double h[3], Order2 &o) {
  const std::vector<Fn> fn = local_functions();
  for (int p = 0; p < 6; ++p) {
    double X[4][3] = {};
    int pos[3] = {0, 0, 0};
    for (int s = 0; s < 3; ++s) {
      pos[kPermO2[p][s]] = 1;
      for (int d = 0; d < 3; ++d) X[s + 1][d] = pos[d] * h[d];
    }
    double J[3][3], Ji[3][3];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) J[r][c] = X[c + 1][r] - X[0][r];  // columns: edge vectors
    const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                       J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                       J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
    Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
    Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
    Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
    Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
    Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
    Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
    Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
    Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
    double g[4][3];  // barycentric gradients: rows of the inverse Jacobian, g0 = -sum
    for (int d = 0; d < 3; ++d) {
      g[1][d] = Ji[0][d], g[2][d] = Ji[1][d], g[3][d] = Ji[2][d];
      g[0][d] = -(Ji[0][d] + Ji[1][d] + Ji[2][d]);
    }
    const double vol = std::fabs(det) / 6.0;
    // curls: sum c a_q l^(a - e_q) (grad l_q x grad l_m)
    struct CTerm {
      double c;
      int a[4];
      double v[3];
    };
    std::vector<std::vector<CTerm>> curl(20);
    for (int u = 0; u < 20; ++u)
      for (const Term &t : fn[u])
        for (int q = 0; q < 4; ++q) {
          if (!t.a[q]) continue;
          CTerm ct{t.c * t.a[q], {t.a[0], t.a[1], t.a[2], t.a[3]}, {0, 0, 0}};
          --ct.a[q];
          cross3(g[q], g[t.m], ct.v);
          curl[u].push_back(ct);
        }
    for (int u = 0; u < 20; ++u)
      for (int v = 0; v < 20; ++v) {
        double mass = 0, stiff = 0;
        for (const Term &s : fn[u])
          for (const Term &t : fn[v]) {
            int a[4];
            for (int q = 0; q < 4; ++q) a[q] = s.a[q] + t.a[q];
            mass += s.c * t.c * int_tet(a, vol) *
                    (g[s.m][0] * g[t.m][0] + g[s.m][1] * g[t.m][1] + g[s.m][2] * g[t.m][2]);
          }
        for (const CTerm &s : curl[u])
          for (const CTerm &t : curl[v]) {
            int a[4];
            for (int q = 0; q < 4; ++q) a[q] = s.a[q] + t.a[q];
            stiff += s.c * t.c * int_tet(a, vol) * (s.v[0] * t.v[0] + s.v[1] * t.v[1] + s.v[2] * t.v[2]);
          }
        o.M[p][u][v] = mass;
        o.K[p][u][v] = stiff;
      }
    for (int lf = 0; lf < 4; ++lf) {
      const double *x0 = X[kLF[lf][0]], *x1 = X[kLF[lf][1]], *x2 = X[kLF[lf][2]];
      double e1[3], e2[3], nrm[3];
      for (int d = 0; d < 3; ++d) e1[d] = x1[d] - x0[d], e2[d] = x2[d] - x0[d];
      cross3(e1, e2, nrm);
      const double len = std::sqrt(nrm[0] * nrm[0] + nrm[1] * nrm[1] + nrm[2] * nrm[2]);
      const double area = 0.5 * len;
      const double n[3] = {nrm[0] / len, nrm[1] / len, nrm[2] / len};
      double gt[4][3];  // tangential parts of the gradients
      for (int q = 0; q < 4; ++q) {
        const double dn = g[q][0] * n[0] + g[q][1] * n[1] + g[q][2] * n[2];
        for (int d = 0; d < 3; ++d) gt[q][d] = g[q][d] - dn * n[d];
      }
      for (int u = 0; u < 20; ++u)
        for (int v = 0; v < 20; ++v) {
          double b = 0;
          if (on_face(u, lf) && on_face(v, lf))
            for (const Term &s : fn[u])
              for (const Term &t : fn[v]) {
                int a[4];
                for (int q = 0; q < 4; ++q) a[q] = s.a[q] + t.a[q];
                b += s.c * t.c * int_tri(a, area, lf) *
                     (gt[s.m][0] * gt[t.m][0] + gt[s.m][1] * gt[t.m][1] + gt[s.m][2] * gt[t.m][2]);
              }
          o.B[p][lf][u][v] = b;
        }
    }
  }
}

void build_order2(const Mesh &m, Order2 &o) {
  o.E = m.ne;
  // faces: sorted vertex triples of every tetrahedron's four faces, made unique
  struct FR {
    int32_t v[3];
    int32_t t;
    int8_t lf;
  };
  std::vector<FR> all((size_t)m.nt * 4);
  parallel_for(m.nt, [&](int64_t a, int64_t b) {
    for (int64_t t = a; t < b; ++t) {
      const int32_t *tv = &m.tet_vert[4 * t];
      for (int lf = 0; lf < 4; ++lf) {
        int32_t v[3] = {tv[kLF[lf][0]], tv[kLF[lf][1]], tv[kLF[lf][2]]};  // ascending already
        all[4 * t + lf] = {{v[0], v[1], v[2]}, (int32_t)t, (int8_t)lf};
      }
    }
  });
  std::sort(all.begin(), all.end(), [](const FR &x, const FR &y) {
    if (x.v[0] != y.v[0]) return x.v[0] < y.v[0];
    if (x.v[1] != y.v[1]) return x.v[1] < y.v[1];
    if (x.v[2] != y.v[2]) return x.v[2] < y.v[2];
    return x.t < y.t;
  });
  o.tet_face.assign((size_t)m.nt * 4, -1);
  o.face_vert.clear();
  o.face_tet.clear();
  o.face_lf.clear();
  for (size_t i = 0; i < all.size();) {
    size_t j = i + 1;
    while (j < all.size() && all[j].v[0] == all[i].v[0] && all[j].v[1] == all[i].v[1] &&
           all[j].v[2] == all[i].v[2])
      ++j;
    if (j - i > 2) fail(MX_EINVAL, "internal: a face shared by more than two tetrahedra");
    const int32_t f = (int32_t)(o.face_vert.size() / 3);
    for (int d = 0; d < 3; ++d) o.face_vert.push_back(all[i].v[d]);
    o.face_tet.push_back(all[i].t);
    o.face_tet.push_back(j - i == 2 ? all[i + 1].t : -1);
    o.face_lf.push_back(all[i].lf);
    o.face_lf.push_back(j - i == 2 ? all[i + 1].lf : -1);
    for (size_t q = i; q < j; ++q) o.tet_face[4 * (size_t)all[q].t + all[q].lf] = f;
    i = j;
  }
  o.F = (int64_t)o.face_vert.size() / 3;
  o.N = 2 * o.E + 2 * o.F;
  if (o.N > INT32_MAX) fail(MX_EINVAL, "too many order-2 degrees of freedom");
  o.dof_boundary.assign(o.N, 0);
  for (int64_t e = 0; e < o.E; ++e) o.dof_boundary[e] = o.dof_boundary[o.E + e] = m.edge_on_boundary[e];
  for (int64_t f = 0; f < o.F; ++f)
    if (o.face_tet[2 * f + 1] < 0) o.dof_boundary[2 * o.E + 2 * f] = o.dof_boundary[2 * o.E + 2 * f + 1] = 1;
  const double h[3] = {m.lx / m.nx, m.ly / m.ny, m.lz / m.nz};
  order2_elements(h, o);
}

int32_t order2_dof(const Mesh &m, const Order2 &o, int64_t t, int a) {
  if (a < 6) return m.tet_edge[6 * t + a];
  if (a < 12) return (int32_t)(o.E + m.tet_edge[6 * t + a - 6]);
  return (int32_t)(2 * o.E + 2 * o.tet_face[4 * t + (a - 12) / 2] + (a - 12) % 2);
}

int32_t order2_face_of(const Order2 &o, const int32_t v[3]) {
  int64_t lo = 0, hi = o.F;
  while (lo < hi) {
    const int64_t mid = (lo + hi) / 2;
    const int32_t *w = &o.face_vert[3 * mid];
    const bool less = w[0] != v[0] ? w[0] < v[0] : w[1] != v[1] ? w[1] < v[1] : w[2] < v[2];
    if (less) lo = mid + 1;
    else hi = mid;
  }
  if (lo < o.F && o.face_vert[3 * lo] == v[0] && o.face_vert[3 * lo + 1] == v[1] && o.face_vert[3 * lo + 2] == v[2])
    return (int32_t)lo;
  return -1;
}

namespace {
struct CEntry {
  int32_t col;
  double re, im;
};
void merge(std::vector<CEntry> &ent) {  // stable by column, sums in push order
  std::stable_sort(ent.begin(), ent.end(), [](const CEntry &a, const CEntry &b) { return a.col < b.col; });
  size_t w = 0;
  for (size_t i = 0; i < ent.size(); ++i) {
    if (w > 0 && ent[w - 1].col == ent[i].col) {
      ent[w - 1].re += ent[i].re;
      ent[w - 1].im += ent[i].im;
    } else {
      ent[w++] = ent[i];
    }
  }
  ent.resize(w);
}
// local index of global DOF d in tetrahedron t, for the incidences of d
struct Inc {
  int32_t t;
  int8_t a;
};
void incidences(const Mesh &m, const Order2 &o, int64_t d, std::vector<Inc> &out) {
  out.clear();
  if (d < 2 * o.E) {
    const int64_t e = d < o.E ? d : d - o.E;
    const int base = d < o.E ? 0 : 6;
    for (int64_t q = m.et_ptr[e]; q < m.et_ptr[e + 1]; ++q) out.push_back({m.et_tet[q], (int8_t)(base + m.et_loc[q])});
  } else {
    const int64_t f = (d - 2 * o.E) / 2, s = (d - 2 * o.E) % 2;
    for (int side = 0; side < 2; ++side)
      if (o.face_tet[2 * f + side] >= 0)
        out.push_back({o.face_tet[2 * f + side], (int8_t)(12 + 2 * o.face_lf[2 * f + side] + s)});
  }
}
}  // namespace

// Row d of K + (sre + i sim) M + i cb M_b over the tetrahedra with inside(t), the boundary term
// on the faces with term_face(t_other); entries merged by global column (summed in a fixed
// order).  The Galerkin matrix has sre = -k^2, sim = -xi, cb = -sign(xi) k; the weight
// D_k = K + k^2 M has sre = k^2, sim = 0 and no boundary term.
template <class Inside, class TermFace>
static void order2_row(const Mesh &m, const Order2 &o, int64_t d, double sre, double sim, double cb,
                       Inside inside, TermFace term_face, std::vector<Inc> &inc,
                       std::vector<CEntry> &ent) {
  ent.clear();
  incidences(m, o, d, inc);
  for (const Inc &x : inc) {
    if (!inside(x.t)) continue;
    const int p = x.t % 6;
    for (int b = 0; b < 20; ++b)
      ent.push_back({order2_dof(m, o, x.t, b), o.K[p][x.a][b] + sre * o.M[p][x.a][b], sim * o.M[p][x.a][b]});
    for (int lf = 0; lf < 4; ++lf) {
      if (!on_face(x.a, lf)) continue;
      const int32_t f = o.tet_face[4 * (int64_t)x.t + lf];
      const int32_t t2 = o.face_tet[2 * f] == x.t ? o.face_tet[2 * f + 1] : o.face_tet[2 * f];
      if (!term_face(t2)) continue;
      for (int b = 0; b < 20; ++b)
        if (on_face(b, lf)) ent.push_back({order2_dof(m, o, x.t, b), 0.0, cb * o.B[p][lf][x.a][b]});
    }
  }
  merge(ent);
}

void assemble_order2(const Mesh &m, const Order2 &o, double k, double xi, int bc, HostCSR &A,
                     bool weight) {
  const int64_t N = o.N;
  const double sre = weight ? k * k : -k * k, sim = weight ? 0.0 : -xi;
  const double cb = -(xi >= 0 ? 1.0 : -1.0) * k;
  const bool bterm = bc == MX_BC_IMPEDANCE && !weight;
  // rows in chunks handed out to the host threads; each chunk packs its rows contiguously
  const int64_t cs = 4096, nchunk = (N + cs - 1) / cs;
  std::vector<std::vector<CEntry>> packed(nchunk);
  A.n = N;
  A.rowptr.assign(N + 1, 0);
  parallel_items(nchunk, [&](auto next) {
    std::vector<Inc> inc;
    std::vector<CEntry> ent;
    for (int64_t c; (c = next()) >= 0;) {
      auto &out = packed[c];
      for (int64_t d = c * cs; d < std::min(N, (c + 1) * cs); ++d) {
        order2_row(m, o, d, sre, sim, cb, [](int32_t) { return true; },
                   [bterm](int32_t t2) { return t2 < 0 && bterm; }, inc, ent);
        const size_t before = out.size();
        if (bc == MX_BC_PEC && o.dof_boundary[d]) {
          out.push_back({(int32_t)d, 1.0, 0.0});
        } else {
          for (const auto &x : ent)
            if (bc != MX_BC_PEC || !o.dof_boundary[x.col]) out.push_back(x);
        }
        A.rowptr[d + 1] = (int64_t)(out.size() - before);
      }
    }
  });
  for (int64_t d = 0; d < N; ++d) A.rowptr[d + 1] += A.rowptr[d];
  A.col.resize(A.rowptr[N]);
  A.val.resize(2 * A.rowptr[N]);
  parallel_items(nchunk, [&](auto next) {
    for (int64_t c; (c = next()) >= 0;) {
      int64_t q = A.rowptr[c * cs];
      for (const auto &x : packed[c]) {
        A.col[q] = x.col;
        A.val[2 * q] = x.re;
        A.val[2 * q + 1] = x.im;
        ++q;
      }
      std::vector<CEntry>().swap(packed[c]);
    }
  });
}

void order2_sets(const Mesh &m, const Order2 &o, const Partition &p, int kind,
                 std::vector<std::vector<int32_t>> &sets, std::vector<int32_t> &owner) {
  const int64_t E = o.E;
  sets.assign(p.nsub, {});
  parallel_items(p.nsub, [&](auto next) {
    std::vector<int32_t> stamp(m.nt, -1), fseen;
    for (int64_t l; (l = next()) >= 0;) {
      for (int32_t t : p.tets[l]) stamp[t] = (int32_t)l;
      const auto &es = kind == MX_ORAS ? p.oras_set[l] : p.as_set[l];
      std::vector<int32_t> faces;
      for (int32_t t : p.tets[l])
        for (int lf = 0; lf < 4; ++lf) {
          const int32_t f = o.tet_face[4 * (int64_t)t + lf];
          if (kind != MX_ORAS) {  // AS: every tetrahedron of the face inside the subdomain
            const int32_t t2 = o.face_tet[2 * f + 1] == t ? o.face_tet[2 * f] : o.face_tet[2 * f + 1];
            if (t2 >= 0 && stamp[t2] != l) continue;
          }
          faces.push_back(f);
        }
      std::sort(faces.begin(), faces.end());
      faces.erase(std::unique(faces.begin(), faces.end()), faces.end());
      auto &s = sets[l];
      s.reserve(2 * es.size() + 2 * faces.size());
      for (int32_t e : es) s.push_back(e);
      for (int32_t e : es) s.push_back((int32_t)(E + e));
      for (int32_t f : faces) {
        s.push_back((int32_t)(2 * E + 2 * f));
        s.push_back((int32_t)(2 * E + 2 * f + 1));
      }
    }
  });
  owner.assign(o.N, 0);
  for (int64_t e = 0; e < E; ++e) owner[e] = owner[E + e] = p.owner[e];
  for (int64_t f = 0; f < o.F; ++f) {
    int32_t w = p.part0[o.face_tet[2 * f]];
    if (o.face_tet[2 * f + 1] >= 0) w = std::min(w, p.part0[o.face_tet[2 * f + 1]]);
    owner[2 * E + 2 * f] = owner[2 * E + 2 * f + 1] = w;
  }
}

void local_impedance2(const Mesh &m, const Order2 &o, double k, double xi, int bc,
                      const std::vector<int32_t> &tets, const std::vector<int32_t> &set,
                      LocalCSR &out, std::vector<int32_t> &g2l, std::vector<int32_t> &tet_pos) {
  const int64_t n = (int64_t)set.size();
  const int32_t nt = (int32_t)tets.size();
  for (int64_t i = 0; i < n; ++i) g2l[set[i]] = (int32_t)i;
  // tet_pos[t] = position of t in `tets`; an entry left by an earlier subdomain fails the check
  for (int32_t j = 0; j < nt; ++j) tet_pos[tets[j]] = j;
  auto inside = [&](int32_t t) {
    if (t < 0) return false;
    const int32_t j = tet_pos[t];
    return j >= 0 && j < nt && tets[j] == t;
  };
  // impedance on the faces of the subdomain's boundary; a face of the box keeps PEC under PEC
  auto term_face = [&](int32_t t2) { return t2 < 0 ? bc == MX_BC_IMPEDANCE : !inside(t2); };
  out.n = n;
  out.rowptr.assign(1, 0);
  out.col.clear();
  out.val.clear();
  std::vector<Inc> inc;
  std::vector<CEntry> ent;
  for (int64_t i = 0; i < n; ++i) {
    const int32_t d = set[i];
    order2_row(m, o, d, -k * k, -xi, -(xi >= 0 ? 1.0 : -1.0) * k, inside, term_face, inc, ent);
    const bool rp = bc == MX_BC_PEC && o.dof_boundary[d];
    for (const auto &x : ent) {  // global columns ascending, so local columns ascend too
      const int32_t lc = g2l[x.col];
      if (lc < 0) fail(MX_EINVAL, "internal: order-2 local set misses a DOF of its tetrahedra");
      if (rp || (bc == MX_BC_PEC && o.dof_boundary[x.col])) {
        if (rp && x.col == d) {
          out.col.push_back(lc);
          out.val.push_back(1.0);
          out.val.push_back(0.0);
        }
        continue;
      }
      out.col.push_back(lc);
      out.val.push_back(x.re);
      out.val.push_back(x.im);
    }
    out.rowptr.push_back((int64_t)out.col.size());
  }
  for (int64_t i = 0; i < n; ++i) g2l[set[i]] = -1;
}

}  // namespace mx
