// Overlapping box partition, local DOF sets, Boolean partition of unity, local matrices,
// reverse Cuthill-McKee ordering and block-skyline layout (host side).
//
// Subdomains (Sec. 3.1, Sec. 6.1): non-overlapping boxes of cubes, grown by `layers` sweeps that
// add every tetrahedron sharing a vertex with the current set.  Local DOFs for AS/RAS
// (eq:restriction1): edges all of whose tetrahedra lie in the subdomain, so the minor
// R A R^T (eq:minor) is the PEC local problem; for ORAS (ImpRAS, Sec. 6.3): all edges of the
// subdomain's tetrahedra with the local impedance problem.  Partition of unity
// (eq:algebPartUnity): owner(e) = least non-overlapping part containing a tetrahedron of e.
#include <algorithm>
#include <array>
#include <cmath>
#include <numeric>

#include "mx_internal.hpp"

namespace mx {

static const int kLocalFace[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};

void build_partition(const Mesh &m, int px, int py, int pz, const int32_t *cx, const int32_t *cy,
                     const int32_t *cz, int layers, Partition &p) {
  if (px < 1 || py < 1 || pz < 1 || layers < 0) fail(MX_EINVAL, "partition: bad counts");
  const int n3[3] = {m.nx, m.ny, m.nz};
  const int p3[3] = {px, py, pz};
  const int32_t *c3[3] = {cx, cy, cz};
  p.px = px, p.py = py, p.pz = pz, p.layers = layers, p.nsub = px * py * pz;
  std::vector<int32_t> axis_box[3];
  for (int a = 0; a < 3; ++a) {
    if (p3[a] > n3[a]) fail(MX_EINVAL, "partition: more boxes than cubes along an axis");
    p.cuts[a].resize(p3[a] + 1);
    for (int i = 0; i <= p3[a]; ++i)
      p.cuts[a][i] = c3[a] ? c3[a][i] : (int32_t)(((int64_t)i * n3[a]) / p3[a]);
    if (p.cuts[a][0] != 0 || p.cuts[a][p3[a]] != n3[a]) fail(MX_EINVAL, "partition: cuts must span the box");
    for (int i = 0; i < p3[a]; ++i)
      if (p.cuts[a][i + 1] <= p.cuts[a][i]) fail(MX_EINVAL, "partition: cuts must increase");
    axis_box[a].resize(n3[a]);
    for (int i = 0; i < p3[a]; ++i)
      for (int c = p.cuts[a][i]; c < p.cuts[a][i + 1]; ++c) axis_box[a][c] = i;
  }
  p.part0.resize(m.nt);
  parallel_for(m.nt, [&](int64_t a, int64_t b) {
    for (int64_t t = a; t < b; ++t) {
      int64_t c = t / 6;
      int ci = (int)(c % m.nx), cj = (int)((c / m.nx) % m.ny), ck = (int)(c / ((int64_t)m.nx * m.ny));
      p.part0[t] = axis_box[0][ci] + px * (axis_box[1][cj] + py * axis_box[2][ck]);
    }
  });
  p.tets.assign(p.nsub, {});
  p.as_set.assign(p.nsub, {});
  p.oras_set.assign(p.nsub, {});
  // one subdomain per task; per-thread stamp arrays for vertices, tetrahedra and edges
  parallel_items(p.nsub, [&](auto next) {
    std::vector<int32_t> vstamp(m.nv, -1), tstamp(m.nt, -1), estamp(m.ne, -1);
    int32_t gen = 0;
    for (int64_t l; (l = next()) >= 0;) {
      int b[3] = {(int)(l % px), (int)((l / px) % py), (int)(l / ((int64_t)px * py))};
      int lo[3], hi[3], clo[3], chi[3];
      for (int a = 0; a < 3; ++a) {
        lo[a] = p.cuts[a][b[a]], hi[a] = p.cuts[a][b[a] + 1];
        clo[a] = std::max(0, lo[a] - layers), chi[a] = std::min(n3[a], hi[a] + layers);
      }
      // candidate tetrahedra (cubes within `layers` of the box), ascending tet id
      std::vector<int32_t> cand;
      for (int k = clo[2]; k < chi[2]; ++k)
        for (int j = clo[1]; j < chi[1]; ++j)
          for (int i = clo[0]; i < chi[0]; ++i) {
            int64_t c = i + (int64_t)m.nx * (j + (int64_t)m.ny * k);
            for (int q = 0; q < 6; ++q) cand.push_back((int32_t)(6 * c + q));
          }
      std::vector<int32_t> cur;
      for (int32_t t : cand)
        if (p.part0[t] == l) cur.push_back(t);
      for (int sweep = 0; sweep < layers; ++sweep) {
        ++gen;
        for (int32_t t : cur)
          for (int a = 0; a < 4; ++a) vstamp[m.tet_vert[4 * (int64_t)t + a]] = gen;
        std::vector<int32_t> nxt;
        for (int32_t t : cand) {
          const int32_t *tv = &m.tet_vert[4 * (int64_t)t];
          if (vstamp[tv[0]] == gen || vstamp[tv[1]] == gen || vstamp[tv[2]] == gen ||
              vstamp[tv[3]] == gen)
            nxt.push_back(t);
        }
        cur.swap(nxt);
      }
      ++gen;
      for (int32_t t : cur) tstamp[t] = gen;
      std::vector<int32_t> oras;
      for (int32_t t : cur)
        for (int e = 0; e < 6; ++e) {
          int32_t g = m.tet_edge[6 * (int64_t)t + e];
          if (estamp[g] != gen) {
            estamp[g] = gen;
            oras.push_back(g);
          }
        }
      std::sort(oras.begin(), oras.end());
      std::vector<int32_t> as;
      for (int32_t g : oras) {
        bool all = true;
        for (int64_t q = m.et_ptr[g]; q < m.et_ptr[g + 1] && all; ++q) all = tstamp[m.et_tet[q]] == gen;
        if (all) as.push_back(g);
      }
      p.tets[l].swap(cur);
      p.oras_set[l].swap(oras);
      p.as_set[l].swap(as);
    }
  });
  p.owner.assign(m.ne, 0);
  parallel_for(m.ne, [&](int64_t a, int64_t b) {
    for (int64_t e = a; e < b; ++e) {
      int32_t o = INT32_MAX;
      for (int64_t q = m.et_ptr[e]; q < m.et_ptr[e + 1]; ++q) o = std::min(o, p.part0[m.et_tet[q]]);
      p.owner[e] = o;
    }
  });
}

// ---- local matrices ------------------------------------------------------------------------------
struct LEntry {
  int32_t col;
  double re, im;
};

static void merge_row(std::vector<LEntry> &ent) {
  // stable insertion sort by column: rows hold a few dozen entries, and equal columns keep their
  // order, so the sums below are taken in push order (as a stable sort would)
  for (size_t i = 1; i < ent.size(); ++i) {
    const LEntry x = ent[i];
    size_t j = i;
    for (; j > 0 && ent[j - 1].col > x.col; --j) ent[j] = ent[j - 1];
    ent[j] = x;
  }
  size_t w = 0;
  for (size_t r = 0; r < ent.size(); ++r) {
    if (w > 0 && ent[w - 1].col == ent[r].col) {
      ent[w - 1].re += ent[r].re;
      ent[w - 1].im += ent[r].im;
    } else {
      ent[w++] = ent[r];
    }
  }
  ent.resize(w);
}

static void push_row(LocalCSR &out, const std::vector<LEntry> &ent) {
  for (const auto &x : ent) {
    out.col.push_back(x.col);
    out.val.push_back(x.re);
    out.val.push_back(x.im);
  }
  out.rowptr.push_back((int64_t)out.col.size());
}

void local_minor(const uint8_t *boundary, const HostCSR &A, int bc, const std::vector<int32_t> &set,
                 LocalCSR &out, std::vector<int32_t> &g2l) {
  const int64_t n = (int64_t)set.size();
  for (int64_t i = 0; i < n; ++i) g2l[set[i]] = (int32_t)i;
  out.n = n;
  out.rowptr.assign(1, 0);
  out.col.clear();
  out.val.clear();
  std::vector<LEntry> ent;
  for (int64_t i = 0; i < n; ++i) {
    int32_t g = set[i];
    ent.clear();
    bool row_pec = bc == MX_BC_PEC && boundary[g];
    for (int64_t q = A.rowptr[g]; q < A.rowptr[g + 1]; ++q) {
      int32_t c = A.col[q];
      int32_t lc = g2l[c];
      if (lc < 0) continue;
      if (bc == MX_BC_PEC && (row_pec || boundary[c]) && c != g) continue;
      ent.push_back({lc, A.val[2 * q], A.val[2 * q + 1]});
    }
    push_row(out, ent);
  }
  for (int64_t i = 0; i < n; ++i) g2l[set[i]] = -1;
}

static bool on_box_boundary(const Mesh &m, const int32_t v[3]) {
  int I[3][3];
  for (int a = 0; a < 3; ++a) m.vijk(v[a], I[a][0], I[a][1], I[a][2]);
  const int n3[3] = {m.nx, m.ny, m.nz};
  for (int d = 0; d < 3; ++d)
    for (int side = 0; side < 2; ++side) {
      int want = side ? n3[d] : 0;
      if (I[0][d] == want && I[1][d] == want && I[2][d] == want) return true;
    }
  return false;
}

void local_impedance(const Mesh &m, const KuhnElements &ke, double k, double xi, int bc,
                     const std::vector<int32_t> &tets, const std::vector<int32_t> &set,
                     LocalCSR &out, std::vector<int32_t> &g2l, std::vector<int32_t> &tet_pos) {
  const int64_t n = (int64_t)set.size();
  const int32_t nt = (int32_t)tets.size();
  for (int64_t i = 0; i < n; ++i) g2l[set[i]] = (int32_t)i;
  // tet_pos[t] = position of t in `tets`; an entry left by an earlier subdomain fails the check
  for (int32_t j = 0; j < nt; ++j) tet_pos[tets[j]] = j;
  auto local_tet = [&](int32_t t) {
    const int32_t j = tet_pos[t];
    return j >= 0 && j < nt && tets[j] == t ? j : -1;
  };
  // per tetrahedron of the subdomain: local ids and signs of its 6 edges
  std::vector<std::array<int32_t, 6>> tle(nt);
  std::vector<std::array<double, 6>> tsg(nt);
  for (int32_t j = 0; j < nt; ++j) {
    const int64_t t = tets[j];
    for (int b = 0; b < 6; ++b) {
      tle[j][b] = g2l[m.tet_edge[6 * t + b]];
      tsg[j][b] = m.tet_sign[6 * t + b];
    }
  }
  // faces of the subdomain's tetrahedra that appear once: the boundary of the subdomain.  The
  // other tetrahedron on a face (if any) is the one besides t that contains the face's first edge
  // and its third vertex; the face is on the boundary unless that tetrahedron is in the
  // subdomain.  Sorted by vertex triple.
  std::vector<std::array<int32_t, 3>> bfaces;
  for (int32_t t : tets) {
    const int32_t *tv = &m.tet_vert[4 * (int64_t)t];
    for (int f = 0; f < 4; ++f) {
      std::array<int32_t, 3> v = {tv[kLocalFace[f][0]], tv[kLocalFace[f][1]], tv[kLocalFace[f][2]]};
      std::sort(v.begin(), v.end());
      const int32_t e = m.edge_id(v[0], v[1]);
      bool inside = false;
      for (int64_t q = m.et_ptr[e]; q < m.et_ptr[e + 1] && !inside; ++q) {
        const int32_t u = m.et_tet[q];
        if (u == t || local_tet(u) < 0) continue;
        const int32_t *uv = &m.tet_vert[4 * (int64_t)u];
        inside = uv[0] == v[2] || uv[1] == v[2] || uv[2] == v[2] || uv[3] == v[2];
      }
      if (!inside && !(bc == MX_BC_PEC && on_box_boundary(m, v.data()))) bfaces.push_back(v);
    }
  }
  std::sort(bfaces.begin(), bfaces.end());
  // local row -> boundary faces incidence
  const double cb = -(xi >= 0 ? 1.0 : -1.0) * k;
  std::vector<std::array<int32_t, 3>> fedge(bfaces.size());
  std::vector<std::array<double, 9>> fmass(bfaces.size());
  std::vector<int64_t> rf_ptr(n + 1, 0);
  for (size_t f = 0; f < bfaces.size(); ++f) {
    const auto &v = bfaces[f];
    int32_t ge[3] = {m.edge_id(v[0], v[1]), m.edge_id(v[0], v[2]), m.edge_id(v[1], v[2])};
    for (int a = 0; a < 3; ++a) {
      fedge[f][a] = g2l[ge[a]];
      rf_ptr[fedge[f][a] + 1]++;
    }
    double x0[3], x1[3], x2[3], Mb[3][3];
    m.xyz(v[0], x0), m.xyz(v[1], x1), m.xyz(v[2], x2);
    triangle_mass(x0, x1, x2, Mb);
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) fmass[f][3 * a + b] = Mb[a][b];
  }
  for (int64_t i = 0; i < n; ++i) rf_ptr[i + 1] += rf_ptr[i];
  std::vector<int32_t> rf(rf_ptr[n]);
  {
    std::vector<int64_t> pos(rf_ptr.begin(), rf_ptr.end() - 1);
    for (size_t f = 0; f < bfaces.size(); ++f)
      for (int a = 0; a < 3; ++a) rf[pos[fedge[f][a]]++] = (int32_t)f;
  }
  out.n = n;
  out.rowptr.assign(1, 0);
  out.col.clear();
  out.val.clear();
  std::vector<LEntry> ent;
  const double sre = -k * k, sim = -xi;
  for (int64_t i = 0; i < n; ++i) {
    int32_t g = set[i];
    ent.clear();
    for (int64_t q = m.et_ptr[g]; q < m.et_ptr[g + 1]; ++q) {
      const int32_t t = m.et_tet[q];
      const int32_t j = local_tet(t);
      if (j < 0) continue;
      const int a = m.et_loc[q], pp = t % 6;
      const double sa = tsg[j][a];
      for (int b = 0; b < 6; ++b) {
        const double s = sa * tsg[j][b];
        ent.push_back({tle[j][b], s * (ke.K[pp][a][b] + sre * ke.M[pp][a][b]), s * sim * ke.M[pp][a][b]});
      }
    }
    for (int64_t q = rf_ptr[i]; q < rf_ptr[i + 1]; ++q) {
      int32_t f = rf[q];
      int a = 0;
      while (fedge[f][a] != i) ++a;
      for (int b = 0; b < 3; ++b) ent.push_back({fedge[f][b], 0.0, cb * fmass[f][3 * a + b]});
    }
    merge_row(ent);
    if (bc == MX_BC_PEC) {
      bool row_pec = m.edge_on_boundary[g];
      std::vector<LEntry> kept;
      for (const auto &x : ent) {
        bool col_pec = m.edge_on_boundary[set[x.col]];
        if (row_pec || col_pec) {
          if (x.col == i && row_pec) kept.push_back({x.col, 1.0, 0.0});
        } else {
          kept.push_back(x);
        }
      }
      ent.swap(kept);
    }
    push_row(out, ent);
  }
  for (int64_t i = 0; i < n; ++i) g2l[set[i]] = -1;
}

// ---- reverse Cuthill-McKee ------------------------------------------------------------------------
// key(u) = (degree, index); per component: least-key start, George-Liu pseudo-peripheral root
// (move to the least-key vertex of the last level while the level structure gets deeper),
// Cuthill-McKee order with neighbours appended by increasing key; the whole order reversed.
void rcm_order(const LocalCSR &a, std::vector<int32_t> &perm) {
  const int64_t n = a.n;
  std::vector<int32_t> deg(n);
  std::vector<int64_t> ptr(n + 1, 0);
  for (int64_t u = 0; u < n; ++u) {
    int32_t d = 0;
    for (int64_t q = a.rowptr[u]; q < a.rowptr[u + 1]; ++q) d += a.col[q] != u;
    deg[u] = d;
    ptr[u + 1] = ptr[u] + d;
  }
  std::vector<int32_t> adj(ptr[n]);
  for (int64_t u = 0; u < n; ++u) {
    int64_t w = ptr[u];
    for (int64_t q = a.rowptr[u]; q < a.rowptr[u + 1]; ++q)
      if (a.col[q] != u) adj[w++] = a.col[q];
  }
  auto less = [&](int32_t x, int32_t y) { return deg[x] != deg[y] ? deg[x] < deg[y] : x < y; };
  std::vector<int32_t> by_key(n);
  std::iota(by_key.begin(), by_key.end(), 0);
  std::sort(by_key.begin(), by_key.end(), less);
  std::vector<uint8_t> visited(n, 0);
  std::vector<int32_t> seen(n, -1);
  int32_t seen_gen = 0;
  std::vector<int32_t> frontier, nxt, last;
  auto levels = [&](int32_t root, std::vector<int32_t> &last_out) {
    ++seen_gen;
    seen[root] = seen_gen;
    frontier.assign(1, root);
    int depth = 0;
    while (!frontier.empty()) {
      ++depth;
      last_out = frontier;
      nxt.clear();
      for (int32_t u : frontier)
        for (int64_t q = ptr[u]; q < ptr[u + 1]; ++q) {
          int32_t v = adj[q];
          if (seen[v] != seen_gen && !visited[v]) {
            seen[v] = seen_gen;
            nxt.push_back(v);
          }
        }
      frontier.swap(nxt);
    }
    return depth;
  };
  std::vector<int32_t> order;
  order.reserve(n);
  int64_t cursor = 0;
  std::vector<int32_t> cand, lx;
  while ((int64_t)order.size() < n) {
    while (visited[by_key[cursor]]) ++cursor;
    int32_t root = by_key[cursor];
    int depth = levels(root, last);
    while (true) {
      int32_t x = last[0];
      for (int32_t v : last)
        if (less(v, x)) x = v;
      int dx = levels(x, lx);
      if (dx > depth) {
        root = x, depth = dx;
        last.swap(lx);
      } else {
        break;
      }
    }
    size_t head = order.size();
    visited[root] = 1;
    order.push_back(root);
    while (head < order.size()) {
      int32_t u = order[head++];
      cand.clear();
      for (int64_t q = ptr[u]; q < ptr[u + 1]; ++q)
        if (!visited[adj[q]]) cand.push_back(adj[q]);
      std::sort(cand.begin(), cand.end(), less);
      cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
      for (int32_t v : cand) visited[v] = 1;
      order.insert(order.end(), cand.begin(), cand.end());
    }
  }
  perm.assign(order.rbegin(), order.rend());
}

// ---- block skyline ------------------------------------------------------------------------------
void build_skyline(const LocalCSR &a, Skyline &s) {
  const int64_t n = a.n;
  s.n = n;
  rcm_order(a, s.perm);
  s.iperm.assign(n, 0);
  for (int64_t i = 0; i < n; ++i) s.iperm[s.perm[i]] = (int32_t)i;
  s.first.assign(n, 0);
  s.env = 0;
  s.env_flops = 0;
  for (int64_t i = 0; i < n; ++i) {
    int32_t old = s.perm[i];
    int32_t f = (int32_t)i;
    for (int64_t q = a.rowptr[old]; q < a.rowptr[old + 1]; ++q) f = std::min(f, s.iperm[a.col[q]]);
    s.first[i] = f;
    double w = (double)(i - f);
    s.env += (int64_t)(i - f + 1);
    s.env_flops += 8.0 * w * w / 2.0;
  }
  s.nb = (n + TILE - 1) / TILE;
  s.bfirst.assign(s.nb, 0);
  for (int64_t I = 0; I < s.nb; ++I) {
    int32_t f = INT32_MAX;
    for (int64_t i = I * TILE; i < std::min(n, (I + 1) * TILE); ++i) f = std::min(f, s.first[i]);
    s.bfirst[I] = f / TILE;
  }
  for (int64_t I = s.nb - 2; I >= 0; --I) s.bfirst[I] = std::min(s.bfirst[I], s.bfirst[I + 1]);
  s.brow_off.assign(s.nb + 1, 0);
  for (int64_t I = 0; I < s.nb; ++I) s.brow_off[I + 1] = s.brow_off[I] + (I - s.bfirst[I] + 1);
  s.tiles = s.brow_off[s.nb];
  s.blast.assign(s.nb, 0);
  int64_t I = 0;
  for (int64_t K = 0; K < s.nb; ++K) {
    while (I + 1 < s.nb && s.bfirst[I + 1] <= K) ++I;
    s.blast[K] = (int32_t)std::max<int64_t>(I, K);
  }
  const double t3 = (double)TILE * TILE * TILE * 8.0;
  s.tile_flops = 0;
  for (int64_t K = 0; K < s.nb; ++K) {
    double mK = (double)(s.blast[K] - K);
    s.tile_flops += t3 * (mK + mK * (mK + 1) / 2.0);
  }
}

}  // namespace mx
