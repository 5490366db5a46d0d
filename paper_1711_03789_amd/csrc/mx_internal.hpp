// Internal types shared by the host topology code and the device code of libmx.
#pragma once

#include <cstdint>
#include <cstdio>
#include <string>
#include <memory>
#include <utility>
#include <vector>
#include <atomic>
#include <thread>
#include <algorithm>
#include <exception>
#include <mutex>

#include "../../include/mx.h"

namespace mx {

// ---- errors ------------------------------------------------------------------------------------
struct Error {
  int code;
  std::string msg;
};
void set_error(int code, const std::string &msg);
[[noreturn]] void fail(int code, const std::string &msg);

// Exceptions thrown on worker threads: the first one is kept, every thread is joined, then it is
// rethrown on the calling thread (an exception escaping a std::thread, or a joinable thread
// destroyed during unwinding, would terminate the process).
struct FirstError {
  std::mutex mu;
  std::exception_ptr e;
  std::atomic<bool> failed{false};
  template <class G>
  void run(G &&g) {
    try {
      g();
    } catch (...) {
      std::lock_guard<std::mutex> lk(mu);
      if (!e) e = std::current_exception();
      failed.store(true);
    }
  }
  void rethrow() {
    if (e) std::rethrow_exception(e);
  }
};

// Runs f(begin, end) over [0, n) split across up to 16 host threads.
template <class F>
void parallel_for(int64_t n, F &&f, int64_t grain = 4096) {
  unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if (n < grain || nt == 1) {
    f((int64_t)0, n);
    return;
  }
  FirstError err;
  std::vector<std::thread> th;
  const int64_t chunk = (n + nt - 1) / nt;
  err.run([&] {
    for (unsigned t = 1; t < nt; ++t) {
      const int64_t a = (int64_t)t * chunk, b = std::min(n, a + chunk);
      if (a >= b) break;
      th.emplace_back([&f, &err, a, b] { err.run([&] { f(a, b); }); });
    }
  });
  err.run([&] { f((int64_t)0, std::min(n, chunk)); });
  for (auto &x : th) x.join();
  err.rethrow();
}

// Items of very different cost (subdomains): f(next) runs once on each of up to 16 threads, so
// it can set up per-thread scratch; next() hands out the unclaimed items in order, then -1.
// After a failure on any thread the remaining items are not handed out.
template <class F>
void parallel_items(int64_t n, F &&f) {
  unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  nt = (unsigned)std::max<int64_t>(1, std::min<int64_t>(nt, n));
  std::atomic<int64_t> counter(0);
  FirstError err;
  auto next = [&counter, n]() -> int64_t {
    const int64_t i = counter.fetch_add(1);
    return i < n ? i : -1;
  };
  auto body = [&] {
    err.run([&] { f(next); });
    if (err.failed.load()) counter.store(n);
  };
  std::vector<std::thread> th;
  err.run([&] {
    for (unsigned t = 1; t < nt; ++t) th.emplace_back(body);
  });
  body();
  for (auto &x : th) x.join();
  err.rethrow();
}

// ---- structured Kuhn mesh ------------------------------------------------------------------------
struct Mesh {
  int nx = 0, ny = 0, nz = 0;
  double lx = 1, ly = 1, lz = 1;
  int64_t nv = 0, nt = 0, ne = 0;
  std::vector<int32_t> tet_vert;     // [nt][4]
  std::vector<int32_t> tet_edge;     // [nt][6]
  std::vector<int8_t> tet_sign;      // [nt][6]
  std::vector<int32_t> edge_vert;    // [ne][2]
  std::vector<int64_t> et_ptr;       // edge -> incident tetrahedra (CSR, tet ids ascending)
  std::vector<int32_t> et_tet;
  std::vector<int8_t> et_loc;        // local edge index of the edge in that tet
  std::vector<int32_t> bface_vert;   // [nbf][3] boundary triangles, vertices ascending
  std::vector<int32_t> bface_edge;   // [nbf][3] edges (0,1) (0,2) (1,2) of the triangle
  std::vector<int64_t> eb_ptr;       // edge -> incident boundary triangles (CSR)
  std::vector<int32_t> eb_face;
  std::vector<uint8_t> edge_on_boundary;
  std::vector<int64_t> edge_first_;  // first edge id with lo = v (closed-form numbering)

  int32_t vid(int i, int j, int k) const { return i + (nx + 1) * (j + (ny + 1) * k); }
  void vijk(int64_t v, int &i, int &j, int &k) const {
    i = (int)(v % (nx + 1));
    int64_t r = v / (nx + 1);
    j = (int)(r % (ny + 1));
    k = (int)(r / (ny + 1));
  }
  void xyz(int64_t v, double out[3]) const {
    int i, j, k;
    vijk(v, i, j, k);
    out[0] = i * (lx / nx);
    out[1] = j * (ly / ny);
    out[2] = k * (lz / nz);
  }
  int32_t edge_id(int32_t lo, int32_t hi) const;  // -1 if not an edge
};
void build_mesh(Mesh &m, int nx, int ny, int nz, double lx, double ly, double lz);

// Whitney element matrices of the 6 Kuhn tetrahedra of a cube with spacing (hx, hy, hz):
// K[p][a][b], M[p][a][b] in local edge orientation; they are translation invariant.
struct KuhnElements {
  double K[6][6][6];
  double M[6][6][6];
};
void kuhn_elements(double hx, double hy, double hz, KuhnElements &out);
// Tangential Whitney mass of a triangle with vertices x0, x1, x2 (local edges (0,1) (0,2) (1,2)).
void triangle_mass(const double x0[3], const double x1[3], const double x2[3], double Mb[3][3]);
void tet_element(const double X[4][3], double K[6][6], double M[6][6], double *vol);

// ---- complex CSR ---------------------------------------------------------------------------------
// std::vector whose resize leaves new elements uninitialised (for arrays filled right after, where
// zero-filling gigabytes single-threaded would cost seconds)
template <class T>
struct NoInitAlloc : std::allocator<T> {
  template <class U>
  struct rebind {
    using other = NoInitAlloc<U>;
  };
  NoInitAlloc() = default;
  template <class U>
  NoInitAlloc(const NoInitAlloc<U> &) noexcept {}
  template <class U>
  void construct(U *p) noexcept {
    ::new ((void *)p) U;
  }
  template <class U, class... Args>
  void construct(U *p, Args &&...args) {
    ::new ((void *)p) U(std::forward<Args>(args)...);
  }
};
template <class T>
using raw_vector = std::vector<T, NoInitAlloc<T>>;

struct HostCSR {
  int64_t n = 0;
  std::vector<int64_t> rowptr;
  raw_vector<int32_t> col;
  raw_vector<double> val;  // interleaved complex, 2 * nnz
  int64_t nnz() const { return (int64_t)col.size(); }
};
// A = K - (k^2 + i xi) M - i sign(xi) k M_b (impedance) or with PEC identity rows; with weight,
// the Gram matrix D_k = K + k^2 M of the k-weighted inner product instead (xi unused)
void assemble_global(const Mesh &m, double k, double xi, int bc, HostCSR &A, bool weight = false);
void rhs_gaussian(const Mesh &m, int bc, const double c[3], const double pol[3], double sigma,
                  double *f);

// ---- partition -----------------------------------------------------------------------------------
struct Partition {
  int px = 1, py = 1, pz = 1, layers = 0, nsub = 1;
  std::vector<int32_t> cuts[3];
  std::vector<int32_t> part0;                       // per tet
  std::vector<std::vector<int32_t>> tets;           // tets of each subdomain, ascending
  std::vector<std::vector<int32_t>> as_set, oras_set;  // local DOFs, ascending global ids
  std::vector<int32_t> owner;                       // per edge
  const std::vector<std::vector<int32_t>> &set(int kind) const {
    return kind == MX_ORAS ? oras_set : as_set;
  }
};
void build_partition(const Mesh &m, int px, int py, int pz, const int32_t *cx, const int32_t *cy,
                     const int32_t *cz, int layers, Partition &p);

// ---- local problems, ordering, block skyline -------------------------------------------------------
struct LocalCSR {  // a local matrix in local (sorted global id) numbering
  int64_t n = 0;
  std::vector<int64_t> rowptr;
  std::vector<int32_t> col;
  std::vector<double> val;  // interleaved complex
};
// AS/RAS minor of the global matrix (PEC-constrained rows/cols reduced to their diagonal);
// boundary[d] flags the degrees of freedom on the box boundary.
void local_minor(const uint8_t *boundary, const HostCSR &A, int bc, const std::vector<int32_t> &set,
                 LocalCSR &out, std::vector<int32_t> &g2l_scratch);
// ORAS local impedance problem on the tetrahedra `tets` (local DOFs `set`).
// Scratch: g2l_scratch[E] all -1 on entry and exit; tet_pos[T] any contents (caller-owned, -1
// initially), reusable across calls.
void local_impedance(const Mesh &m, const KuhnElements &ke, double k, double xi, int bc,
                     const std::vector<int32_t> &tets, const std::vector<int32_t> &set,
                     LocalCSR &out, std::vector<int32_t> &g2l_scratch, std::vector<int32_t> &tet_pos);
// ---- second-order Nedelec elements -----------------------------------------------------------------
// DOFs: E Whitney functions (edge ids), E edge gradients, then two per face (faces sorted by vertex
// triple).  Element integrals per Kuhn type p of a cube: K, M (20 x 20, local order 6 Whitney,
// 6 gradients, 2 per local face (1,2,3) (0,2,3) (0,1,3) (0,1,2)) and the tangential face masses B.
struct Order2 {
  int64_t E = 0, F = 0, N = 0;
  std::vector<int32_t> tet_face;      // [nt][4] face ids by local face
  std::vector<int32_t> face_vert;     // [F][3] ascending
  std::vector<int32_t> face_tet;      // [F][2] the tetrahedra on each side (-1: box boundary)
  std::vector<int8_t> face_lf;        // [F][2] local face index in those tetrahedra
  std::vector<uint8_t> dof_boundary;  // [N] tangential trace lives on the box boundary
  double K[6][20][20], M[6][20][20], B[6][4][20][20];
};
void build_order2(const Mesh &m, Order2 &o);
int32_t order2_dof(const Mesh &m, const Order2 &o, int64_t t, int a);
int32_t order2_face_of(const Order2 &o, const int32_t v[3]);  // -1 if not a face
// A = K - (k^2 + i xi) M - i sign(xi) k M_b of the order-2 space (PEC: identity rows and columns);
// with weight, the Gram matrix D_k = K + k^2 M instead (xi unused)
void assemble_order2(const Mesh &m, const Order2 &o, double k, double xi, int bc, HostCSR &A,
                     bool weight = false);
// order-2 local DOF sets (kind AS/RAS: Whitney and gradient functions of the lowest-order AS set
// and the faces whose tetrahedra are all in the subdomain; ORAS: every DOF of its tetrahedra),
// and the Boolean owner (least part0 of a tetrahedron holding the DOF)
void order2_sets(const Mesh &m, const Order2 &o, const Partition &p, int kind,
                 std::vector<std::vector<int32_t>> &sets, std::vector<int32_t> &owner);
// ORAS local impedance problem of the order-2 space; scratch as for local_impedance (g2l sized N)
void local_impedance2(const Mesh &m, const Order2 &o, double k, double xi, int bc,
                      const std::vector<int32_t> &tets, const std::vector<int32_t> &set,
                      LocalCSR &out, std::vector<int32_t> &g2l_scratch, std::vector<int32_t> &tet_pos);

// Reverse Cuthill-McKee of the pattern of `a` (perm[new] = old).
void rcm_order(const LocalCSR &a, std::vector<int32_t> &perm);

constexpr int TILE = 64;

struct Skyline {
  int64_t n = 0, nb = 0;              // rows, block rows
  std::vector<int32_t> perm, iperm;   // new -> old, old -> new
  std::vector<int32_t> first;         // envelope start per permuted row
  std::vector<int32_t> bfirst;        // first stored tile column per block row (monotone)
  std::vector<int32_t> blast;         // last block row storing a tile in block column K
  std::vector<int64_t> brow_off;      // tile offset (in tiles) of block row I, relative
  int64_t tiles = 0;
  int64_t env = 0;                    // exact lower envelope entries (diagonal included)
  double env_flops = 0, tile_flops = 0;
};
void build_skyline(const LocalCSR &a, Skyline &s);

}  // namespace mx
