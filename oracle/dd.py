"""Oracle: overlapping subdomains, restrictions, partition of unity and the one-level Schwarz
preconditioners AS, RAS and ORAS (ImpRAS).

Test infrastructure only (see oracle/__init__.py).

* Non-overlapping partition (Sec. 6.1, "by hand" for a structured mesh): boxes of cubes cut at
  the planes cx, cy, cz; part0(tet) = bx + px*(by + py*bz) of the box holding its cube.
* Overlap (Sec. 6.1): Omega^{p+1} = Omega^p plus every tetrahedron touching it; "touching" is
  read as sharing at least one vertex.  `layers` sweeps from part0.
* AS / RAS local DOF set (Sec. 3.1, eq:restriction1): DOFs whose support lies in Omega_l, read as
  "every tetrahedron containing the edge lies in Omega_l"; the minor R A R^T (eq:minor) is then
  the Galerkin matrix of the PEC local problem.
* ORAS (ImpRAS, Sec. 6.3): all edges of tetrahedra of Omega_l, local matrix assembled on Omega_l
  with the impedance term - i sign(xi) k M_b on the faces of dOmega_l (same coefficient k on the
  interface faces as on the boundary of the box); on dOmega_l that lies on the box boundary the
  global boundary condition is kept.
* Partition of unity (eq:algebPartUnity): Boolean owner, owner(e) = min part0 over the
  tetrahedra containing e, D^l_ee = [owner(e) = l]; sum_l R^T D R = I holds exactly.
* Preconditioners: AS = sum_l R^T (A^l)^-1 R (eq:defAS without the coarse term, Sec. 6.2),
  RAS = sum_l R^T D^l (A^l)^-1 R (one-level RAS, Sec. 6.3), ORAS = RAS with impedance local
  matrices.  Local solves are exact sparse LU (SuperLU, factor_local), independent of the
  ordering and factorisation the library uses.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from threadpoolctl import threadpool_limits

from . import fem

AS, RAS, ORAS = 0, 1, 2


def even_cuts(n, p):
    return [(i * n) // p for i in range(p + 1)]


class Partition:
    def __init__(self, mesh, px, py, pz, layers, cx=None, cy=None, cz=None):
        nx, ny, nz = mesh.n
        self.mesh = mesh
        self.p = (px, py, pz)
        self.layers = layers
        self.cuts = [np.asarray(c if c is not None else even_cuts(n, p), dtype=np.int64)
                     for c, n, p in ((cx, nx, px), (cy, ny, py), (cz, nz, pz))]
        for c, n, p in zip(self.cuts, (nx, ny, nz), (px, py, pz)):
            assert len(c) == p + 1 and c[0] == 0 and c[-1] == n and np.all(np.diff(c) > 0)
        ijk = mesh.cube_ijk[mesh.tet_cube]
        b = [np.searchsorted(self.cuts[a], ijk[:, a], side="right") - 1 for a in range(3)]
        self.part0 = b[0] + px * (b[1] + py * b[2])
        self.N = px * py * pz
        T, E = mesh.n_tet, mesh.n_edge
        self.tet_masks = []
        for l in range(self.N):
            m = self.part0 == l
            for _ in range(layers):
                vm = np.zeros(mesh.n_vert, dtype=bool)
                vm[mesh.tet_vert[m].ravel()] = True
                m = vm[mesh.tet_vert].any(axis=1)
            self.tet_masks.append(m)
        cnt_all = np.bincount(mesh.tet_edge.ravel(), minlength=E)
        self.as_sets, self.oras_sets = [], []
        for m in self.tet_masks:
            cnt = np.bincount(mesh.tet_edge[m].ravel(), minlength=E)
            self.oras_sets.append(np.nonzero(cnt > 0)[0])
            self.as_sets.append(np.nonzero((cnt == cnt_all) & (cnt_all > 0))[0])
        owner = np.full(E, self.N, dtype=np.int64)
        np.minimum.at(owner, mesh.tet_edge.ravel(), np.repeat(self.part0, 6))
        self.owner = owner

    def local_set(self, kind):
        return self.oras_sets if kind == ORAS else self.as_sets

    def restriction(self, l, kind):
        idx = self.local_set(kind)[l]
        E = self.mesh.n_edge
        return sp.csr_matrix((np.ones(len(idx)), (np.arange(len(idx)), idx)), shape=(len(idx), E))

    def pou(self, l, kind):
        """Diagonal of D^l (Boolean owner) on the local DOFs."""
        idx = self.local_set(kind)[l]
        return (self.owner[idx] == l).astype(np.float64)

    def subdomain_boundary_faces(self, l):
        """Vertex triples of the faces of dOmega_l (faces of its tetrahedra not shared by two of
        them)."""
        mesh = self.mesh
        m = self.tet_masks[l]
        fid = mesh.tet_face[m].ravel()
        u, c = np.unique(fid, return_counts=True)
        keys = mesh.face_key[u[c == 1]]
        nv = mesh.n_vert
        return np.stack([keys // (nv * nv), (keys // nv) % nv, keys % nv], axis=1)

    def neighbours(self, l):
        """Lambda(l) of eq:finoverlap: subdomains whose tetrahedron sets meet Omega_l."""
        return [j for j in range(self.N) if j != l and (self.tet_masks[l] & self.tet_masks[j]).any()]


def sub_box(n, lengths, parts, layers, cuts, l):
    """The ORAS local problem of box l of a large jittered-box partition, on a small mesh.  Its
    overlapped subdomain reaches only `layers` cubes past the box (each sweep adds tetrahedra
    sharing a vertex, hence at most one more cube per axis), and on its boundary the local matrix
    has the impedance term with coefficient k whether the boundary lies on the box of the whole
    domain (eq:imp) or inside it (ImpRAS, Sec. 6.3).  So the sub-box of cubes [rlo, rhi) (box l
    extended by `layers` per side, clipped to the domain), cut at l's planes, holds the same
    local problem with impedance boundary conditions (up to numbering; sub-box vertex ijk + rlo
    is the whole mesh's).  Returns (sub-box mesh, its Partition, index of l in it, l's cube range
    lo / hi and the sub-box origin rlo, in cubes of the whole mesh)."""
    from .mesh import Mesh
    px, py, _ = parts
    b = (l % px, (l // px) % py, l // (px * py))
    lo = [int(cuts[a][b[a]]) for a in range(3)]
    hi = [int(cuts[a][b[a] + 1]) for a in range(3)]
    rlo = [max(0, lo[a] - layers) for a in range(3)]
    rhi = [min(n[a], hi[a] + layers) for a in range(3)]
    sc, pos = [], []
    for a in range(3):
        c = sorted({0, lo[a] - rlo[a], hi[a] - rlo[a], rhi[a] - rlo[a]})
        sc.append(c)
        pos.append(c.index(lo[a] - rlo[a]))
    ns = [rhi[a] - rlo[a] for a in range(3)]
    m = Mesh(*ns, *[ns[a] * lengths[a] / n[a] for a in range(3)])
    part = Partition(m, len(sc[0]) - 1, len(sc[1]) - 1, len(sc[2]) - 1, layers, *sc)
    lr = pos[0] + (len(sc[0]) - 1) * (pos[1] + (len(sc[1]) - 1) * pos[2])
    return m, part, lr, lo, hi, rlo


def local_pattern(part, l, kind, bc=fem.BC_IMPEDANCE):
    """Structural pattern of A^l: local DOF pairs sharing a tetrahedron of Omega_l; with the PEC
    condition the constrained boundary edges keep only their diagonal."""
    mesh = part.mesh
    idx = part.local_set(kind)[l]
    tets = np.nonzero(part.tet_masks[l])[0]
    P = fem.sparsity_pattern(mesh, tets)[idx][:, idx].tocsr()
    if bc == fem.BC_PEC:
        pec = mesh.boundary_edge_mask()[idx].astype(np.float64)
        keep = sp.diags(1.0 - pec)
        P = (keep @ P @ keep + sp.diags(pec)).tocsr()
        P.eliminate_zeros()
    P.sort_indices()
    return P


def local_matrix(part, A, kind, k, xi, l, bc=fem.BC_IMPEDANCE):
    """A^l of subdomain l: the minor of A (AS, RAS; eq:minor) or the impedance local problem
    assembled on the tetrahedra of Omega_l (ORAS = ImpRAS, Sec. 6.3)."""
    mesh = part.mesh
    if kind in (AS, RAS):
        idx = part.as_sets[l]
        return A[idx][:, idx].tocsc()
    idx = part.oras_sets[l]
    tets = np.nonzero(part.tet_masks[l])[0]
    faces = part.subdomain_boundary_faces(l)
    if bc == fem.BC_PEC:  # PEC faces of the box keep PEC, only interface faces get impedance
        gb = set(map(tuple, mesh.bface_vert))
        faces = np.array([f for f in faces if tuple(f) not in gb]).reshape(-1, 3)
    K, M, Mb = fem.assemble_parts(mesh, tets, faces)
    Al = (K.astype(np.complex128) - (k * k + 1j * xi) * M
          - 1j * fem.impedance_sign(xi) * k * Mb).tocsr()
    if bc == fem.BC_PEC:
        pec = mesh.boundary_edge_mask()
        if pec.any():
            keep = sp.diags((~pec).astype(np.float64))
            Al = (keep @ Al @ keep + sp.diags(pec.astype(np.float64))).tocsr()
    return Al[idx][:, idx].tocsc()


def factor_local(Al):
    """Exact sparse LU of a local matrix (SuperLU).  Fill-reducing minimum-degree order on the
    pattern of A^l + (A^l)^T, applied symmetrically, with diagonal pivots: A^l is complex
    symmetric, and every principal submatrix of it is nonsingular for xi != 0 by the coercivity
    estimate of Sec. 2.3 (eq:coercivity), applied to the local problems as in Sec. 3.3, so no
    row interchange is needed; a vanishing pivot raises instead of returning a wrong factor.
    The order only changes rounding.  BLAS runs on one thread (here and in the local solves), so
    the rounding does not depend on the host's core count."""
    with threadpool_limits(1):
        return spla.splu(Al, permc_spec="MMD_AT_PLUS_A", diag_pivot_thresh=0.0,
                         options=dict(SymmetricMode=True))


def local_matrices(part, A, kind, k, xi, bc=fem.BC_IMPEDANCE):
    """A^l for every subdomain: minors of A (AS, RAS) or impedance local problems (ORAS)."""
    return [local_matrix(part, A, kind, k, xi, l, bc) for l in range(part.N)]


class Schwarz:
    """One-level Schwarz preconditioner z = sum_l R^T D^l (A^l)^-1 R v (D^l = I for AS)."""

    def __init__(self, part, A, kind, k, xi, bc=fem.BC_IMPEDANCE, local=None):
        self.part, self.kind = part, kind
        self.sets = part.local_set(kind)
        self.local = local if local is not None else local_matrices(part, A, kind, k, xi, bc)
        self.lu = [factor_local(Al) for Al in self.local]
        self.D = [part.pou(l, kind) if kind in (RAS, ORAS) else None for l in range(part.N)]
        self.n = A.shape[0]

    def local_solve(self, l, r):
        with threadpool_limits(1):
            return self.lu[l].solve(r)

    def apply(self, v):
        z = np.zeros(self.n, dtype=np.complex128)
        for l, idx in enumerate(self.sets):
            x = self.local_solve(l, v[idx])
            if self.D[l] is not None:
                x = self.D[l] * x
            np.add.at(z, idx, x)
        return z

    __call__ = apply


def dense_schwarz(part, A, kind, k, xi, bc=fem.BC_IMPEDANCE):
    """Brute-force dense B^-1 = sum_l R^T D (A^l)^-1 R with explicit inverses (tiny meshes)."""
    loc = local_matrices(part, A, kind, k, xi, bc)
    n = A.shape[0]
    B = np.zeros((n, n), dtype=np.complex128)
    for l, idx in enumerate(part.local_set(kind)):
        inv = np.linalg.inv(loc[l].toarray())
        if kind in (RAS, ORAS):
            inv = part.pou(l, kind)[:, None] * inv
        B[np.ix_(idx, idx)] += inv
    return B
