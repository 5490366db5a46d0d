"""Oracle: structured tetrahedral box mesh and lowest-order edge numbering.

Test infrastructure only (see oracle/__init__.py).

The paper's experiments use FreeFem++ meshes of the unit cube (Sec. 6.1) made of conforming
tetrahedra (Sec. 2.2).  The split of a cube into tetrahedra is not stated; this oracle uses the
Kuhn (Freudenthal) split: the tetrahedron of permutation s of the axes is the monotone path
o -> o+e_s0 -> o+e_s0+e_s1 -> o+(1,1,1).  Numbering readings:

* vertex (i, j, k)    -> i + (nx+1) * (j + (ny+1) * k)
* cube (ci, cj, ck)   -> ci + nx * (cj + ny * ck); tetrahedron = 6 * cube + permutation rank,
                         permutations in lexicographic order 012, 021, 102, 120, 201, 210
* edges               -> all distinct vertex pairs of the tetrahedra, oriented from the lower to
                         the higher vertex id and sorted lexicographically by (lo, hi)
* local edges of a tet-> (0,1) (0,2) (0,3) (1,2) (1,3) (2,3) in its local vertex order

The degree of freedom of edge e is the line integral of the tangential component along the
edge oriented lo -> hi (the lowest-order case of the duality psi_i(w_j) = delta_ij, Sec. 2.2).
This module derives the edge list generically (sort and unique), not from the closed form
that the library uses, so the two can be compared bit for bit.
"""
from itertools import permutations

import numpy as np

LOCAL_EDGES = np.array([(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)], dtype=np.int64)
LOCAL_FACES = np.array([(1, 2, 3), (0, 2, 3), (0, 1, 3), (0, 1, 2)], dtype=np.int64)
PERMS = list(permutations(range(3)))  # lexicographic: 012 021 102 120 201 210


class Mesh:
    """Box [0,lx]x[0,ly]x[0,lz] split into nx*ny*nz cubes of 6 tetrahedra each."""

    def __init__(self, nx, ny, nz, lx=1.0, ly=1.0, lz=1.0):
        self.n = (int(nx), int(ny), int(nz))
        self.L = (float(lx), float(ly), float(lz))
        nx, ny, nz = self.n
        ii, jj, kk = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), np.arange(nz + 1),
                                 indexing="ij")
        vid = lambda i, j, k: i + (nx + 1) * (j + (ny + 1) * k)
        nv = (nx + 1) * (ny + 1) * (nz + 1)
        xyz = np.zeros((nv, 3))
        ids = vid(ii, jj, kk).ravel()
        xyz[ids, 0] = ii.ravel() * (lx / nx)
        xyz[ids, 1] = jj.ravel() * (ly / ny)
        xyz[ids, 2] = kk.ravel() * (lz / nz)
        self.xyz = xyz
        # tetrahedra
        ci, cj, ck = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
        cube = (ci + nx * (cj + ny * ck)).ravel()
        order = np.argsort(cube, kind="stable")
        ci, cj, ck = ci.ravel()[order], cj.ravel()[order], ck.ravel()[order]
        ncube = nx * ny * nz
        tv = np.zeros((ncube, 6, 4), dtype=np.int64)
        for p, s in enumerate(PERMS):
            pos = np.stack([ci, cj, ck], axis=1).copy()
            tv[:, p, 0] = vid(pos[:, 0], pos[:, 1], pos[:, 2])
            for step in range(3):
                pos[:, s[step]] += 1
                tv[:, p, step + 1] = vid(pos[:, 0], pos[:, 1], pos[:, 2])
        self.tet_vert = tv.reshape(-1, 4)
        self.tet_cube = np.repeat(np.arange(ncube), 6)
        self.cube_ijk = np.stack([ci, cj, ck], axis=1)
        self._edges()
        self._faces()

    @property
    def n_vert(self):
        return self.xyz.shape[0]

    @property
    def n_tet(self):
        return self.tet_vert.shape[0]

    @property
    def n_edge(self):
        return self.edge_vert.shape[0]

    def _edges(self):
        tv = self.tet_vert
        a = tv[:, LOCAL_EDGES[:, 0]]
        b = tv[:, LOCAL_EDGES[:, 1]]
        lo, hi = np.minimum(a, b), np.maximum(a, b)
        nv = self.n_vert
        key = lo * nv + hi
        uniq, inv = np.unique(key.ravel(), return_inverse=True)
        self.edge_vert = np.stack([uniq // nv, uniq % nv], axis=1)
        self.tet_edge = inv.reshape(-1, 6)
        self.tet_edge_sign = np.where(a < b, 1, -1).astype(np.int8)

    def _faces(self):
        tv = self.tet_vert
        f = np.sort(tv[:, LOCAL_FACES], axis=2)  # (T,4,3)
        nv = self.n_vert
        key = (f[..., 0] * nv + f[..., 1]) * nv + f[..., 2]
        uniq, inv, cnt = np.unique(key.ravel(), return_inverse=True, return_counts=True)
        self.face_key = uniq
        self.tet_face = inv.reshape(-1, 4)
        self.face_count = cnt
        bkeys = uniq[cnt == 1]
        self.bface_vert = np.stack([bkeys // (nv * nv), (bkeys // nv) % nv, bkeys % nv], axis=1)

    def boundary_edge_mask(self):
        """Edges lying on the boundary of the box (edges of boundary triangles)."""
        m = np.zeros(self.n_edge, dtype=bool)
        nv = self.n_vert
        keys = self.edge_vert[:, 0] * nv + self.edge_vert[:, 1]
        bf = self.bface_vert
        for a, b in ((0, 1), (0, 2), (1, 2)):
            k = bf[:, a] * nv + bf[:, b]
            idx = np.searchsorted(keys, k)
            m[idx] = True
        return m

    def edge_index(self, lo, hi):
        nv = self.n_vert
        keys = self.edge_vert[:, 0] * nv + self.edge_vert[:, 1]
        k = np.asarray(lo) * nv + np.asarray(hi)
        idx = np.searchsorted(keys, k)
        assert np.all(keys[idx] == k)
        return idx


def gradient_matrix(mesh):
    """Signed edge-vertex incidence G (E x V): (G phi)_e = phi(hi) - phi(lo).

    For a P1 function phi, G phi are the edge DOFs of grad phi, which lies in the lowest-order
    Nedelec space (gradients of the scalar space belong to Q_h, Sec. 3.4)."""
    import scipy.sparse as sp
    E = mesh.n_edge
    rows = np.repeat(np.arange(E), 2)
    cols = mesh.edge_vert.ravel()
    vals = np.tile([-1.0, 1.0], E)
    return sp.csr_matrix((vals, (rows, cols)), shape=(E, mesh.n_vert))
