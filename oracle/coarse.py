"""Oracle: the coarse space and the two-level Schwarz preconditioners.

Test infrastructure only (see oracle/__init__.py).

* Coarse mesh (Sec. 3.2): a box mesh of the same domain with nx/r x ny/r x nz/r cubes (one ratio
  r for all axes), split the same way; or any coarse box mesh (Sec. 6.1 also uses coarse meshes
  that are not nested), with R^0 by a Gauss rule along each fine edge
  (restriction_quadrature).  Every coarse tetrahedron is then a union of fine ones (the
  planes bounding a coarse tetrahedron, x_i/H_i = const and x_i/H_i - x_j/H_j = const at integers,
  are planes of the fine split when H_i = r h_i), so the meshes are nested as the theory
  assumes.
* Coarse basis: the lowest-order Whitney functions w^H_p of the coarse edges.  The paper takes
  those with zero tangential trace on the boundary (the PEC setting of its theory); with the
  impedance condition every coarse edge is kept (reading: the coarse space is the edge-element
  space of the coarse mesh under the same boundary condition as the fine problem).
* Restriction (eq:restriction): (R^0)_{pj} = psi^h_j(w^H_p), the fine degree of freedom j (line
  integral along fine edge j, oriented lo -> hi, with the unnormalised tangent) of the coarse
  basis function p.  Inside one coarse tetrahedron w^H_p is affine, so the line integral equals
  w^H_p(midpoint) . t exactly; the coarse tetrahedron holding the midpoint is found by its
  barycentric coordinates (any one of several, on a shared face, gives the same tangential
  value).
* Coarse matrix (eq:minor with l = 0): A^0 = R^0 A (R^0)^T.
* Coarse correction G = (R^0)^T (A^0)^{-1} R^0 and, for a one-level preconditioner B1 (AS, RAS or
  ImpRAS = ORAS of dd.Schwarz):
    additive (eq:defAS, eq:RAS2):        B = B1 + G
    hybrid / BNN (eq:HRAS):              B = (I - G A) B1 (I - A G) + G
    adapted deflation (eq:ADEF1ras):     B = B1 (I - A G) + G
  A is the matrix the preconditioner is built for (A at xi_prec).
"""
import numpy as np
import scipy.sparse as sp

from . import dd, fem
from .mesh import LOCAL_EDGES, Mesh

ADDITIVE, HYBRID, DEFLATION = "additive", "hybrid", "deflation"


def coarse_mesh(fine, ratio):
    """The box of `fine` with `ratio` times fewer cubes along every axis.  The ratio must divide
    every cube count and be the same on all axes: the planes x_i/h_i - x_j/h_j = const of the
    split are shared by both meshes only when H_i/h_i is the same for every axis."""
    ratio = int(ratio)
    for n in fine.n:
        assert n % ratio == 0, "coarse mesh must be nested: cube counts must be divisible"
    return Mesh(*(n // ratio for n in fine.n), *fine.L)


def coarse_dofs(coarse, bc=fem.BC_IMPEDANCE):
    """Coarse edges carrying a basis function: all of them (impedance) or those not on the
    boundary (PEC, zero tangential trace)."""
    if bc == fem.BC_PEC:
        return np.nonzero(~coarse.boundary_edge_mask())[0]
    return np.arange(coarse.n_edge)


def restriction(fine, coarse, bc=fem.BC_IMPEDANCE):
    """R^0 (n_coarse_dofs x E) of eq:restriction, entry by entry: for fine edge j with midpoint
    m and tangent t, the coarse tetrahedron T holding m (barycentric coordinates of m in T, from
    the barycentric gradients, all >= 0), and (R^0)_{pj} = sign * w^H_p(m) . t for the six edges
    p of T."""
    g, _ = fem.tet_geometry(coarse)  # (Tc,4,3) barycentric gradients of every coarse tetrahedron
    H = np.array(coarse.L) / np.array(coarse.n)
    nc = np.array(coarse.n)
    keep = coarse_dofs(coarse, bc)
    row_of = np.full(coarse.n_edge, -1)
    row_of[keep] = np.arange(len(keep))
    xa = fine.xyz[fine.edge_vert[:, 0]]
    xb = fine.xyz[fine.edge_vert[:, 1]]
    t = xb - xa
    mid = 0.5 * (xa + xb)
    ijk = np.minimum((mid / H).astype(np.int64), nc - 1)
    cube = ijk[:, 0] + nc[0] * (ijk[:, 1] + nc[1] * ijk[:, 2])
    E = fine.n_edge
    tet = np.full(E, -1)
    lam = np.zeros((E, 4))
    for q in range(6):  # the six tetrahedra of the coarse cube, first one holding the midpoint
        cand = 6 * cube + q
        X0 = coarse.xyz[coarse.tet_vert[cand, 0]]
        l = np.einsum("eai,ei->ea", g[cand], mid - X0)
        l[:, 0] += 1.0
        take = (tet < 0) & (l.min(axis=1) >= -1e-12)
        tet[take] = cand[take]
        lam[take] = l[take]
    assert np.all(tet >= 0), "fine edge midpoint outside its coarse cube"
    rows, cols, vals = [], [], []
    for le, (a, b) in enumerate(LOCAL_EDGES):
        p = coarse.tet_edge[tet, le]
        w = lam[:, a, None] * g[tet, b] - lam[:, b, None] * g[tet, a]  # Whitney function a -> b
        v = coarse.tet_edge_sign[tet, le] * np.einsum("ei,ei->e", w, t)
        ok = (row_of[p] >= 0) & (v != 0.0)
        rows.append(row_of[p][ok])
        cols.append(np.nonzero(ok)[0])
        vals.append(v[ok])
    R = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(len(keep), E))
    R.sum_duplicates()
    R.sort_indices()
    return R


class TwoLevel:
    """Two-level Schwarz preconditioner: one-level B1 (a dd.Schwarz, or anything callable built
    for the matrix A) combined with the coarse correction G by `combine`."""

    def __init__(self, B1, A, R0, combine=ADDITIVE):
        self.B1, self.A, self.R0, self.combine = B1, A, R0.tocsr(), combine
        self.A0 = (self.R0 @ A @ self.R0.T).tocsc()
        self.lu0 = dd.factor_local(self.A0)
        self.n = A.shape[0]

    def coarse(self, v):
        """G v = (R^0)^T (A^0)^{-1} R^0 v."""
        from threadpoolctl import threadpool_limits
        with threadpool_limits(1):
            return self.R0.T @ self.lu0.solve(self.R0 @ v)

    def apply(self, v):
        v = np.asarray(v, dtype=np.complex128)
        Gv = self.coarse(v)
        if self.combine == ADDITIVE:
            return self.B1(v) + Gv
        t = v - self.A @ Gv                      # (I - A G) v
        s = self.B1(t)
        if self.combine == DEFLATION:
            return s + Gv
        return s - self.coarse(self.A @ s) + Gv  # (I - G A) s + G v

    __call__ = apply


def coarse_box_mesh(fine, cn):
    """A coarse box mesh of the same domain with cn = (cnx, cny, cnz) cubes, nested or not."""
    return Mesh(*(int(c) for c in cn), *fine.L)


def restriction_quadrature(fine, coarse, bc=fem.BC_IMPEDANCE, nq=12):
    """R^0 of eq:restriction for a coarse mesh that need not be nested (Sec. 6.1): the fine DOF
    (line integral along fine edge j, tangent x_hi - x_lo) of coarse basis function p by the
    nq-point Gauss-Legendre rule on the edge: (R^0)_pj = sum_q w_q w^H_p(x_q) . t, with x_q
    located in the coarse mesh by barycentric coordinates (the first of its cube's six
    tetrahedra holding it).  On a nested mesh the integrand is affine along each fine edge and
    this equals restriction() up to rounding."""
    g, _ = fem.tet_geometry(coarse)
    H = np.array(coarse.L) / np.array(coarse.n)
    nc = np.array(coarse.n)
    keep = coarse_dofs(coarse, bc)
    row_of = np.full(coarse.n_edge, -1)
    row_of[keep] = np.arange(len(keep))
    s, w = np.polynomial.legendre.leggauss(nq)
    s, w = 0.5 * (s + 1.0), 0.5 * w
    xa = fine.xyz[fine.edge_vert[:, 0]]
    t = fine.xyz[fine.edge_vert[:, 1]] - xa
    E = fine.n_edge
    rows, cols, vals = [], [], []
    for sq, wq in zip(s, w):
        x = xa + sq * t
        ijk = np.clip(np.floor(x / H).astype(np.int64), 0, nc - 1)
        cube = ijk[:, 0] + nc[0] * (ijk[:, 1] + nc[1] * ijk[:, 2])
        tet = np.full(E, -1)
        lam = np.zeros((E, 4))
        for q in range(6):
            cand = 6 * cube + q
            X0 = coarse.xyz[coarse.tet_vert[cand, 0]]
            l = np.einsum("eai,ei->ea", g[cand], x - X0)
            l[:, 0] += 1.0
            take = (tet < 0) & (l.min(axis=1) >= -1e-12)
            tet[take] = cand[take]
            lam[take] = l[take]
        assert np.all(tet >= 0), "quadrature point outside its coarse cube"
        for le, (a, b) in enumerate(LOCAL_EDGES):
            p = coarse.tet_edge[tet, le]
            wv = lam[:, a, None] * g[tet, b] - lam[:, b, None] * g[tet, a]
            v = wq * coarse.tet_edge_sign[tet, le] * np.einsum("ei,ei->e", wv, t)
            ok = row_of[p] >= 0
            rows.append(row_of[p][ok])
            cols.append(np.nonzero(ok)[0])
            vals.append(v[ok])
    R = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(len(keep), E))
    R.sum_duplicates()
    R.eliminate_zeros()
    R.sort_indices()
    return R
