"""Oracle: lowest-order Nedelec (Whitney) element matrices, Galerkin matrix and load vector.

Test infrastructure only (see oracle/__init__.py).

Sesquilinear form (eq:Helmholtzvf_intro) with the first-order impedance condition (eq:imp):
the boundary term follows from  int curl curl E . conj(v) = int curl E . curl conj(v)
+ int_dOmega (n x curl E) . conj(v)  and  n x curl E = -i sign(xi) k E_T, so

    a(E, v) = int curl E . curl conj(v) - (k^2 + i xi) int E . conj(v)
              - i sign(xi) k int_dOmega E_T . conj(v_T)

and the Galerkin matrix (A)_ij = a(w_j, w_i) (Sec. 2.2) is  A = K - (k^2 + i xi) M - i s k M_b
with s = sign(xi) (s = +1 when xi = 0, the outgoing choice for the e^{-i omega t} convention of
eq:new1).  With the PEC condition (eq:PECcond) the DOFs of boundary edges are fixed to zero: their
rows and columns are replaced by identity rows/columns, which keeps A complex symmetric.

Basis (Whitney): for the edge (a -> b) of a tetrahedron with barycentrics lambda,
w = lambda_a grad lambda_b - lambda_b grad lambda_a, curl w = 2 grad lambda_a x grad lambda_b.
Integrals of lambda products: int_T lambda_a lambda_b = |T| (1 + delta_ab) / 20 and on a
triangle int lambda_a lambda_b = |tau| (1 + delta_ab) / 12.
Load f_i = int F . w_i (F real here) with the 4-point degree-2 symmetric tetrahedron rule.
"""
import numpy as np
import scipy.sparse as sp

from .mesh import LOCAL_EDGES

BC_PEC = 0
BC_IMPEDANCE = 1


def tet_geometry(mesh, tets=None):
    """Barycentric gradients (T,4,3) and volumes (T,) of the tetrahedra."""
    tv = mesh.tet_vert if tets is None else mesh.tet_vert[tets]
    x = mesh.xyz[tv]  # (T,4,3)
    J = np.stack([x[:, 1] - x[:, 0], x[:, 2] - x[:, 0], x[:, 3] - x[:, 0]], axis=2)  # columns
    Jinv = np.linalg.inv(J)  # rows = grad lambda_1..3
    g = np.zeros((tv.shape[0], 4, 3))
    g[:, 1:, :] = Jinv
    g[:, 0, :] = -Jinv.sum(axis=1)
    vol = np.abs(np.linalg.det(J)) / 6.0
    return g, vol


def element_matrices(g, vol):
    """Stiffness K_T and mass M_T (T,6,6) in local edge orientation (a -> b)."""
    a, b = LOCAL_EDGES[:, 0], LOCAL_EDGES[:, 1]
    curl = 2.0 * np.cross(g[:, a, :], g[:, b, :])  # (T,6,3)
    K = vol[:, None, None] * np.einsum("tei,tfi->tef", curl, curl)
    GG = np.einsum("tai,tbi->tab", g, g)  # grad l_a . grad l_b  (T,4,4)
    lam = (np.ones((4, 4)) + np.eye(4)) / 20.0  # int l_a l_b / |T|
    M = np.zeros_like(K)
    for e in range(6):
        i, j = a[e], b[e]
        for f in range(6):
            k, l = a[f], b[f]
            M[:, e, f] = (lam[i, k] * GG[:, j, l] - lam[i, l] * GG[:, j, k]
                          - lam[j, k] * GG[:, i, l] + lam[j, l] * GG[:, i, k])
    M *= vol[:, None, None]
    return K, M


def face_mass(mesh, fverts):
    """Tangential Whitney mass on triangles given by vertex triples (F,3), local edge order
    (0,1) (0,2) (1,2), each oriented from the lower to the higher local vertex.  Returns (F,3,3)
    and the global edge ids and signs (F,3)."""
    x = mesh.xyz[fverts]  # (F,3,3)
    G = np.stack([x[:, 1] - x[:, 0], x[:, 2] - x[:, 0]], axis=2)  # (F,3,2)
    GtG = np.einsum("fia,fib->fab", G, G)
    Pinv = np.linalg.solve(GtG, np.transpose(G, (0, 2, 1)))  # (F,2,3) rows = surface grads l1,l2
    g = np.zeros((fverts.shape[0], 3, 3))
    g[:, 1:, :] = Pinv
    g[:, 0, :] = -Pinv.sum(axis=1)
    area = 0.5 * np.sqrt(np.linalg.det(GtG))
    GG = np.einsum("fai,fbi->fab", g, g)
    lam = (np.ones((3, 3)) + np.eye(3)) / 12.0
    le = [(0, 1), (0, 2), (1, 2)]
    Mb = np.zeros((fverts.shape[0], 3, 3))
    for e, (i, j) in enumerate(le):
        for f, (k, l) in enumerate(le):
            Mb[:, e, f] = (lam[i, k] * GG[:, j, l] - lam[i, l] * GG[:, j, k]
                           - lam[j, k] * GG[:, i, l] + lam[j, l] * GG[:, i, k])
    Mb *= area[:, None, None]
    lo = np.stack([fverts[:, i] for i, _ in le], axis=1)
    hi = np.stack([fverts[:, j] for _, j in le], axis=1)
    eid = mesh.edge_index(np.minimum(lo, hi).ravel(), np.maximum(lo, hi).ravel()).reshape(-1, 3)
    sign = np.where(lo < hi, 1.0, -1.0)
    return Mb, eid, sign


def _scatter(rows, cols, vals, n):
    return sp.coo_matrix((vals.ravel(), (rows.ravel(), cols.ravel())), shape=(n, n)).tocsr()


def assemble_parts(mesh, tets=None, bfaces=None):
    """Global (or tetrahedron-subset) K, M and boundary mass M_b as real CSR matrices.

    tets: indices of tetrahedra to assemble over (default: all).
    bfaces: (F,3) vertex triples of the impedance faces (default: the boundary of the box)."""
    E = mesh.n_edge
    g, vol = tet_geometry(mesh, tets)
    K, M = element_matrices(g, vol)
    te = mesh.tet_edge if tets is None else mesh.tet_edge[tets]
    ts = (mesh.tet_edge_sign if tets is None else mesh.tet_edge_sign[tets]).astype(np.float64)
    S = ts[:, :, None] * ts[:, None, :]
    rows = np.repeat(te[:, :, None], 6, axis=2)
    cols = np.repeat(te[:, None, :], 6, axis=1)
    Kg = _scatter(rows, cols, K * S, E)
    Mg = _scatter(rows, cols, M * S, E)
    if bfaces is None:
        bfaces = mesh.bface_vert
    if len(bfaces):
        Mb, eid, sgn = face_mass(mesh, bfaces)
        Sb = sgn[:, :, None] * sgn[:, None, :]
        rb = np.repeat(eid[:, :, None], 3, axis=2)
        cb = np.repeat(eid[:, None, :], 3, axis=1)
        Bg = _scatter(rb, cb, Mb * Sb, E)
    else:
        Bg = sp.csr_matrix((E, E))
    return Kg, Mg, Bg


def impedance_sign(xi):
    return 1.0 if xi >= 0 else -1.0


def combine(K, M, Mb, k, xi, bc, pec_mask=None):
    """A = K - (k^2 + i xi) M - i sign(xi) k M_b  (impedance) or K - (k^2 + i xi) M with
    identity rows/columns on the PEC-constrained edges."""
    A = (K.astype(np.complex128) - (k * k + 1j * xi) * M)
    if bc == BC_IMPEDANCE:
        A = A - 1j * impedance_sign(xi) * k * Mb
    A = A.tocsr()
    if bc == BC_PEC and pec_mask is not None and pec_mask.any():
        keep = sp.diags((~pec_mask).astype(np.float64))
        A = (keep @ A @ keep + sp.diags(pec_mask.astype(np.float64))).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    return A


def assemble(mesh, k, xi, bc=BC_IMPEDANCE):
    """Global Galerkin matrix A_xi (complex CSR, Sec. 2.2)."""
    K, M, Mb = assemble_parts(mesh)
    pec = mesh.boundary_edge_mask() if bc == BC_PEC else None
    return combine(K, M, Mb, k, xi, bc, pec)


def weight_matrix(mesh, k, bc=BC_IMPEDANCE):
    """D_k of eq:ip: the Gram matrix of the wavenumber-weighted inner product of eq:weight,
    (v, w)_{curl,k} = (curl v, curl w) + k^2 (v, w), in the Whitney basis, i.e. D = K + k^2 M
    (real symmetric positive definite; the boundary term of the impedance form is not part of
    it).  With the PEC condition the constrained boundary edges get identity rows and columns,
    as in the Galerkin matrix, so D stays positive definite on the full DOF vector and the
    constrained DOFs do not enter the norm of the free ones."""
    K, M, _ = assemble_parts(mesh, bfaces=np.zeros((0, 3), dtype=np.int64))
    D = (K + (k * k) * M).tocsr()
    if bc == BC_PEC:
        pec = mesh.boundary_edge_mask()
        if pec.any():
            keep = sp.diags((~pec).astype(np.float64))
            D = (keep @ D @ keep + sp.diags(pec.astype(np.float64))).tocsr()
    D.sum_duplicates()
    D.sort_indices()
    return D


def sparsity_pattern(mesh, tets=None):
    """Structural pattern: edge pairs sharing a tetrahedron (of the given subset)."""
    E = mesh.n_edge
    te = mesh.tet_edge if tets is None else mesh.tet_edge[tets]
    rows = np.repeat(te[:, :, None], 6, axis=2)
    cols = np.repeat(te[:, None, :], 6, axis=1)
    P = sp.coo_matrix((np.ones(rows.size), (rows.ravel(), cols.ravel())), shape=(E, E)).tocsr()
    P.sum_duplicates()
    P.sort_indices()
    P.data[:] = 1.0
    return P


# 4-point degree-2 rule on the tetrahedron (Hammer-Marlowe-Stroud): barycentrics
# (alpha, beta, beta, beta) and permutations, weight |T|/4 each.
_Q_ALPHA = (5.0 + 3.0 * np.sqrt(5.0)) / 20.0
_Q_BETA = (5.0 - np.sqrt(5.0)) / 20.0


def quad_points():
    P = np.full((4, 4), _Q_BETA)
    np.fill_diagonal(P, _Q_ALPHA)
    return P  # row q = barycentric coordinates of point q


def load_vector(mesh, F, bc=BC_IMPEDANCE):
    """f_e = int F . w_e  (Sec. 2.2), F: callable (N,3) -> (N,3) real or complex."""
    g, vol = tet_geometry(mesh)
    x = mesh.xyz[mesh.tet_vert]  # (T,4,3)
    P = quad_points()
    f = np.zeros(mesh.n_edge, dtype=np.complex128)
    a, b = LOCAL_EDGES[:, 0], LOCAL_EDGES[:, 1]
    loc = np.zeros((mesh.n_tet, 6), dtype=np.complex128)
    for q in range(4):
        lam = P[q]
        xq = np.einsum("a,tai->ti", lam, x)
        Fq = np.asarray(F(xq))
        w = lam[a][None, :, None] * g[:, b, :] - lam[b][None, :, None] * g[:, a, :]  # (T,6,3)
        loc += (vol / 4.0)[:, None] * np.einsum("tei,ti->te", w, Fq)
    loc *= mesh.tet_edge_sign
    np.add.at(f, mesh.tet_edge.ravel(), loc.ravel())
    if bc == BC_PEC:
        f[mesh.boundary_edge_mask()] = 0.0
    return f


def gaussian_source(center, pol, sigma):
    """F(x) = pol * exp(-|x - c|^2 / (2 sigma^2)) (the Gaussian stand-in for the point source of
    Sec. 6.1)."""
    c = np.asarray(center, dtype=np.float64)
    p = np.asarray(pol, dtype=np.float64)

    def F(x):
        r2 = ((x - c) ** 2).sum(axis=1)
        return np.exp(-r2 / (2.0 * sigma * sigma))[:, None] * p[None, :]
    return F


def interpolate(mesh, Efun):
    """Edge DOFs psi_e(E) = int_e E . t, t = x_hi - x_lo (unnormalised tangent), with 5-point
    Gauss-Legendre along each edge."""
    xa = mesh.xyz[mesh.edge_vert[:, 0]]
    xb = mesh.xyz[mesh.edge_vert[:, 1]]
    t = xb - xa
    s, w = np.polynomial.legendre.leggauss(5)
    s = 0.5 * (s + 1.0)
    w = 0.5 * w
    out = np.zeros(mesh.n_edge, dtype=np.complex128)
    for sq, wq in zip(s, w):
        xq = xa + sq * t
        out += wq * (np.asarray(Efun(xq)) * t).sum(axis=1)
    return out
