"""Oracle: second-order Nedelec (first family) edge elements.

Test infrastructure only (see oracle/__init__.py).

The paper's order-2 experiments (Sec. 6.1, Tables tab:theoryDeltamin and tab:6bis) use the
Nedelec space of order 2 with the degrees of freedom of BoRa:17, which are not given in the
paper.  The space itself is fixed (Sec. 2.2: curl-conforming Nedelec elements of order m), and
the Galerkin solution does not depend on the basis; this oracle uses a hierarchical basis of the
same space (20 functions per tetrahedron, two per edge and two per face), with every function
defined from the global vertex numbering so that tangential traces match across faces:

* edge (i -> j), i < j:   w_ij = l_i grad l_j - l_j grad l_i   (the lowest-order Whitney function)
                          g_ij = l_i grad l_j + l_j grad l_i   (= grad(l_i l_j))
* face (i, j, k), i<j<k:  f1 = l_k w_ij,   f2 = l_j w_ik

with l the barycentric coordinates.  Global numbering: the E Whitney functions first (in the
lowest-order edge numbering, so the lowest-order space is the leading block), then the E edge
gradients, then two per face (faces sorted by their vertex triples).  The Schwarz
preconditioners only depend on the subspaces spanned by the functions of each subdomain, which
any basis attached to edges and faces spans alike (reading).

Every basis function is a sum of terms c * l^a * grad l_m (a a multi-index of barycentric
exponents), so element integrals are exact:  int_T l^a = 6 |T| a! / (|a| + 3)!  and on a
triangle  int l^a = 2 |tau| a! / (|a| + 2)!;  curl(l^a grad l_m) = sum_p a_p l^(a - e_p)
grad l_p x grad l_m.  The load uses a collapsed (Duffy) tensor Gauss rule.
"""
from math import factorial

import numpy as np
import scipy.sparse as sp

from . import dd, fem
from .mesh import LOCAL_EDGES, LOCAL_FACES

NLOC = 20


def _e(*idx):
    a = [0, 0, 0, 0]
    for i in idx:
        a[i] += 1
    return tuple(a)


def local_terms(gv):
    """The 20 local functions of a tetrahedron whose local vertices have global ids gv (4,):
    list of lists of (coef, exponents (4,), gradient index), in the local order
    [6 Whitney, 6 gradient, 4 faces x (f1, f2)] over LOCAL_EDGES and LOCAL_FACES."""
    out = []
    pairs = []
    for a, b in LOCAL_EDGES:
        i, j = (a, b) if gv[a] < gv[b] else (b, a)
        pairs.append((i, j))
    for i, j in pairs:
        out.append([(1.0, _e(i), j), (-1.0, _e(j), i)])
    for i, j in pairs:
        out.append([(1.0, _e(i), j), (1.0, _e(j), i)])
    for f in LOCAL_FACES:
        i, j, k = sorted(f, key=lambda q: gv[q])
        out.append([(1.0, _e(k, i), j), (-1.0, _e(k, j), i)])
        out.append([(1.0, _e(j, i), k), (-1.0, _e(j, k), i)])
    return out


def _curl_terms(terms):
    """curl of sum c l^a grad l_m as sum c' l^a' (grad l_p x grad l_m): (c', a', p, m)."""
    out = []
    for c, a, m in terms:
        for p in range(4):
            if a[p]:
                b = list(a)
                b[p] -= 1
                out.append((c * a[p], tuple(b), p, m))
    return out


def _int_tet(a, vol):
    s = sum(a)
    return 6.0 * vol * np.prod([factorial(x) for x in a]) / factorial(s + 3)


def _int_tri(a, area, opp):
    if a[opp]:
        return 0.0
    s = sum(a)
    return 2.0 * area * np.prod([factorial(x) for x in a]) / factorial(s + 2)


def element(X, gv):
    """K, M (20x20) of the tetrahedron with vertices X (4,3) and global vertex ids gv."""
    T = np.stack([X[1] - X[0], X[2] - X[0], X[3] - X[0]], axis=1)
    Ji = np.linalg.inv(T)
    g = np.zeros((4, 3))
    g[1:] = Ji
    g[0] = -Ji.sum(axis=0)
    vol = abs(np.linalg.det(T)) / 6.0
    terms = local_terms(gv)
    curls = [_curl_terms(t) for t in terms]
    K = np.zeros((NLOC, NLOC))
    M = np.zeros((NLOC, NLOC))
    for u in range(NLOC):
        for v in range(NLOC):
            M[u, v] = sum(c1 * c2 * _int_tet(tuple(x + y for x, y in zip(a1, a2)), vol) * (g[m1] @ g[m2])
                          for c1, a1, m1 in terms[u] for c2, a2, m2 in terms[v])
            K[u, v] = sum(c1 * c2 * _int_tet(tuple(x + y for x, y in zip(a1, a2)), vol)
                          * (np.cross(g[p1], g[m1]) @ np.cross(g[p2], g[m2]))
                          for c1, a1, p1, m1 in curls[u] for c2, a2, p2, m2 in curls[v])
    return K, M, g, vol


def face_mass(X, gv, lf):
    """Tangential mass int_tau phi_T . psi_T (20x20) over local face lf of the tetrahedron."""
    T = np.stack([X[1] - X[0], X[2] - X[0], X[3] - X[0]], axis=1)
    Ji = np.linalg.inv(T)
    g = np.zeros((4, 3))
    g[1:] = Ji
    g[0] = -Ji.sum(axis=0)
    opp = [q for q in range(4) if q not in LOCAL_FACES[lf]][0]
    fv = X[list(LOCAL_FACES[lf])]
    nrm = np.cross(fv[1] - fv[0], fv[2] - fv[0])
    area = 0.5 * np.linalg.norm(nrm)
    n = nrm / np.linalg.norm(nrm)
    P = np.eye(3) - np.outer(n, n)  # tangential projector
    terms = local_terms(gv)
    B = np.zeros((NLOC, NLOC))
    for u in range(NLOC):
        for v in range(NLOC):
            B[u, v] = sum(c1 * c2 * _int_tri(tuple(x + y for x, y in zip(a1, a2)), area, opp)
                          * (g[m1] @ P @ g[m2])
                          for c1, a1, m1 in terms[u] for c2, a2, m2 in terms[v])
    return B


_CACHE = {}


def _key(X, gv, extra=()):
    """Element integrals depend only on the shape (edge vectors) and on the order of the global
    vertex ids; identical tetrahedra (a structured mesh has few kinds) are computed once."""
    return (tuple(np.round((X[1:] - X[0]).ravel(), 13)), tuple(np.argsort(gv))) + tuple(extra)


def element_cached(X, gv):
    k = _key(X, gv, ("KM",))
    if k not in _CACHE:
        _CACHE[k] = element(X, gv)[:2]
    return _CACHE[k]


def face_mass_cached(X, gv, lf):
    k = _key(X, gv, ("B", lf))
    if k not in _CACHE:
        _CACHE[k] = face_mass(X, gv, lf)
    return _CACHE[k]


class Space:
    """DOF numbering of the order-2 space on an oracle Mesh."""

    def __init__(self, mesh):
        self.mesh = mesh
        E = mesh.n_edge
        self.E, self.F = E, len(mesh.face_key)
        self.n = 2 * E + 2 * self.F
        te, tf = mesh.tet_edge, mesh.tet_face
        self.tet_dof = np.concatenate([te, E + te, 2 * E + 2 * tf[:, [0]], 2 * E + 2 * tf[:, [0]] + 1,
                                       2 * E + 2 * tf[:, [1]], 2 * E + 2 * tf[:, [1]] + 1,
                                       2 * E + 2 * tf[:, [2]], 2 * E + 2 * tf[:, [2]] + 1,
                                       2 * E + 2 * tf[:, [3]], 2 * E + 2 * tf[:, [3]] + 1], axis=1)
        nv = mesh.n_vert
        keys = mesh.face_key
        self.face_vert = np.stack([keys // (nv * nv), (keys // nv) % nv, keys % nv], axis=1)

    def boundary_dof_mask(self):
        m = np.zeros(self.n, dtype=bool)
        eb = self.mesh.boundary_edge_mask()
        m[: self.E] = eb
        m[self.E: 2 * self.E] = eb
        fb = self.mesh.face_count == 1
        m[2 * self.E + 2 * np.nonzero(fb)[0]] = True
        m[2 * self.E + 2 * np.nonzero(fb)[0] + 1] = True
        return m

    def dofs_of_tets(self, tet_mask):
        return np.unique(self.tet_dof[tet_mask].ravel())


def assemble_parts(space, tets=None, faces=None):
    """K, M and the impedance mass M_b over the tetrahedra `tets` (default all) and the boundary
    triangles `faces` (vertex triples; default the box boundary)."""
    mesh = space.mesh
    idx = np.arange(mesh.n_tet) if tets is None else np.asarray(tets)
    N = space.n
    rows, cols, kv, mv = [], [], [], []
    for t in idx:
        gv = mesh.tet_vert[t]
        K, M = element_cached(mesh.xyz[gv], gv)
        d = space.tet_dof[t]
        rows.append(np.repeat(d, NLOC))
        cols.append(np.tile(d, NLOC))
        kv.append(K.ravel())
        mv.append(M.ravel())
    r, c = np.concatenate(rows), np.concatenate(cols)
    Kg = sp.coo_matrix((np.concatenate(kv), (r, c)), shape=(N, N)).tocsr()
    Mg = sp.coo_matrix((np.concatenate(mv), (r, c)), shape=(N, N)).tocsr()
    if faces is None:
        faces = mesh.bface_vert
    faces = np.asarray(faces).reshape(-1, 3)
    B = sp.csr_matrix((N, N))
    if len(faces):
        nv = mesh.n_vert
        fs = np.sort(faces, axis=1)
        fkey = (fs[:, 0] * nv + fs[:, 1]) * nv + fs[:, 2]
        fid = np.searchsorted(mesh.face_key, fkey)
        # a tetrahedron holding each face (restricted to `tets` when given)
        allowed = np.zeros(mesh.n_tet, dtype=bool)
        allowed[idx] = True
        owner = np.full(len(mesh.face_key), -1)
        lfo = np.full(len(mesh.face_key), -1)
        for lf in range(4):
            t_all = np.nonzero(allowed)[0]
            f_all = mesh.tet_face[t_all, lf]
            owner[f_all] = t_all
            lfo[f_all] = lf
        br, bc, bv = [], [], []
        for f in fid:
            t, lf = owner[f], lfo[f]
            gv = mesh.tet_vert[t]
            Bl = face_mass_cached(mesh.xyz[gv], gv, lf)
            d = space.tet_dof[t]
            br.append(np.repeat(d, NLOC))
            bc.append(np.tile(d, NLOC))
            bv.append(Bl.ravel())
        B = sp.coo_matrix((np.concatenate(bv), (np.concatenate(br), np.concatenate(bc))),
                          shape=(N, N)).tocsr()
    return Kg, Mg, B


def assemble(space, k, xi, bc=fem.BC_IMPEDANCE):
    """A = K - (k^2 + i xi) M - i sign(xi) k M_b, or with PEC identity rows and columns on the
    boundary degrees of freedom (edges and faces of the boundary)."""
    K, M, B = assemble_parts(space)
    pec = space.boundary_dof_mask() if bc == fem.BC_PEC else None
    return fem.combine(K, M, B, k, xi, bc, pec)


def _duffy_rule(nq):
    """Points (barycentric, (P,4)) and weights (sum 1/6 on the unit tetrahedron) of the collapsed
    tensor Gauss-Legendre rule with nq points per direction."""
    s, w = np.polynomial.legendre.leggauss(nq)
    s, w = 0.5 * (s + 1.0), 0.5 * w
    pts, wts = [], []
    for u, wu in zip(s, w):
        for v, wv in zip(s, w):
            for t, wt in zip(s, w):
                x = u
                y = v * (1 - u)
                z = t * (1 - u) * (1 - v)
                pts.append([1 - x - y - z, x, y, z])
                wts.append(wu * wv * wt * (1 - u) ** 2 * (1 - v))
    return np.array(pts), np.array(wts)


def evaluate(space, t, coef, lam):
    """Field sum_a coef_a phi_a at barycentric points lam (P,4) of tetrahedron t -> (P,3)."""
    mesh = space.mesh
    gv = mesh.tet_vert[t]
    X = mesh.xyz[gv]
    T = np.stack([X[1] - X[0], X[2] - X[0], X[3] - X[0]], axis=1)
    Ji = np.linalg.inv(T)
    g = np.zeros((4, 3))
    g[1:] = Ji
    g[0] = -Ji.sum(axis=0)
    out = np.zeros((lam.shape[0], 3), dtype=np.complex128)
    for c, terms in zip(coef, local_terms(gv)):
        for cc, a, m in terms:
            out += (c * cc) * np.prod(lam ** np.array(a)[None, :], axis=1)[:, None] * g[m][None, :]
    return out


def load_vector(space, F, bc=fem.BC_IMPEDANCE, nq=4):
    """f_a = int F . phi_a (collapsed Gauss rule, nq^3 points per tetrahedron)."""
    mesh = space.mesh
    lam, wts = _duffy_rule(nq)
    f = np.zeros(space.n, dtype=np.complex128)
    eye = np.eye(NLOC)
    for t in range(mesh.n_tet):
        gv = mesh.tet_vert[t]
        X = mesh.xyz[gv]
        k = _key(X, gv, ("phi", nq))
        if k not in _CACHE:  # basis values at the rule's points, (20, P, 3)
            _CACHE[k] = np.stack([evaluate(space, t, eye[a], lam).real for a in range(NLOC)])
        phi = _CACHE[k]
        vol6 = abs(np.linalg.det(np.stack([X[1] - X[0], X[2] - X[0], X[3] - X[0]], axis=1)))
        Fq = np.asarray(F(lam @ X))
        f[space.tet_dof[t]] += vol6 * np.einsum("q,qi,aqi->a", wts, Fq, phi)
    if bc == fem.BC_PEC:
        f[space.boundary_dof_mask()] = 0.0
    return f


class Partition:
    """Order-2 local DOF sets and Boolean owners from the tetrahedron sets of dd.Partition."""

    def __init__(self, space, part):
        self.space, self.part, self.N = space, part, part.N
        mesh = space.mesh
        E, F = space.E, space.F
        cnt_f_all = np.bincount(mesh.tet_face.ravel(), minlength=F)
        self.oras_sets, self.as_sets = [], []
        for l in range(part.N):
            m = part.tet_masks[l]
            self.oras_sets.append(space.dofs_of_tets(m))
            cf = np.bincount(mesh.tet_face[m].ravel(), minlength=F)
            fin = np.nonzero(cf == cnt_f_all)[0]
            e1 = part.as_sets[l]
            self.as_sets.append(np.sort(np.concatenate([e1, E + e1, 2 * E + 2 * fin, 2 * E + 2 * fin + 1])))
        owner = np.full(space.n, part.N, dtype=np.int64)
        np.minimum.at(owner, space.tet_dof.ravel(), np.repeat(part.part0, NLOC))
        self.owner = owner

    def local_set(self, kind):
        return self.oras_sets if kind == dd.ORAS else self.as_sets

    def pou(self, l, kind):
        idx = self.local_set(kind)[l]
        return (self.owner[idx] == l).astype(np.float64)


def local_matrix(p2, A, kind, k, xi, l, bc=fem.BC_IMPEDANCE):
    """Order-2 A^l: the minor of A (AS, RAS) or the impedance problem assembled on the
    tetrahedra of Omega_l with the impedance term on its boundary faces (ORAS; PEC faces of the
    box keep PEC), as dd.local_matrix for the lowest order."""
    if kind in (dd.AS, dd.RAS):
        idx = p2.as_sets[l]
        return A[idx][:, idx].tocsc()
    space, part = p2.space, p2.part
    mesh = space.mesh
    idx = p2.oras_sets[l]
    tets = np.nonzero(part.tet_masks[l])[0]
    faces = part.subdomain_boundary_faces(l)
    if bc == fem.BC_PEC:
        gb = set(map(tuple, mesh.bface_vert))
        faces = np.array([f for f in faces if tuple(f) not in gb]).reshape(-1, 3)
    K, M, B = assemble_parts(space, tets, faces)
    Al = (K.astype(np.complex128) - (k * k + 1j * xi) * M - 1j * fem.impedance_sign(xi) * k * B).tocsr()
    if bc == fem.BC_PEC:
        pec = space.boundary_dof_mask()
        if pec.any():
            keep = sp.diags((~pec).astype(np.float64))
            Al = (keep @ Al @ keep + sp.diags(pec.astype(np.float64))).tocsr()
    return Al[idx][:, idx].tocsc()


def schwarz(p2, A, kind, k, xi, bc=fem.BC_IMPEDANCE):
    """One-level AS / RAS / ORAS of the order-2 space (dd.Schwarz with these local problems)."""
    loc = [local_matrix(p2, A, kind, k, xi, l, bc) for l in range(p2.N)]
    return dd.Schwarz(p2, A, kind, k, xi, bc, local=loc)


def coarse_restriction(space, coarse_mesh, bc=fem.BC_IMPEDANCE):
    """R^0 of eq:restriction for the order-2 fine space, with the coarse space of lowest-order
    Whitney functions on the nested coarse mesh (reading: the paper does not say which coarse
    element order goes with order-2 fine elements; the lowest order keeps the coarse problem the
    one of the lowest-order runs).  A coarse Whitney function is, on every fine tetrahedron, a
    field a + b x x, i.e. a member of the fine lowest-order space, which in the hierarchical basis
    is spanned by the Whitney functions alone: its order-2 coefficients are its lowest-order
    ones (oracle/coarse.py) followed by zeros for the gradient and face functions."""
    from . import coarse as _coarse
    R1 = _coarse.restriction(space.mesh, coarse_mesh, bc)
    zero = sp.csr_matrix((R1.shape[0], space.n - space.E))
    return sp.hstack([R1, zero]).tocsr()


def weight_matrix(space, k, bc=fem.BC_IMPEDANCE):
    """D_k = K + k^2 M (eq:ip, eq:weight) of the order-2 space, the Gram matrix of
    (curl v, curl w) + k^2 (v, w) in the hierarchical basis; no boundary term; with PEC, identity
    rows and columns on the boundary DOFs (as fem.weight_matrix at the lowest order)."""
    K, M, _ = assemble_parts(space, faces=np.zeros((0, 3), dtype=np.int64))
    D = (K + (k * k) * M).tocsr()
    if bc == fem.BC_PEC:
        pec = space.boundary_dof_mask()
        if pec.any():
            keep = sp.diags((~pec).astype(np.float64))
            D = (keep @ D @ keep + sp.diags(pec.astype(np.float64))).tocsr()
    D.sum_duplicates()
    D.sort_indices()
    return D
