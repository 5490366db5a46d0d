"""The oracle's second-order Nedelec elements (oracle/order2.py) against what the mathematics
fixes: the lowest-order Whitney functions are the leading block of the hierarchical basis, so the
leading block of the order-2 K, M and M_b equals the lowest-order matrices of fem.py (closed
forms, independent code); the 20 local functions span the 20-dimensional first-family space of
order 2 (all linear fields included); the curl vanishes exactly on gradients of quadratic scalar
fields and nowhere else (rank K = N - (V + E - 1)); the Galerkin solution of a smooth
manufactured PEC problem converges at second order in L2 (first order for the lowest order);
Schwarz with one subdomain is the exact inverse and the local problems match a dense brute
force."""
import numpy as np
import pytest
import scipy.sparse as sp

from mx_inputs import random_rhs
from oracle import dd, fem, gmres, order2
from oracle.mesh import Mesh


@pytest.mark.parametrize("bc", [fem.BC_IMPEDANCE, fem.BC_PEC])
def test_lowest_order_is_the_leading_block(bc):
    m = Mesh(3, 2, 4, 1.0, 0.7, 1.3)
    S = order2.Space(m)
    E = m.n_edge
    K, M, B = order2.assemble_parts(S)
    K1, M1, B1 = fem.assemble_parts(m)
    for X, Y in ((K, K1), (M, M1), (B, B1)):
        assert abs(X[:E, :E] - Y).max() <= 1e-13 * abs(Y).max()
    A2 = order2.assemble(S, 3.0, 5.0, bc)
    A1 = fem.assemble(m, 3.0, 5.0, bc)
    assert abs(A2[:E, :E] - A1).max() <= 1e-13 * abs(A1).max()
    assert abs(A2 - A2.T).max() <= 1e-14 * abs(A2).max()
    assert abs(A2 - A2.conj().T).max() > 1e-3 * abs(A2).max()


def test_local_space_is_first_family_order_two():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((4, 3))
    gv = np.array([7, 2, 9, 4])
    terms = order2.local_terms(gv)
    T = np.stack([X[1] - X[0], X[2] - X[0], X[3] - X[0]], axis=1)
    g = np.zeros((4, 3))
    g[1:] = np.linalg.inv(T)
    g[0] = -g[1:].sum(axis=0)
    lam = rng.dirichlet(np.ones(4), size=80)
    pts = lam @ X
    cols = []
    for t in terms:
        v = np.zeros((80, 3))
        for c, a, mm in t:
            v += c * np.prod(lam ** np.array(a), axis=1)[:, None] * g[mm][None, :]
        cols.append(v.ravel())
    Phi = np.stack(cols, axis=1)
    assert np.linalg.matrix_rank(Phi, tol=1e-10) == 20
    for i in range(3):  # every linear vector field lies in the span
        for j in range(4):
            f = np.zeros((80, 3))
            f[:, i] = 1.0 if j == 3 else pts[:, j]
            c, *_ = np.linalg.lstsq(Phi, f.ravel(), rcond=None)
            assert np.abs(Phi @ c - f.ravel()).max() <= 1e-10


def test_curl_kernel_is_gradients_of_quadratics():
    m = Mesh(3, 3, 2)
    S = order2.Space(m)
    K, _, _ = order2.assemble_parts(S)
    E, V = m.n_edge, m.n_vert
    rng = np.random.default_rng(4)
    v, b = rng.standard_normal(V), rng.standard_normal(E)
    grad = np.zeros(S.n)  # grad(sum v_i l_i + sum_e b_e l_lo l_hi) in the hierarchical basis
    grad[:E] = v[m.edge_vert[:, 1]] - v[m.edge_vert[:, 0]]
    grad[E:2 * E] = b
    assert np.abs(K @ grad).max() <= 1e-12 * abs(K).max() * np.abs(grad).max()
    rank = np.linalg.matrix_rank(K.toarray(), tol=1e-9 * abs(K).max())
    assert rank == S.n - (V + E - 1)


def _l2_error(S, coef, Efun, nq=4):
    mesh = S.mesh
    lam, wts = order2._duffy_rule(nq)
    err = 0.0
    eye = np.eye(order2.NLOC)
    for t in range(mesh.n_tet):
        gv = mesh.tet_vert[t]
        X = mesh.xyz[gv]
        k = order2._key(X, gv, ("phi", nq))
        if k not in order2._CACHE:
            order2._CACHE[k] = np.stack([order2.evaluate(S, t, eye[a], lam).real for a in range(20)])
        phi = order2._CACHE[k]
        vol6 = abs(np.linalg.det(np.stack([X[1] - X[0], X[2] - X[0], X[3] - X[0]], axis=1)))
        Eh = np.einsum("a,aqi->qi", coef[S.tet_dof[t]], phi)
        err += vol6 * np.sum(wts * np.sum(np.abs(Efun(lam @ X) - Eh) ** 2, axis=1))
    return np.sqrt(err)


def test_manufactured_solution_second_order():
    """E = (sin pi y sin pi z, sin pi x sin pi z, sin pi x sin pi y) solves the PEC problem with
    F = (2 pi^2 - k^2 - i xi) E; the order-2 L2 error falls by about 4 per halving of h."""
    k, xi = 2.0, 1.0
    c = 2 * np.pi ** 2 - k * k - 1j * xi
    Efun = lambda x: np.stack([np.sin(np.pi * x[:, 1]) * np.sin(np.pi * x[:, 2]),
                               np.sin(np.pi * x[:, 0]) * np.sin(np.pi * x[:, 2]),
                               np.sin(np.pi * x[:, 0]) * np.sin(np.pi * x[:, 1])], axis=1)
    errs = []
    for n in (2, 4, 8):
        S = order2.Space(Mesh(n, n, n))
        A = order2.assemble(S, k, xi, fem.BC_PEC)
        f = order2.load_vector(S, lambda x: c * Efun(x), fem.BC_PEC)
        u = sp.linalg.spsolve(A.tocsc(), f)
        errs.append(_l2_error(S, u, Efun))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 1.8), (errs, rates)


def test_schwarz_order_two():
    m = Mesh(4, 4, 4)
    S = order2.Space(m)
    k, xi = 3.0, 9.0
    A = order2.assemble(S, k, xi)
    b = random_rhs(S.n, 5)
    # one subdomain: the preconditioner is A^-1
    p1 = order2.Partition(S, dd.Partition(m, 1, 1, 1, 0))
    for kind in (dd.AS, dd.ORAS):
        B = order2.schwarz(p1, A, kind, k, xi)
        res = gmres.gmres(A, b, B, restart=10, rtol=1e-10)
        assert res.converged and res.iters == 1
    # dense brute force of sum_l R^T D (A^l)^-1 R on a partition with overlap
    p2 = order2.Partition(S, dd.Partition(m, 2, 2, 1, 1))
    assert np.all(np.bincount(p2.owner, minlength=p2.N)[: p2.N] > 0)
    one = np.zeros(S.n)
    for l in range(p2.N):
        one[p2.oras_sets[l]] += p2.pou(l, dd.ORAS)
    assert np.array_equal(one, np.ones(S.n))  # Boolean partition of unity (eq:algebPartUnity)
    cover = np.zeros(S.n, bool)
    for l in range(p2.N):
        cover[p2.as_sets[l]] = True
    assert cover.all()
    for kind in (dd.AS, dd.ORAS):
        B = order2.schwarz(p2, A, kind, k, xi)
        D = np.zeros((S.n, S.n), dtype=np.complex128)
        for l, idx in enumerate(p2.local_set(kind)):
            inv = np.linalg.inv(order2.local_matrix(p2, A, kind, k, xi, l).toarray())
            if kind == dd.ORAS:
                inv = p2.pou(l, kind)[:, None] * inv
            D[np.ix_(idx, idx)] += inv
        assert np.linalg.norm(B(b) - D @ b) <= 1e-10 * np.linalg.norm(D @ b)


@pytest.mark.parametrize("box", [(1, 1, 1), (0, 0, 0)])
def test_oras_local_matrix_is_the_box_problem_order_two(box):
    """ImpRAS at order 2: with no overlap layers the local problem of a box subdomain equals the
    order-2 impedance Galerkin matrix of that box assembled on a mesh of its own (interface and
    global faces alike carry eq:imp with coefficient k).  Vertex numberings of the box and of the
    whole mesh order vertices the same way, so edges and faces match by vertex coordinates with
    no sign changes."""
    m = Mesh(5, 4, 6)
    cuts = ([0, 2, 4, 5], [0, 1, 3, 4], [0, 2, 4, 6])
    k, xi = 3.0, 5.0
    S = order2.Space(m)
    A = order2.assemble(S, k, xi)
    part = dd.Partition(m, 3, 3, 3, 0, *cuts)
    p2 = order2.Partition(S, part)
    l = box[0] + 3 * (box[1] + 3 * box[2])
    Al = order2.local_matrix(p2, A, dd.ORAS, k, xi, l).tocsr()
    lo = [cuts[a][box[a]] for a in range(3)]
    hi = [cuts[a][box[a] + 1] for a in range(3)]
    h = np.array([1.0 / 5, 1.0 / 4, 1.0 / 6])
    sub = Mesh(hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2], *((np.array(hi) - np.array(lo)) * h))
    Ss = order2.Space(sub)
    As = order2.assemble(Ss, k, xi).tocsr()

    def key(x):
        return tuple(np.round(x / h, 6).astype(int).ravel())

    gkey = {}
    for e in range(m.n_edge):
        gkey[("e",) + key(m.xyz[m.edge_vert[e]])] = e
    for f in range(S.F):
        gkey[("f",) + key(m.xyz[S.face_vert[f]])] = f
    off = np.array(lo) * h
    mp = np.zeros(Ss.n, dtype=np.int64)
    for e in range(sub.n_edge):
        ge = gkey[("e",) + key(sub.xyz[sub.edge_vert[e]] + off)]
        mp[e], mp[Ss.E + e] = ge, S.E + ge
    for f in range(Ss.F):
        gf = gkey[("f",) + key(sub.xyz[Ss.face_vert[f]] + off)]
        mp[2 * Ss.E + 2 * f], mp[2 * Ss.E + 2 * f + 1] = 2 * S.E + 2 * gf, 2 * S.E + 2 * gf + 1
    idx = p2.oras_sets[l]
    assert len(idx) == Ss.n and np.array_equal(np.sort(mp), idx)
    pos = np.searchsorted(idx, mp)
    P = sp.csr_matrix((np.ones(Ss.n), (pos, np.arange(Ss.n))), shape=(len(idx), Ss.n))
    mapped = (P @ As @ P.T).tocsr()
    assert abs(Al - mapped).max() <= 1e-12 * abs(Al).max()


@pytest.mark.parametrize("bc", [fem.BC_IMPEDANCE, fem.BC_PEC])
def test_coarse_restriction_reproduces_coarse_whitney_fields(bc):
    """Each row of the order-2 R^0, used as fine coefficients, is the coarse Whitney function
    itself: evaluated on fine tetrahedra at random points it equals l_a grad l_b - l_b grad l_a
    computed directly on the coarse tetrahedron holding the point."""
    from oracle import coarse
    fine = Mesh(4, 4, 4)
    cm = coarse.coarse_mesh(fine, 2)
    S = order2.Space(fine)
    R = order2.coarse_restriction(S, cm, bc)
    assert R.shape == (len(coarse.coarse_dofs(cm, bc)), S.n)
    keep = coarse.coarse_dofs(cm, bc)
    gc, _ = fem.tet_geometry(cm)
    rng = np.random.default_rng(5)
    for p in rng.choice(R.shape[0], 6, replace=False):
        ce = keep[p]
        a, b = cm.edge_vert[ce]
        coef = R[p].toarray().ravel()
        # coarse tetrahedra holding the edge, and a fine tetrahedron inside each at random
        for T in np.nonzero((cm.tet_edge == ce).any(axis=1))[0][:3]:
            la, lb = list(cm.tet_vert[T]).index(a), list(cm.tet_vert[T]).index(b)
            X = cm.xyz[cm.tet_vert[T]]
            # random point inside T, then the fine tetrahedron holding it
            w = rng.dirichlet(np.ones(4))
            x = w @ X
            gf, _ = fem.tet_geometry(fine)
            lam_all = np.einsum("tai,ti->ta", gf, x[None, :] - fine.xyz[fine.tet_vert[:, 0]])
            lam_all[:, 0] += 1.0
            t = int(np.argmax(lam_all.min(axis=1)))
            lam = lam_all[t][None, :]
            u = order2.evaluate(S, t, coef[S.tet_dof[t]], lam)[0].real
            direct = w[la] * gc[T, lb] - w[lb] * gc[T, la]
            assert np.allclose(u, direct, atol=1e-12 * np.abs(direct).max() + 1e-13), (p, T)


@pytest.mark.parametrize("k", [0.0, 3.0])
def test_weight_matrix_is_the_gram_matrix_order_two(k):
    """D_k = K + k^2 M of the order-2 space is the Gram matrix of (curl v, curl w) + k^2 (v, w)
    (eq:ip, eq:weight): for fields the order-2 space holds exactly -- the rotation (-y, x, 0), the
    gradient (y, x, 0) of xy and the quadratic (y^2, -xy, 0) (whose product with x vanishes) --
    the coefficients c of the L2 projection give c^T D c = int |curl u|^2 + k^2 int |u|^2 on the
    unit cube: 4 + 2k^2/3, 2k^2/3 and 3 + 14k^2/45."""
    from scipy.sparse.linalg import spsolve
    S = order2.Space(Mesh(2, 2, 2))
    D = order2.weight_matrix(S, k)
    _, M, _ = order2.assemble_parts(S, faces=np.zeros((0, 3), dtype=np.int64))
    cases = [(lambda x: np.stack([-x[:, 1], x[:, 0], 0 * x[:, 0]], 1), 4.0, 2.0 / 3.0),
             (lambda x: np.stack([x[:, 1], x[:, 0], 0 * x[:, 0]], 1), 0.0, 2.0 / 3.0),
             (lambda x: np.stack([x[:, 1] ** 2, -x[:, 0] * x[:, 1], 0 * x[:, 0]], 1), 3.0, 14.0 / 45.0)]
    for F, curl2, mass2 in cases:
        b = order2.load_vector(S, F).real
        c = spsolve(M.tocsc(), b)
        assert abs(c @ (M @ c) - mass2) <= 1e-12
        assert abs(c @ (D @ c) - (curl2 + k * k * mass2)) <= 1e-11 * (1 + curl2 + k * k)


def test_weight_matrix_pec_rows_order_two():
    S = order2.Space(Mesh(2, 3, 2))
    Dp = order2.weight_matrix(S, 4.0, fem.BC_PEC).toarray()
    Di = order2.weight_matrix(S, 4.0).toarray()
    pec = S.boundary_dof_mask()
    free = ~pec
    assert np.array_equal(Dp[np.ix_(pec, pec)], np.eye(pec.sum()))
    assert not Dp[np.ix_(pec, free)].any() and not Dp[np.ix_(free, pec)].any()
    assert np.array_equal(Dp[np.ix_(free, free)], Di[np.ix_(free, free)])
    assert np.linalg.eigvalsh(Dp).min() > 0
