"""Pins of the oracle's mesh, edge numbering and Galerkin assembly against what the paper and
the mathematics fix (no GPU).  Each test checks the oracle through a route that does not reuse
the oracle's own formula: closed forms, brute force, independent quadrature, exact identities."""
import itertools

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import fem
from oracle.mesh import LOCAL_EDGES, Mesh, gradient_matrix


def edge_count(nx, ny, nz):
    # one edge per vertex pair (v, v + s), s a nonzero 0/1 vector, both ends in the grid
    tot = 0
    for s in itertools.product((0, 1), repeat=3):
        if any(s):
            tot += (nx + 1 - s[0]) * (ny + 1 - s[1]) * (nz + 1 - s[2])
    return tot


@pytest.mark.parametrize("n", [(1, 1, 1), (2, 2, 2), (3, 3, 3), (2, 3, 4), (8, 8, 8)])
def test_counts_closed_form(n):
    m = Mesh(*n)
    nx, ny, nz = n
    assert m.n_vert == (nx + 1) * (ny + 1) * (nz + 1)
    assert m.n_tet == 6 * nx * ny * nz
    assert m.n_edge == edge_count(*n)
    if nx == ny == nz:
        c = nx
        assert m.n_edge == 3 * c * (c + 1) ** 2 + 3 * c * c * (c + 1) + c ** 3
    # Euler characteristic of a ball: V - E + F - T = 1
    assert m.n_vert - m.n_edge + len(m.face_key) - m.n_tet == 1
    # boundary: two triangles per boundary square
    assert len(m.bface_vert) == 4 * (nx * ny + ny * nz + nx * nz)


@pytest.mark.parametrize("n,E,nnz", [(1, 19, 163), (2, 98, 1106), (8, 4184, 61784)])
def test_pattern_brute_force(n, E, nnz):
    m = Mesh(n, n, n)
    pairs = set()
    for t in range(m.n_tet):
        es = [int(e) for e in m.tet_edge[t]]
        assert len(set(es)) == 6
        pairs.update(itertools.product(es, es))
    assert m.n_edge == E
    assert len(pairs) == nnz
    A = fem.assemble(m, 3.0, 9.0)
    assert A.nnz == nnz


def test_edges_and_orientation():
    m = Mesh(3, 2, 2)
    ev = m.edge_vert
    assert np.all(ev[:, 0] < ev[:, 1])
    key = ev[:, 0] * m.n_vert + ev[:, 1]
    assert np.all(np.diff(key) > 0)  # lexicographic (lo, hi)
    for t in range(m.n_tet):
        for le, (a, b) in enumerate(LOCAL_EDGES):
            va, vb = m.tet_vert[t, a], m.tet_vert[t, b]
            e = m.tet_edge[t, le]
            assert {va, vb} == set(ev[e])
            assert m.tet_edge_sign[t, le] == (1 if va < vb else -1)
    # tetrahedra fill the box with positive volume
    g, vol = fem.tet_geometry(m)
    assert np.all(vol > 0)
    assert abs(vol.sum() - 1.0) < 1e-13


def _duffy_rule(q=5):
    s, w = np.polynomial.legendre.leggauss(q)
    s, w = 0.5 * (s + 1), 0.5 * w
    pts, wts = [], []
    for (u, wu), (v, wv), (t, wt) in itertools.product(zip(s, w), zip(s, w), zip(s, w)):
        x = u
        y = (1 - u) * v
        z = (1 - u) * (1 - v) * t
        pts.append((x, y, z))
        wts.append(wu * wv * wt * (1 - u) ** 2 * (1 - v))
    return np.array(pts), np.array(wts)


def _bary(X, x):
    """Barycentric coordinates of points x (N,3) in tet X (4,3) by direct solve."""
    T = np.vstack([X.T, np.ones(4)])
    rhs = np.vstack([x.T, np.ones(len(x))])
    return np.linalg.solve(T, rhs).T


def _whitney(X, x, h=1e-6):
    """Whitney functions (N,6,3) and their curls (N,6,3) from barycentrics, gradients and curls
    by central differences (exact for these linear fields up to rounding)."""
    def w_at(pts):
        lam = _bary(X, pts)
        grads = np.zeros((4, 3))
        for d in range(3):
            e = np.zeros(3)
            e[d] = h
            grads[:, d] = (_bary(X, pts[:1] + e)[0] - _bary(X, pts[:1] - e)[0]) / (2 * h)
        out = np.zeros((len(pts), 6, 3))
        for k, (a, b) in enumerate(LOCAL_EDGES):
            out[:, k] = lam[:, a, None] * grads[b] - lam[:, b, None] * grads[a]
        return out
    W = w_at(x)
    C = np.zeros_like(W)
    J = np.zeros((len(x), 6, 3, 3))  # d w_i / d x_j
    for d in range(3):
        e = np.zeros(3)
        e[d] = h
        J[..., d] = (w_at(x + e) - w_at(x - e)) / (2 * h)
    C[..., 0] = J[..., 2, 1] - J[..., 1, 2]
    C[..., 1] = J[..., 0, 2] - J[..., 2, 0]
    C[..., 2] = J[..., 1, 0] - J[..., 0, 1]
    return W, C


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_element_matrices_by_quadrature(seed):
    rng = np.random.default_rng(seed)
    X = np.eye(4, 3, k=-1) + 0.2 * rng.standard_normal((4, 3))
    X[0] = 0.1 * rng.standard_normal(3)

    class M1:
        xyz = X
        tet_vert = np.arange(4)[None, :]
    g, vol = fem.tet_geometry(M1)
    K, M = fem.element_matrices(g, vol)
    ref_pts, ref_w = _duffy_rule()
    Jm = np.stack([X[1] - X[0], X[2] - X[0], X[3] - X[0]], axis=1)
    x = X[0] + ref_pts @ Jm.T
    wq = ref_w * abs(np.linalg.det(Jm))
    W, C = _whitney(X, x)
    Mq = np.einsum("q,qei,qfi->ef", wq, W, W)
    Kq = np.einsum("q,qei,qfi->ef", wq, C, C)
    assert np.allclose(M[0], Mq, rtol=1e-8, atol=1e-9)
    assert np.allclose(K[0], Kq, rtol=1e-6, atol=1e-6)
    assert np.all(np.linalg.eigvalsh(M[0]) > 0)
    # duality: line integral of w_e along edge f (tangent x_b - x_a) is delta_ef
    s, w = np.polynomial.legendre.leggauss(3)
    s, w = 0.5 * (s + 1), 0.5 * w
    for f, (a, b) in enumerate(LOCAL_EDGES):
        t = X[b] - X[a]
        pts = X[a] + s[:, None] * t
        Wf, _ = _whitney(X, pts)
        li = np.einsum("q,qei,i->e", w, Wf, t)
        expect = np.zeros(6)
        expect[f] = 1.0
        assert np.allclose(li, expect, atol=1e-8)
    # gradients of P1 functions are in the kernel of the local curl-curl matrix
    Gl = np.zeros((6, 4))
    for k, (a, b) in enumerate(LOCAL_EDGES):
        Gl[k, a], Gl[k, b] = -1.0, 1.0
    assert np.abs(K[0] @ Gl).max() < 1e-10 * np.abs(K[0]).max()


def test_reference_tet_hand_values():
    # reference tetrahedron: grad l0 = (-1,-1,-1), grad l1..3 = unit vectors, |T| = 1/6
    class M1:
        xyz = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], dtype=float)
        tet_vert = np.arange(4)[None, :]
    g, vol = fem.tet_geometry(M1)
    K, M = fem.element_matrices(g, vol)
    # edge (0,1): curl w = 2 (-1,-1,-1) x (1,0,0) = (0,-2,2): K = |T| * 8 = 4/3
    # |w|^2 integral: |T| (2/20 * 1 + 2/20 * 1 + 2/20 * 3) = 1/12
    assert abs(K[0, 0, 0] - 4.0 / 3.0) < 1e-14
    assert abs(M[0, 0, 0] - 1.0 / 12.0) < 1e-14
    # edge (2,3): curl w = 2 e_y x e_z = (2,0,0): K = 4/6; mass |T| (2/20 + 2/20) = 1/30
    assert abs(K[0, 5, 5] - 2.0 / 3.0) < 1e-14
    assert abs(M[0, 5, 5] - 1.0 / 30.0) < 1e-14


def test_face_mass_by_quadrature():
    m = Mesh(1, 1, 1, 1.0, 2.0, 0.5)
    bf = m.bface_vert[:4]
    Mb, eid, sgn = fem.face_mass(m, bf)
    s, w = np.polynomial.legendre.leggauss(6)
    s, w = 0.5 * (s + 1), 0.5 * w
    for f in range(len(bf)):
        P = m.xyz[bf[f]]
        n = np.cross(P[1] - P[0], P[2] - P[0])
        area = 0.5 * np.linalg.norm(n)
        n /= np.linalg.norm(n)
        pts, wts = [], []
        for (u, wu), (v, wv) in itertools.product(zip(s, w), zip(s, w)):
            pts.append(P[0] + u * (P[1] - P[0]) + (1 - u) * v * (P[2] - P[0]))
            wts.append(wu * wv * (1 - u) * 2 * area)
        pts, wts = np.array(pts), np.array(wts)
        # barycentrics on the triangle by least squares, gradients by differences
        def lam(x):
            T = np.vstack([P.T, np.ones(3)])
            return np.linalg.lstsq(T, np.vstack([x.T, np.ones(len(x))]), rcond=None)[0].T
        L = lam(pts)
        grads = np.zeros((3, 3))
        for d in range(3):
            e = np.zeros(3)
            e[d] = 1e-6
            grads[:, d] = (lam(pts[:1] + e)[0] - lam(pts[:1] - e)[0]) / 2e-6
        grads -= np.outer(grads @ n, n)  # in-plane part
        le = [(0, 1), (0, 2), (1, 2)]
        Wt = np.stack([L[:, a, None] * grads[b] - L[:, b, None] * grads[a] for a, b in le], axis=1)
        Mq = np.einsum("q,qei,qfi->ef", wts, Wt, Wt)
        assert np.allclose(Mb[f], Mq, rtol=1e-7, atol=1e-9)


@pytest.mark.parametrize("bc", [fem.BC_IMPEDANCE, fem.BC_PEC])
def test_complex_symmetric_not_hermitian(bc):
    m = Mesh(3, 3, 3)
    A = fem.assemble(m, 3.0, 2.0, bc)
    assert abs(A - A.T).max() < 1e-14 * abs(A).max()
    assert abs(A - A.conj().T).max() > 1e-3 * abs(A).max()


def test_curl_kills_gradients_and_rank():
    m = Mesh(2, 2, 2)
    K, M, Mb = fem.assemble_parts(m)
    G = gradient_matrix(m)
    assert abs(K @ G).max() < 1e-12 * abs(K).max()
    Kd = K.toarray()
    rank = np.linalg.matrix_rank(Kd, tol=1e-9 * np.abs(Kd).max())
    assert rank == m.n_edge - m.n_vert + 1
    # impedance form on gradients: A G phi = -(k^2 + i xi) M G phi - i k M_b G phi
    k, xi = 2.5, 3.0
    A = fem.assemble(m, k, xi)
    phi = np.random.default_rng(0).standard_normal(m.n_vert)
    lhs = A @ (G @ phi)
    rhs = -(k * k + 1j * xi) * (M @ (G @ phi)) - 1j * k * (Mb @ (G @ phi))
    assert np.abs(lhs - rhs).max() < 1e-12 * np.abs(rhs).max()


@pytest.mark.parametrize("k,xi", [(4.0, 16.0), (4.0, 4.0), (3.0, -5.0)])
def test_coercivity_identity_pec(k, xi):
    """Lemma (coercivity) proof: Im[Theta a(v,v)] = (Im z/|z|)(||curl v||^2 + |z|^2 ||v||^2),
    Theta = -conj(z)/|z|, z = sqrt(k^2 + i xi) with Im z > 0 (Definition of z)."""
    m = Mesh(3, 3, 3)
    K, M, Mb = fem.assemble_parts(m)
    interior = ~m.boundary_edge_mask()
    A = fem.assemble(m, k, xi, fem.BC_PEC)
    z = np.sqrt(complex(k * k, xi))
    if z.imag < 0:
        z = -z
    assert z.imag > 0 and np.sign(xi) * z.real > 0
    theta = -np.conj(z) / abs(z)
    rng = np.random.default_rng(1)
    for _ in range(3):
        v = (rng.standard_normal(m.n_edge) + 1j * rng.standard_normal(m.n_edge)) * interior
        a = np.vdot(v, A @ v)
        kv = np.vdot(v, K @ v).real
        mv = np.vdot(v, M @ v).real
        lhs = (theta * a).imag
        rhs = z.imag / abs(z) * (kv + abs(z) ** 2 * mv)
        assert abs(lhs - rhs) < 1e-10 * abs(rhs)
        assert abs(a) >= lhs > 0


def test_impedance_energy_identity():
    m = Mesh(3, 2, 4)
    K, M, Mb = fem.assemble_parts(m)
    k, xi = 5.0, 7.0
    A = fem.assemble(m, k, xi)
    rng = np.random.default_rng(2)
    v = rng.standard_normal(m.n_edge) + 1j * rng.standard_normal(m.n_edge)
    lhs = np.vdot(v, A @ v).imag
    rhs = -xi * np.vdot(v, M @ v).real - k * np.vdot(v, Mb @ v).real
    assert abs(lhs - rhs) < 1e-11 * abs(rhs)
    assert abs(np.vdot(v, A @ v).real - (np.vdot(v, K @ v).real - k * k * np.vdot(v, M @ v).real)) \
        < 1e-10 * abs(np.vdot(v, K @ v))


def test_consistency_linear_field():
    """E = a + b x x lies in the lowest-order space, curl curl E = 0, so on interior edges
    (A Pi_h E)_e = int F . w_e with F = -(k^2 + i xi) E; the load rule is exact for E . w."""
    m = Mesh(4, 3, 3, 1.0, 0.8, 1.2)
    k, xi = 3.0, 5.0
    a = np.array([0.3, -1.1, 0.7])
    b = np.array([0.5, 0.2, -0.9])
    Efun = lambda x: a[None, :] + np.cross(b[None, :], x)
    u = fem.interpolate(m, Efun)
    A = fem.assemble(m, k, xi)
    f = fem.load_vector(m, lambda x: -(k * k + 1j * xi) * Efun(x))
    interior = ~m.boundary_edge_mask()
    r = (A @ u - f)[interior]
    assert np.abs(r).max() < 1e-12 * np.abs(f).max()


def _l2_error(m, u, Efun):
    """|| E - E_h ||_L2 with the 5^3-point Duffy rule on every tetrahedron."""
    ref_pts, ref_w = _duffy_rule(4)
    g, vol = fem.tet_geometry(m)
    x = m.xyz[m.tet_vert]
    lamq = np.hstack([1 - ref_pts.sum(1, keepdims=True), ref_pts])  # (Q,4)
    err2 = 0.0
    ue = u[m.tet_edge] * m.tet_edge_sign  # (T,6)
    for q in range(len(ref_w)):
        lam = lamq[q]
        xq = np.einsum("a,tai->ti", lam, x)
        w = lam[LOCAL_EDGES[:, 0]][None, :, None] * g[:, LOCAL_EDGES[:, 1], :] \
            - lam[LOCAL_EDGES[:, 1]][None, :, None] * g[:, LOCAL_EDGES[:, 0], :]
        Eh = np.einsum("te,tei->ti", ue, w)
        d = Efun(xq) - Eh
        err2 += (ref_w[q] * 6 * vol * (np.abs(d) ** 2).sum(1)).sum()
    return np.sqrt(err2)


def test_manufactured_first_order():
    """E = (sin pi y sin pi z, sin pi x sin pi z, sin pi x sin pi y) has E x n = 0 on the unit
    cube and curl curl E = 2 pi^2 E, so F = (2 pi^2 - k^2 - i xi) E; lowest-order edge elements
    converge at first order in L2 (Sec. 2.2, order m = 0 Nedelec space)."""
    k, xi = 2.0, 4.0
    pi = np.pi

    def Efun(x):
        X, Y, Z = x[:, 0], x[:, 1], x[:, 2]
        return np.stack([np.sin(pi * Y) * np.sin(pi * Z), np.sin(pi * X) * np.sin(pi * Z),
                         np.sin(pi * X) * np.sin(pi * Y)], axis=1)
    errs = []
    for n in (4, 8, 16):
        m = Mesh(n, n, n)
        A = fem.assemble(m, k, xi, fem.BC_PEC)
        f = fem.load_vector(m, lambda x: (2 * pi * pi - k * k - 1j * xi) * Efun(x), fem.BC_PEC)
        u = spla.spsolve(A.tocsc(), f)
        errs.append(_l2_error(m, u, Efun))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 0.85) and np.all(rates < 1.3), (errs, rates)


@pytest.mark.parametrize("lengths", [(1.0, 1.0, 1.0), (0.7, 1.3, 1.1)])
@pytest.mark.parametrize("k", [0.0, 3.0, 11.0])
def test_weight_matrix_is_the_gram_matrix(lengths, k):
    """D_k (eq:ip) is the Gram matrix of (v, w)_{curl,k} = (curl v, curl w) + k^2 (v, w)
    (eq:weight): for fields E = a + b x x, which the lowest-order Whitney space holds exactly,
    V^H D V with V the edge interpolant equals int |curl E|^2 + k^2 int |E|^2 (curl E = 2 b),
    computed here by a tensor Gauss rule exact for the quadratic integrand.  Also for the
    bilinear form between two such fields."""
    m = Mesh(4, 3, 5, *lengths)
    D = fem.weight_matrix(m, k)
    rng = np.random.default_rng(int(10 * k) + int(10 * lengths[0]))
    s, w = np.polynomial.legendre.leggauss(2)
    pts, wts = [], []
    for (si, wi), (sj, wj), (sk, wk) in itertools.product(zip(s, w), repeat=3):
        pts.append([(si + 1) / 2 * lengths[0], (sj + 1) / 2 * lengths[1], (sk + 1) / 2 * lengths[2]])
        wts.append(wi * wj * wk / 8 * lengths[0] * lengths[1] * lengths[2])
    pts, wts = np.array(pts), np.array(wts)
    vol = lengths[0] * lengths[1] * lengths[2]
    fields = []
    for _ in range(2):
        a = rng.standard_normal(3) + 1j * rng.standard_normal(3)
        b = rng.standard_normal(3) + 1j * rng.standard_normal(3)
        fields.append((a, b))
    V = [fem.interpolate(m, lambda x, a=a, b=b: a[None, :] + np.cross(b[None, :], x)) for a, b in fields]
    for (a1, b1), V1 in zip(fields, V):
        for (a2, b2), V2 in zip(fields, V):
            E1 = a1[None, :] + np.cross(b1[None, :], pts)
            E2 = a2[None, :] + np.cross(b2[None, :], pts)
            exact = 4.0 * np.vdot(b2, b1) * vol + k * k * np.sum(wts * np.sum(E1 * np.conj(E2), axis=1))
            got = np.vdot(V2, D @ V1)
            assert abs(got - exact) <= 1e-12 * max(1.0, abs(exact))
    # real symmetric positive definite; k only enters through k^2 M
    assert abs(D - D.T).max() <= 1e-14 * abs(D).max()
    K, M, _ = fem.assemble_parts(m)
    assert abs(D - (K + k * k * M)).max() <= 1e-14 * abs(D).max()


def test_weight_matrix_pec_rows():
    """With PEC, the constrained boundary edges get identity rows and columns in D_k, and the
    free block equals that of K + k^2 M."""
    m = Mesh(3, 3, 3)
    Dp = fem.weight_matrix(m, 5.0, fem.BC_PEC).toarray()
    Di = fem.weight_matrix(m, 5.0).toarray()
    pec = m.boundary_edge_mask()
    free = ~pec
    assert np.array_equal(Dp[np.ix_(pec, pec)], np.eye(pec.sum()))
    assert not Dp[np.ix_(pec, free)].any() and not Dp[np.ix_(free, pec)].any()
    assert np.array_equal(Dp[np.ix_(free, free)], Di[np.ix_(free, free)])
    assert np.linalg.eigvalsh(Dp).min() > 0
