"""Pins of the oracle's partition, Schwarz preconditioners, RCM and GMRES (no GPU)."""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from mx_inputs import jittered_cuts, random_rhs
from oracle import dd, fem, gmres, rcm
from oracle.mesh import Mesh

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_partition_of_unity_and_cover():
    m = Mesh(6, 5, 4)
    part = dd.Partition(m, 3, 2, 2, 2)
    E = m.n_edge
    for kind in (dd.RAS, dd.ORAS):
        S = sp.csr_matrix((E, E))
        cover = np.zeros(E, dtype=bool)
        for l in range(part.N):
            R = part.restriction(l, kind)
            S = S + R.T @ sp.diags(part.pou(l, kind)) @ R
            cover[part.local_set(kind)[l]] = True
        assert abs(S - sp.identity(E)).max() == 0.0  # eq:algebPartUnity exactly
        assert cover.all()  # the local sets cover all DOFs
    for l in range(part.N):
        assert set(part.as_sets[l]) <= set(part.oras_sets[l])
        assert len(part.neighbours(l)) <= 26  # finite overlap for boxes


def test_overlap_monotone_and_touching():
    m = Mesh(6, 6, 6)
    prev = None
    for L in range(4):
        part = dd.Partition(m, 2, 2, 2, L)
        if prev is not None:
            for l in range(part.N):
                assert np.all(part.tet_masks[l] >= prev.tet_masks[l])
        prev = part
    # one sweep adds exactly the tetrahedra sharing a vertex with the previous set
    part0 = dd.Partition(m, 2, 2, 2, 0)
    part1 = dd.Partition(m, 2, 2, 2, 1)
    v0 = set(m.tet_vert[part0.tet_masks[0]].ravel())
    brute = np.array([bool(set(t) & v0) for t in m.tet_vert])
    assert np.array_equal(brute, part1.tet_masks[0])
    # L = 0: AS sets are interior edges of the boxes, ORAS sets all their edges
    assert sum(len(s) for s in part0.oras_sets) > m.n_edge > sum(len(s) for s in part0.as_sets)


def test_config1_local_sizes_symmetry():
    """8^3 cubes, 2x2x2 boxes, 2 layers.  The Kuhn split is invariant under permutations of the
    axes and under the point reflection x -> (1,1,1) - x, so the six boxes off the main diagonal
    have equal local sizes and the two on it (0 and 7) are equal to each other."""
    m = Mesh(8, 8, 8)
    part = dd.Partition(m, 2, 2, 2, 2)
    for sets in (part.oras_sets, part.as_sets):
        n = [len(s) for s in sets]
        assert n[0] == n[7] and len(set(n[1:7])) == 1 and n[0] > n[1]
    assert len(part.oras_sets[0]) == 1854 and len(part.as_sets[0]) == 1512


@pytest.mark.parametrize("kind", [dd.AS, dd.RAS, dd.ORAS])
def test_dense_brute_force(kind):
    m = Mesh(3, 3, 2)
    k, xi = 3.0, 9.0
    A = fem.assemble(m, k, xi)
    part = dd.Partition(m, 2, 2, 1, 1)
    B = dd.Schwarz(part, A, kind, k, xi)
    Bd = dd.dense_schwarz(part, A, kind, k, xi)
    rng = np.random.default_rng(0)
    v = rng.standard_normal(m.n_edge) + 1j * rng.standard_normal(m.n_edge)
    assert np.allclose(B(v), Bd @ v, rtol=1e-10, atol=1e-12 * np.abs(Bd @ v).max())
    if kind == dd.AS:
        assert np.abs(Bd - Bd.T).max() < 1e-10 * np.abs(Bd).max()  # AS is complex symmetric


def test_as_local_projection():
    """T^l = R^T (A^l)^-1 R A is a projection and R A (I - T^l) = 0 (Lemma thm:repQ)."""
    m = Mesh(3, 3, 3)
    k, xi = 3.0, 9.0
    A = fem.assemble(m, k, xi).toarray()
    part = dd.Partition(m, 2, 1, 1, 1)
    idx = part.as_sets[0]
    R = np.zeros((len(idx), m.n_edge))
    R[np.arange(len(idx)), idx] = 1
    Al = R @ A @ R.T
    T = R.T @ np.linalg.solve(Al, R @ A)
    assert np.abs(T @ T - T).max() < 1e-9
    assert np.abs(R @ A @ (np.eye(m.n_edge) - T)).max() < 1e-9 * np.abs(A).max()
    # the oracle's AS minors are exactly these
    loc = dd.local_matrices(part, fem.assemble(m, k, xi), dd.AS, k, xi)
    assert np.abs(loc[0].toarray() - Al).max() == 0.0


@pytest.mark.parametrize("kind", [dd.AS, dd.RAS, dd.ORAS])
def test_single_subdomain_is_exact(kind):
    """N = 1: B^-1 = A^-1 (eq:defAS with one subdomain), GMRES converges in one iteration."""
    m = Mesh(4, 3, 3)
    k, xi = 4.0, 4.0
    A = fem.assemble(m, k, xi)
    part = dd.Partition(m, 1, 1, 1, 2)
    B = dd.Schwarz(part, A, kind, k, xi)
    f = np.random.default_rng(3).standard_normal(m.n_edge) + 0j
    res = gmres.gmres(A, f, B, restart=10, rtol=1e-10)
    assert res.iters == 1 and res.converged
    assert np.linalg.norm(A @ res.x - f) < 1e-10 * np.linalg.norm(f)


@pytest.mark.parametrize("kind", [dd.AS, dd.ORAS])
def test_absorption_only_in_the_preconditioner(kind):
    """A_0 (no absorption) preconditioned by the Schwarz method built at xi_prec (Sec. 1.2,
    eq. key_intro).  A_0 - A_prec = i xi_prec M exactly (the impedance term keeps sign +1 at
    xi = 0).  With one subdomain B^-1 = A_prec^-1, so the preconditioned operator is
    I + i xi_prec M A_prec^-1: GMRES takes more than one iteration (one when xi_prec = xi_prob)
    and converges to the solution of A_0 x = f."""
    m = Mesh(4, 3, 3)
    k, xp = 4.0, 4.0
    A0 = fem.assemble(m, k, 0.0)
    Ap = fem.assemble(m, k, xp)
    _, M, _ = fem.assemble_parts(m)
    assert abs(A0 - Ap - 1j * xp * M).max() <= 1e-14 * abs(A0).max()
    part = dd.Partition(m, 1, 1, 1, 2)
    B = dd.Schwarz(part, Ap, kind, k, xp)
    rng = np.random.default_rng(5)
    v = rng.standard_normal(m.n_edge) + 1j * rng.standard_normal(m.n_edge)
    zp = spla.spsolve(Ap.tocsc(), v)
    assert np.linalg.norm(B(v) - zp) <= 1e-12 * np.linalg.norm(zp)
    f = rng.standard_normal(m.n_edge) + 0j
    res = gmres.gmres(A0, f, B, restart=m.n_edge, rtol=1e-12)
    assert res.converged and 1 < res.iters < m.n_edge
    x = spla.spsolve(A0.tocsc(), f)
    assert np.linalg.norm(res.x - x) <= 1e-9 * np.linalg.norm(x)


def test_full_overlap_limits():
    """Every Omega_l = Omega: RAS and ORAS equal A^-1, AS equals N A^-1."""
    m = Mesh(4, 4, 2)
    k, xi = 3.0, 3.0
    A = fem.assemble(m, k, xi)
    part = dd.Partition(m, 2, 2, 1, 6)
    assert all(mk.all() for mk in part.tet_masks)
    v = np.random.default_rng(4).standard_normal(m.n_edge) + 1j
    x = spla.spsolve(A.tocsc(), v)
    for kind, scale in ((dd.RAS, 1), (dd.ORAS, 1), (dd.AS, part.N)):
        z = dd.Schwarz(part, A, kind, k, xi)(v)
        assert np.linalg.norm(z - scale * x) < 1e-9 * np.linalg.norm(x)


def test_givens():
    rng = np.random.default_rng(5)
    for _ in range(20):
        a, b = rng.standard_normal(2) + 1j * rng.standard_normal(2)
        c, s, rho = gmres.givens(a, b)
        x, y = gmres.apply_givens(c, s, a, b)
        assert abs(x - rho) < 1e-14 and abs(y) < 1e-14
        G = np.array([[c, s], [-np.conj(s), c]])
        assert np.abs(G.conj().T @ G - np.eye(2)).max() < 1e-14
    c, s, rho = gmres.givens(0.0, 2.0 - 1j)
    assert c == 0 and rho == 2.0 - 1j


@pytest.mark.parametrize("flexible", [False, True])
def test_gmres_minimal_residual_brute_force(flexible):
    """x_m minimises ||b - A x|| over x0 + M^-1 K_m(A M^-1, r0) (Sec. 5.2), checked against an
    explicit Krylov basis and a dense least-squares solve for every m."""
    rng = np.random.default_rng(6)
    n = 24
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)) + 6 * np.eye(n)
    Minv = np.linalg.inv(A + 0.5 * rng.standard_normal((n, n)))
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    C = A @ Minv
    for msteps in range(1, 9):
        res = gmres.gmres(A, b, lambda v: Minv @ v, restart=30, fixed_iters=msteps,
                          flexible=flexible)
        Kb = np.stack([np.linalg.matrix_power(C, j) @ b for j in range(msteps)], axis=1)
        Q, _ = np.linalg.qr(Kb)
        c, *_ = np.linalg.lstsq(C @ Q, b, rcond=None)
        x_ref = Minv @ (Q @ c)
        assert np.linalg.norm(res.x - x_ref) < 1e-9 * np.linalg.norm(x_ref)
        assert res.iters == msteps


def test_gmres_terminates_within_n():
    rng = np.random.default_rng(7)
    n = 12
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    b = rng.standard_normal(n) + 0j
    res = gmres.gmres(A, b, restart=n, rtol=1e-12, max_iters=n)
    assert res.converged and res.iters <= n


def test_rcm_path_and_grid():
    # path 0-1-2-3-4: least-key start 0 is already peripheral; CM order 0..4, reversed
    n = 5
    P = sp.diags([np.ones(n - 1), np.ones(n), np.ones(n - 1)], [-1, 0, 1]).tocsr()
    perm = rcm.rcm(*rcm.pattern_graph(P))
    assert list(perm) == [4, 3, 2, 1, 0]
    # a 2-D 7x4 grid: starting at a corner the levels are anti-diagonals of width <= 4, and a
    # Cuthill-McKee order keeps neighbours in adjacent levels, so the bandwidth is <= 2*4 - 1
    nx, ny = 7, 4
    idx = np.arange(nx * ny).reshape(ny, nx)
    rows, cols = [], []
    for (a, b) in [(idx[:, :-1], idx[:, 1:]), (idx[:-1, :], idx[1:, :])]:
        rows += list(a.ravel()) + list(b.ravel())
        cols += list(b.ravel()) + list(a.ravel())
    G = sp.csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(nx * ny, nx * ny))
    perm = rcm.rcm(*rcm.pattern_graph(G))
    assert sorted(perm) == list(range(nx * ny))
    inv = np.empty_like(perm)
    inv[perm] = np.arange(len(perm))
    Gp = G[perm][:, perm].tocoo()
    assert np.abs(Gp.row - Gp.col).max() <= 2 * ny - 1
    assert perm[-1] in (0, nx - 1, nx * (ny - 1), nx * ny - 1)  # a corner is the root
    # envelope: first column of each permuted row, brute force
    first = rcm.envelope(*rcm.pattern_graph(G), perm)
    D = Gp.toarray() + np.eye(nx * ny)
    assert np.array_equal(first, np.array([np.nonzero(D[i])[0].min() for i in range(nx * ny)]))


def test_rcm_disconnected_components():
    # two components {0,2} and {1,3,4}; isolated node 5
    rows = [0, 2, 1, 3, 3, 4]
    cols = [2, 0, 3, 1, 4, 3]
    G = sp.csr_matrix((np.ones(6), (rows, cols)), shape=(6, 6))
    perm = rcm.rcm(*rcm.pattern_graph(G))
    assert sorted(perm) == list(range(6))
    # isolated vertex has least key (0, 5): visited first, so it is last after reversal
    assert perm[-1] == 5


def test_paper_ordering_ras_beats_as():
    """Sec. 6.3: RAS (and ORAS) need fewer iterations than AS at equal overlap (Table tab:rasHras
    against tab:1 / tab:minOverlap).  The paper's counts are context (other meshes), only the
    ordering is checked."""
    with open(os.path.join(GOLDEN, "paper_one_level_counts.json")) as fh:
        paper = json.load(fh)
    t6 = paper["tab:rasHras"]["one_level_RAS_minimal_overlap"]
    t2 = paper["tab:minOverlap"]["alpha_0.8"]
    assert all(r < a for r, a in zip(t6, t2))
    m = Mesh(8, 8, 8)
    k, xi = 4.0, 16.0
    A = fem.assemble(m, k, xi)
    f = fem.load_vector(m, fem.gaussian_source((0.5, 0.5, 0.5), (1, 0, 0), 0.1))
    part = dd.Partition(m, 2, 2, 2, 2)
    its = {}
    for kind in (dd.AS, dd.RAS, dd.ORAS):
        res = gmres.gmres(A, f, dd.Schwarz(part, A, kind, k, xi), restart=50, rtol=1e-6)
        assert res.converged and res.relres_true <= 1e-6
        its[kind] = res.iters
    assert its[dd.RAS] < its[dd.AS] and its[dd.ORAS] <= its[dd.RAS]


def test_paper_low_absorption_and_weighting():
    """Sec. 6.2, Tables tab:1, tab:lowAbs and tab:weighted (PEC on the global boundary, AS with
    its PEC local problems, generous overlap).  At xi = k^2 the one-level iteration counts stay
    flat as k grows; at xi = k (tab:lowAbs) they are larger and grow quickly with k; GMRES
    weighted by D_k (tab:weighted) takes about as many iterations as the standard method.  The
    paper's counts are context (other meshes and partition of unity): only these three
    properties are checked, on one 16^3 mesh with 4x4x4 boxes and 2 layers at k = 8 and 10."""
    with open(os.path.join(GOLDEN, "paper_one_level_counts.json")) as fh:
        paper = json.load(fh)
    for a in ("alpha_0.8", "alpha_0.9"):
        flat, low, wtd = paper["tab:1"][a], paper["tab:lowAbs"][a], paper["tab:weighted"][a]
        assert max(flat) - min(flat) <= 8 and low[0] > 2.5 * flat[0] and low[1] > 4 * flat[1]
        assert all(abs(x - y) <= 2 for x, y in zip(wtd, flat))
    m = Mesh(16, 16, 16)
    f = fem.load_vector(m, fem.gaussian_source((0.5, 0.5, 0.5), (1, 0, 0), 0.1), fem.BC_PEC)
    part = dd.Partition(m, 4, 4, 4, 2)
    its = {}
    for k in (8.0, 10.0):
        for xi in (k * k, k):
            A = fem.assemble(m, k, xi, fem.BC_PEC)
            B = dd.Schwarz(part, A, dd.AS, k, xi, fem.BC_PEC)
            res = gmres.gmres(A, f, B, restart=200, rtol=1e-6, max_iters=400)
            assert res.converged and res.relres_true <= 1e-6
            its[k, xi] = res.iters
            if k == 8.0 and xi == k * k:
                resw = gmres.gmres(A, f, B, restart=200, rtol=1e-6, max_iters=400,
                                   D=fem.weight_matrix(m, k, fem.BC_PEC))
                assert resw.converged and abs(resw.iters - res.iters) <= 3, (resw.iters, res.iters)
    assert abs(its[10.0, 100.0] - its[8.0, 64.0]) <= 4, its
    assert its[8.0, 8.0] >= 1.5 * its[8.0, 64.0] and its[10.0, 10.0] >= 2.5 * its[10.0, 100.0], its
    assert its[10.0, 10.0] >= 1.4 * its[8.0, 8.0], its


def test_sub_box_local_problem_is_the_whole_problems():
    """dd.sub_box (the oracle's stand-in for one subdomain of a problem too large to partition
    whole): on a 24x24x48 box with jittered 3x3x6 boxes and 2 layers, for a corner, an interior
    and the last box, the sub-box's ORAS local set maps (through integer vertex coordinates) onto
    the whole partition's set in the same order, the whole partition's owner of every edge
    interior to the box is that box, and the local matrices agree to rounding."""
    n, lengths, parts, layers = (24, 24, 48), (1.0, 1.0, 2.0), (3, 3, 6), 2
    cuts = (jittered_cuts(24, 3, 0.2, 0), jittered_cuts(24, 3, 0.2, 1), jittered_cuts(48, 6, 0.2, 2))
    k = xi = 6.0
    og = Mesh(*n, *lengths)
    whole = dd.Partition(og, *parts, layers, *cuts)
    h = np.array([L / c for L, c in zip(lengths, n)])
    for l in (0, 1 + 3 * (1 + 3 * 3), 53):
        m, part, lr, lo, hi, rlo = dd.sub_box(n, lengths, parts, layers, cuts, l)
        ijk = np.rint(m.xyz / h).astype(np.int64) + np.array(rlo)
        gv = ijk[:, 0] + (n[0] + 1) * (ijk[:, 1] + (n[1] + 1) * ijk[:, 2])
        a, b = gv[m.edge_vert[:, 0]], gv[m.edge_vert[:, 1]]
        assert np.all(a < b)
        gid = og.edge_index(a, b)
        s = part.oras_sets[lr]
        assert np.array_equal(whole.oras_sets[l], gid[s])
        inner = np.ones(len(s), bool)
        for end in (0, 1):
            c = ijk[m.edge_vert[s, end]]
            inner &= np.all((c > np.array(lo)) & (c < np.array(hi)), axis=1)
        assert inner.sum() > 0 and np.all(whole.owner[gid[s][inner]] == l)
        Al = dd.local_matrix(part, None, dd.ORAS, k, xi, lr)
        Ag = dd.local_matrix(whole, None, dd.ORAS, k, xi, l)
        assert abs(Al - Ag).max() <= 1e-13 * abs(Ag).max()


def _box_problem_on_own_mesh(m, cuts, box, k, xi, bc):
    """The local problem of box `box` of the cut planes, built independently of dd: a mesh of
    the box alone, its Galerkin matrix with the impedance term of eq:imp on its own boundary
    triangles (PEC variant: impedance only on the triangles inside the global box, identity rows
    on edges lying in a face of the global box), and the map of its edges to global edge ids
    through integer vertex coordinates.  Returns (global edge id, orientation sign) per box edge,
    the box matrix, and its impedance face mass over the interface triangles alone."""
    o = [int(cuts[a][box[a]]) for a in range(3)]
    nb = [int(cuts[a][box[a] + 1]) - o[a] for a in range(3)]
    h = [m.L[a] / m.n[a] for a in range(3)]
    sub = Mesh(*nb, *[nb[a] * h[a] for a in range(3)])
    ijk = np.rint(sub.xyz / np.array(h)).astype(np.int64) + np.array(o)
    nx, ny, _ = m.n
    gid = ijk[:, 0] + (nx + 1) * (ijk[:, 1] + (ny + 1) * ijk[:, 2])
    a, b = gid[sub.edge_vert[:, 0]], gid[sub.edge_vert[:, 1]]
    sign = np.where(a < b, 1.0, -1.0)
    eid = m.edge_index(np.minimum(a, b), np.maximum(a, b))

    def on_global_face(verts):  # all vertices on one boundary plane of the global box
        c = ijk[verts]  # (F, nv, 3)
        hit = np.zeros(verts.shape[0], dtype=bool)
        for ax in range(3):
            for plane in (0, m.n[ax]):
                hit |= np.all(c[:, :, ax] == plane, axis=1)
        return hit

    glob_face = on_global_face(sub.bface_vert)
    interface = sub.bface_vert[~glob_face]
    K, M, _ = fem.assemble_parts(sub, bfaces=np.zeros((0, 3), np.int64))
    _, _, Mb_if = fem.assemble_parts(sub, bfaces=interface)
    if bc == fem.BC_IMPEDANCE:
        As = fem.assemble(sub, k, xi, fem.BC_IMPEDANCE)  # eq:imp on every face of the box
    else:
        As = (K - (k * k + 1j * xi) * M - 1j * fem.impedance_sign(xi) * k * Mb_if).tocsr()
        pec = on_global_face(sub.edge_vert)
        keep = sp.diags((~pec).astype(np.float64))
        As = (keep @ As @ keep + sp.diags(pec.astype(np.float64))).tocsr()
    return eid, sign, As, Mb_if


@pytest.mark.parametrize("bc,box", [(fem.BC_IMPEDANCE, (1, 1, 1)), (fem.BC_IMPEDANCE, (0, 0, 0)),
                                    (fem.BC_IMPEDANCE, (2, 1, 0)), (fem.BC_PEC, (0, 0, 0)),
                                    (fem.BC_PEC, (1, 2, 1))])
def test_oras_local_matrix_is_the_box_impedance_problem(bc, box):
    """ImpRAS (Sec. 6.3): the local problem of Omega_l carries the impedance condition of eq:imp
    (coefficient k) on the faces of dOmega_l inside Omega, and the global condition on the faces
    of dOmega.  With no overlap layers a subdomain is a box of cubes, and its local matrix must
    then equal the Galerkin matrix of that box assembled on a mesh of its own, with the
    impedance term on the box's own boundary triangles (interior box: every face an interface;
    corner and edge boxes: interface and global faces mixed; PEC: global faces stay PEC).  The
    two are matched through vertex coordinates and (lo, hi) edge keys.  A coefficient other than
    k on the interface faces (0.7k, 1.5k, 2k) changes the matrix by far more than the bar."""
    m = Mesh(7, 8, 6)
    cuts = ([0, 2, 5, 7], [0, 3, 5, 8], [0, 2, 4, 6])
    k, xi = 3.0, 5.0
    A = fem.assemble(m, k, xi, bc)
    part = dd.Partition(m, 3, 3, 3, 0, *cuts)
    l = box[0] + 3 * (box[1] + 3 * box[2])
    Al = dd.local_matrix(part, A, dd.ORAS, k, xi, l, bc).tocsr()
    eid, sign, As, Mb_if = _box_problem_on_own_mesh(m, cuts, box, k, xi, bc)
    idx = part.oras_sets[l]
    assert len(idx) == len(eid)  # the ORAS DOFs are exactly the edges of the box
    pos = np.searchsorted(idx, eid)
    assert np.array_equal(idx[pos], eid)
    S = sp.csr_matrix((sign, (pos, np.arange(len(eid)))), shape=(len(idx), len(eid)))
    mapped = (S @ As @ S.T).tocsr()
    scale = abs(Al).max()
    assert abs(Al - mapped).max() <= 1e-12 * scale
    # sensitivity: the interface term is resolved far above the bar
    Mif = (S @ Mb_if @ S.T).tocsr()
    assert Mif.nnz > 0
    for factor in (0.7, 1.5, 2.0):
        assert abs((factor - 1.0) * k * Mif).max() > 1e6 * 1e-12 * scale


@pytest.mark.parametrize("kind,bc,cuts", [("oras", fem.BC_IMPEDANCE, False), ("as", fem.BC_IMPEDANCE, True),
                                          ("ras", fem.BC_PEC, True), ("oras", fem.BC_PEC, False)])
def test_pooled_schwarz_equals_serial(kind, bc, cuts):
    """The worker-pool form of the oracle's Schwarz preconditioner (local problems factored and
    solved in separate processes, summed in subdomain order here) returns exactly what the
    one-process form returns."""
    from oracle import pool
    n, parts, k, xi = (8, 7, 6), (3, 2, 2), 4.0, 7.0
    c = (jittered_cuts(8, 3, 0.2, 1), jittered_cuts(7, 2, 0.2, 2), None) if cuts else (None, None, None)
    m = Mesh(*n)
    A = fem.assemble(m, k, xi, bc)
    P = dd.Partition(m, *parts, 2, *c)
    K = {"as": dd.AS, "ras": dd.RAS, "oras": dd.ORAS}[kind]
    ref = dd.Schwarz(P, A, K, k, xi, bc)
    v = random_rhs(m.n_edge, 3)
    with pool.PooledSchwarz(P, A, K, k, xi, bc, workers=3) as B:
        assert len(B.procs) == 3 and len(B.t_lu) == P.N
        for _ in range(2):
            assert np.array_equal(B(v), ref(v))


def test_local_factor_is_exact():
    """The oracle's local factorisation (symmetric minimum-degree order, diagonal pivots) solves
    the local problems to rounding: against a dense solve on small subdomains of every kind, and
    against SuperLU with partial pivoting in its default column order."""
    m = Mesh(6, 5, 4)
    for bc in (fem.BC_IMPEDANCE, fem.BC_PEC):
        A = fem.assemble(m, 3.0, 9.0, bc)
        P = dd.Partition(m, 2, 2, 1, 1)
        for K in (dd.AS, dd.ORAS):
            for l in range(P.N):
                Al = dd.local_matrix(P, A, K, 3.0, 9.0, l, bc)
                r = random_rhs(Al.shape[0], l)
                x = dd.factor_local(Al).solve(r)
                xd = np.linalg.solve(Al.toarray(), r)
                xp = spla.splu(Al).solve(r)
                assert np.linalg.norm(x - xd) <= 1e-12 * np.linalg.norm(xd)
                assert np.linalg.norm(x - xp) <= 1e-12 * np.linalg.norm(xp)
                assert np.linalg.norm(Al @ x - r) <= 1e-12 * np.linalg.norm(r)


@pytest.mark.parametrize("flexible", [False, True])
def test_weighted_gmres_minimal_residual_brute_force(flexible):
    """Weighted GMRES (Sec. 5.2): x_m minimises ||b - A x||_D over x0 + M^-1 K_m(A M^-1, r0) for a
    Hermitian positive definite D, checked for every m against an explicit Krylov basis and a
    dense least-squares solve in the Cholesky-transformed norm ||L^H r||_2 (D = L L^H); the
    residual estimates are the D-norms of the residuals.  The Euclidean minimiser differs."""
    rng = np.random.default_rng(16)
    n = 24
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)) + 6 * np.eye(n)
    Minv = np.linalg.inv(A + 0.5 * rng.standard_normal((n, n)))
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    G = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    D = G @ G.conj().T + 0.5 * np.eye(n)
    L = np.linalg.cholesky(D)
    C = A @ Minv
    dn = lambda r: np.linalg.norm(L.conj().T @ r)
    for msteps in range(1, 9):
        res = gmres.gmres(A, b, lambda v: Minv @ v, restart=30, fixed_iters=msteps,
                          flexible=flexible, D=D)
        Kb = np.stack([np.linalg.matrix_power(C, j) @ b for j in range(msteps)], axis=1)
        Q, _ = np.linalg.qr(Kb)
        c, *_ = np.linalg.lstsq(L.conj().T @ (C @ Q), L.conj().T @ b, rcond=None)
        x_ref = Minv @ (Q @ c)
        assert np.linalg.norm(res.x - x_ref) < 1e-9 * np.linalg.norm(x_ref)
        assert res.iters == msteps
        assert abs(res.history[-1] - dn(b - A @ x_ref) / dn(b)) < 1e-9
        if msteps >= 3:
            c2, *_ = np.linalg.lstsq(C @ Q, b, rcond=None)
            assert np.linalg.norm(Minv @ (Q @ c2) - x_ref) > 1e-6 * np.linalg.norm(x_ref)


def test_weighted_gmres_identity_weight_and_restarts():
    """With D = I the weighted method reproduces the standard iterates (to rounding); with the
    finite-element weight D_k on a preconditioned Maxwell problem it converges in the D_k-norm,
    across restarts, with the true D-norm residual below rtol."""
    m = Mesh(6, 6, 6)
    k, xi = 4.0, 16.0
    A = fem.assemble(m, k, xi)
    P = dd.Partition(m, 2, 2, 2, 2)
    B = dd.Schwarz(P, A, dd.ORAS, k, xi)
    f = random_rhs(m.n_edge, 9)
    std = gmres.gmres(A, f, B, restart=3, rtol=1e-8)
    ide = gmres.gmres(A, f, B, restart=3, rtol=1e-8, D=sp.identity(m.n_edge, format="csr"))
    assert ide.iters == std.iters and ide.cycles == std.cycles
    assert np.linalg.norm(ide.x - std.x) <= 1e-12 * np.linalg.norm(std.x)
    Dk = fem.weight_matrix(m, k)
    wgt = gmres.gmres(A, f, B, restart=3, rtol=1e-8, D=Dk)
    dn = lambda r: np.sqrt(np.real(np.vdot(r, Dk @ r)))
    assert wgt.converged and wgt.cycles > 1
    assert dn(f - A @ wgt.x) <= 1e-8 * dn(f)
    assert abs(wgt.relres_true - dn(f - A @ wgt.x) / dn(f)) <= 1e-12
    assert abs(wgt.iters - std.iters) <= max(2, std.iters // 5)  # Sec. 6.2: little difference
