"""Host logic of the library's second-order Nedelec space (Sec. 2.2 with order 2) against the
oracle (oracle/order2.py), no GPU: the DOF numbering (faces, their tetrahedra, boundary flags),
the local DOF sets and Boolean owners are bit-exact; the assembled matrix, the AS/RAS minors, the
ORAS local impedance problems and the coarse operators agree to rounding, for both boundary
conditions, on boxes with unequal sides and partitions with unequal cuts."""
import numpy as np
import pytest
import scipy.sparse as sp

from mx_inputs import jittered_cuts
from oracle import coarse, dd, fem, order2
from oracle.mesh import Mesh as OMesh
from paper_1711_03789_amd import mx

LENGTHS = (1.0, 0.8, 1.1)


def _csr(A):
    rp, col, val = A.export()
    return sp.csr_matrix((val, col, rp), shape=(A.n, A.n))


@pytest.mark.parametrize("n", [(1, 1, 1), (3, 2, 4), (4, 4, 3)])
def test_numbering_bit_exact(n):
    om, lm = OMesh(*n, *LENGTHS), mx.Mesh(*n, *LENGTHS)
    S = order2.Space(om)
    info = lm.order2()
    assert info["n_face"] == S.F and info["n_dof"] == S.n == 2 * om.n_edge + 2 * S.F
    assert np.array_equal(info["face_vert"], S.face_vert)
    assert np.array_equal(info["tet_face"], om.tet_face)
    assert np.array_equal(info["dof_boundary"], S.boundary_dof_mask())


@pytest.mark.parametrize("bc", [mx.MX_BC_IMPEDANCE, mx.MX_BC_PEC])
def test_matrix_matches_oracle(bc):
    n = (3, 4, 2)
    om, lm = OMesh(*n, *LENGTHS), mx.Mesh(*n, *LENGTHS)
    S = order2.Space(om)
    for k, xi in ((4.0, 16.0), (3.0, -2.0), (2.5, 0.0)):
        L = _csr(mx.Matrix(None, lm, k, xi, bc, order=2))
        O = order2.assemble(S, k, xi, bc)
        assert abs(L - O).max() <= 1e-14 * abs(O).max()
    # the lowest-order matrix is the leading block (Whitney functions first)
    A1 = _csr(mx.Matrix(None, lm, 4.0, 16.0, bc))
    A2 = _csr(mx.Matrix(None, lm, 4.0, 16.0, bc, order=2))
    E = om.n_edge
    assert abs(A2[:E, :E] - A1).max() <= 1e-14 * abs(A1).max()


def test_order_rejected():
    lm = mx.Mesh(2, 2, 2)
    with pytest.raises(mx.MxError):
        mx.Matrix(None, lm, 3.0, 1.0, order=3)


@pytest.mark.parametrize("bc", [mx.MX_BC_IMPEDANCE, mx.MX_BC_PEC])
def test_sets_owners_and_local_problems(bc):
    n = (6, 5, 4)
    om, lm = OMesh(*n, *LENGTHS), mx.Mesh(*n, *LENGTHS)
    S = order2.Space(om)
    cx, cy, cz = jittered_cuts(n[0], 3, 0.3, 3), jittered_cuts(n[1], 2, 0.3, 4), jittered_cuts(n[2], 1, 0.3, 5)
    op = dd.Partition(om, 3, 2, 1, 1, cx, cy, cz)
    lp = mx.Partition(lm, 3, 2, 1, 1, cx, cy, cz)
    p2 = order2.Partition(S, op)
    k, xi = 5.0, 25.0
    A = mx.Matrix(None, lm, k, xi, bc, order=2)
    oA = order2.assemble(S, k, xi, bc)
    for kind, okind in (("as", dd.AS), ("ras", dd.RAS), ("oras", dd.ORAS)):
        ex = lp.export_order2(lm, kind)
        assert np.array_equal(ex["owner"], p2.owner)
        for l in range(op.N):
            assert np.array_equal(ex["sets"][l], p2.local_set(okind)[l]), (kind, l)
            loc = mx.local_problem(lm, A, lp, l, kind=kind, xi_prec=xi)
            L = sp.csr_matrix((loc["val"], loc["col"], loc["rowptr"]), shape=(len(loc["perm"]),) * 2)
            O = order2.local_matrix(p2, oA, okind, k, xi, l, bc)
            assert abs(L - O).max() <= 1e-14 * abs(O).max(), (kind, l)
            assert np.array_equal(np.sort(loc["perm"]), np.arange(len(loc["perm"])))
    # ORAS at another absorption than the matrix's (xi_prec != xi_prob)
    A0 = mx.Matrix(None, lm, k, 0.0, bc, order=2)
    oA0 = order2.assemble(S, k, 0.0, bc)
    loc = mx.local_problem(lm, A0, lp, 2, kind="oras", xi_prec=k)
    L = sp.csr_matrix((loc["val"], loc["col"], loc["rowptr"]), shape=(len(loc["perm"]),) * 2)
    O = order2.local_matrix(p2, oA0, dd.ORAS, k, k, 2, bc)
    assert abs(L - O).max() <= 1e-14 * abs(O).max()


@pytest.mark.parametrize("bc", [mx.MX_BC_IMPEDANCE, mx.MX_BC_PEC])
def test_coarse_operators_order2(bc):
    """R^0 of the order-2 space is the lowest-order one followed by zero columns, and A^0 =
    R^0 A R^0^T with the order-2 A."""
    n = (4, 4, 6)
    om, lm = OMesh(*n, *LENGTHS), mx.Mesh(*n, *LENGTHS)
    S = order2.Space(om)
    k, xi = 4.0, 4.0
    A = mx.Matrix(None, lm, k, xi, bc, order=2)
    R, A0 = mx.coarse_operators(lm, A, 2)
    oc = coarse.coarse_mesh(om, 2)
    keep = coarse.coarse_dofs(oc, bc)
    oR = order2.coarse_restriction(S, oc, bc)
    assert R.shape == (oc.n_edge, S.n)
    assert abs(R[keep] - oR).max() <= 1e-14 * abs(oR).max()
    oA0 = (oR @ order2.assemble(S, k, xi, bc) @ oR.T).tocsr()
    assert abs(A0[keep][:, keep] - oA0).max() <= 1e-13 * abs(oA0).max()


@pytest.mark.parametrize("bc", [mx.MX_BC_IMPEDANCE, mx.MX_BC_PEC])
def test_weight_matrix_order2(bc):
    """D_k = K + k^2 M of the order-2 space equals the oracle's."""
    n = (3, 2, 3)
    om, lm = OMesh(*n, *LENGTHS), mx.Mesh(*n, *LENGTHS)
    S = order2.Space(om)
    for k in (0.0, 4.0):
        D = mx.Matrix.weight(None, lm, k, bc, order=2)
        L = _csr(D)
        O = order2.weight_matrix(S, k, bc)
        assert not np.any(L.data.imag)
        assert abs(L - O).max() <= 1e-14 * abs(O).max()


@pytest.mark.parametrize("seed", range(4))
def test_randomised_boxes_order2(seed):
    """Seeded random boxes (cube counts, side lengths, partitions with jittered cuts, layers,
    boundary condition, k and xi): the order-2 numbering, owners and sets bit-exact, and the
    matrix and one local problem of each kind equal to the oracle's to rounding."""
    rng = np.random.default_rng(100 + seed)
    n = tuple(int(v) for v in rng.integers(2, 6, 3))
    L = tuple(float(v) for v in rng.uniform(0.5, 1.5, 3))
    parts = tuple(int(min(v, c)) for v, c in zip(rng.integers(1, 3, 3), n))
    layers = int(rng.integers(0, 3))
    bc = int(rng.integers(0, 2))
    k, xi = float(rng.uniform(1, 6)), float(rng.uniform(-10, 30))
    cuts = [jittered_cuts(c, p, 0.3, seed + a) for a, (c, p) in enumerate(zip(n, parts))]
    om, lm = OMesh(*n, *L), mx.Mesh(*n, *L)
    S = order2.Space(om)
    assert np.array_equal(lm.order2()["face_vert"], S.face_vert)
    L2 = _csr(mx.Matrix(None, lm, k, xi, bc, order=2))
    O2 = order2.assemble(S, k, xi, bc)
    assert abs(L2 - O2).max() <= 1e-14 * abs(O2).max()
    op = dd.Partition(om, *parts, layers, *cuts)
    lp = mx.Partition(lm, *parts, layers, *cuts)
    p2 = order2.Partition(S, op)
    A = mx.Matrix(None, lm, k, xi, bc, order=2)
    l = int(rng.integers(0, op.N))
    for kind, okind in (("as", dd.AS), ("oras", dd.ORAS)):
        ex = lp.export_order2(lm, kind)
        assert np.array_equal(ex["owner"], p2.owner)
        for q in range(op.N):
            assert np.array_equal(ex["sets"][q], p2.local_set(okind)[q])
        if len(p2.local_set(okind)[l]) == 0:
            continue
        loc = mx.local_problem(lm, A, lp, l, kind=kind, xi_prec=xi)
        Lc = sp.csr_matrix((loc["val"], loc["col"], loc["rowptr"]), shape=(len(loc["perm"]),) * 2)
        Oc = order2.local_matrix(p2, O2, okind, k, xi, l, bc)
        assert abs(Lc - Oc).max() <= 1e-14 * max(abs(Oc).max(), 1.0)
