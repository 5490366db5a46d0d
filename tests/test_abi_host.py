"""Host logic of the C-ABI library against the oracle (no GPU): the library loads and exports
every symbol of include/mx.h; integer work (mesh, edges, partition, owners, RCM orders,
envelopes) is bit-exact and assembled values agree to rounding."""
import os
import re

import numpy as np
import pytest
import scipy.sparse as sp

from mx_inputs import jittered_cuts
from oracle import dd, fem, rcm
from oracle.mesh import Mesh as OMesh
from paper_1711_03789_amd import mx

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_exports_every_declared_symbol():
    lib = mx.load()
    with open(os.path.join(ROOT, "include", "mx.h")) as fh:
        text = fh.read()
    declared = set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(mx_\w+)\s*\(", text, re.M))
    assert declared, "no declarations parsed"
    assert declared == set(mx.SYMBOLS)
    for name in declared:
        assert hasattr(lib, name), name


@pytest.mark.parametrize("n", [(1, 1, 1), (2, 3, 4), (8, 8, 8), (5, 3, 7)])
def test_mesh_bit_exact(n):
    om = OMesh(*n, 1.0, 0.7, 1.3)
    lm = mx.Mesh(*n, 1.0, 0.7, 1.3)
    e = lm.export()
    assert lm.n_edge == om.n_edge and lm.n_tet == om.n_tet and lm.n_vert == om.n_vert
    assert np.array_equal(e["tet_vert"], om.tet_vert)
    assert np.array_equal(e["edge_vert"], om.edge_vert)
    assert np.array_equal(e["tet_edge"], om.tet_edge)
    assert np.array_equal(e["tet_edge_sign"], om.tet_edge_sign)
    assert np.array_equal(np.sort(e["bface_vert"].view("i4,i4,i4"), axis=0).view(np.int32),
                          np.sort(om.bface_vert.astype(np.int32).view("i4,i4,i4"), axis=0).view(np.int32))


def _csr(rp, col, val, n):
    return sp.csr_matrix((val, col, rp), shape=(n, n))


@pytest.mark.parametrize("bc", [mx.MX_BC_IMPEDANCE, mx.MX_BC_PEC])
@pytest.mark.parametrize("k,xi", [(4.0, 16.0), (3.0, -2.0), (4.0, 0.0)])
def test_matrix_matches_oracle(bc, k, xi):
    n = (4, 3, 5)
    om = OMesh(*n, 1.0, 0.8, 1.1)
    lm = mx.Mesh(*n, 1.0, 0.8, 1.1)
    A = mx.Matrix(None, lm, k, xi, bc)
    rp, col, val = A.export()
    Al = _csr(rp, col, val, A.n)
    Ao = fem.assemble(om, k, xi, bc)
    assert np.all(np.diff(rp) > 0)
    for i in range(A.n):  # columns sorted ascending
        assert np.all(np.diff(col[rp[i]:rp[i + 1]]) > 0)
    if bc == mx.MX_BC_IMPEDANCE:
        assert np.array_equal(rp, Ao.indptr) and np.array_equal(col, Ao.indices)
    diff = abs(Al - Ao).max()
    assert diff <= 1e-14 * abs(Ao).max()


@pytest.mark.parametrize("bc", [mx.MX_BC_IMPEDANCE, mx.MX_BC_PEC])
def test_rhs_matches_oracle(bc):
    n = (6, 5, 4)
    om = OMesh(*n)
    lm = mx.Mesh(*n)
    c, pol, s = (0.45, 0.5, 0.55), (0.3, -0.8, 0.52), 0.1
    fl = lm.rhs_gaussian(c, pol, s, bc)
    fo = fem.load_vector(om, fem.gaussian_source(c, pol, s), bc)
    assert np.abs(fl - fo).max() <= 1e-14 * np.abs(fo).max()


@pytest.mark.parametrize("case", ["even", "jitter", "layers0", "layers3"])
def test_partition_bit_exact(case):
    n, parts, layers, cuts = (12, 10, 9), (3, 2, 2), 2, (None, None, None)
    if case == "jitter":
        cuts = (jittered_cuts(12, 3, 0.2, 1), jittered_cuts(10, 2, 0.2, 2), jittered_cuts(9, 2, 0.2, 3))
    if case == "layers0":
        layers = 0
    if case == "layers3":
        layers = 3
    om = OMesh(*n)
    lm = mx.Mesh(*n)
    op = dd.Partition(om, *parts, layers, *cuts)
    lp = mx.Partition(lm, *parts, layers, *cuts)
    for kind, osets in (("oras", op.oras_sets), ("as", op.as_sets)):
        e = lp.export(kind)
        assert len(e["sets"]) == len(osets)
        for a, b in zip(e["sets"], osets):
            assert np.array_equal(a, b)
        assert np.array_equal(e["owner"], op.owner)
        assert np.array_equal(e["n_tet"], [int(m.sum()) for m in op.tet_masks])


@pytest.mark.parametrize("kind", ["oras", "as", "ras"])
@pytest.mark.parametrize("bc", [mx.MX_BC_IMPEDANCE, mx.MX_BC_PEC])
def test_local_problems_and_rcm(kind, bc):
    n, k, xi = (8, 8, 8), 4.0, 16.0
    okind = {"oras": dd.ORAS, "as": dd.AS, "ras": dd.RAS}[kind]
    om = OMesh(*n)
    lm = mx.Mesh(*n)
    op = dd.Partition(om, 2, 2, 2, 2)
    lp = mx.Partition(lm, 2, 2, 2, 2)
    Ao = fem.assemble(om, k, xi, bc)
    Al = mx.Matrix(None, lm, k, xi, bc)
    oloc = dd.local_matrices(op, Ao, okind, k, xi, bc)
    for l in (0, 3, 7):
        lp_ = mx.local_problem(lm, Al, lp, l, kind)
        nl = len(lp_["perm"])
        L = sp.csr_matrix((lp_["val"], lp_["col"], lp_["rowptr"]), shape=(nl, nl))
        O = oloc[l].tocsr()
        assert abs(L - O).max() <= 1e-13 * abs(O).max()
        P = dd.local_pattern(op, l, okind, bc)
        Lp = L.copy()
        Lp.data[:] = 1
        assert np.array_equal(Lp.indptr, P.indptr) and np.array_equal(Lp.indices, P.indices)
        perm = rcm.rcm(*rcm.pattern_graph(P))
        assert np.array_equal(lp_["perm"], perm)
        first = rcm.envelope(*rcm.pattern_graph(P), perm)
        assert np.array_equal(lp_["first"], first)


def test_rcm_jittered_medium():
    """A larger ORAS subdomain (16^3 mesh, jittered 3x2x2 boxes): RCM order bit-exact."""
    n = (16, 14, 12)
    cuts = (jittered_cuts(16, 3, 0.2, 7), jittered_cuts(14, 2, 0.2, 8), jittered_cuts(12, 2, 0.2, 9))
    om = OMesh(*n)
    lm = mx.Mesh(*n)
    op = dd.Partition(om, 3, 2, 2, 2, *cuts)
    lp = mx.Partition(lm, 3, 2, 2, 2, *cuts)
    Al = mx.Matrix(None, lm, 5.0, 5.0)
    for l in (0, 5, 11):
        P = dd.local_pattern(op, l, dd.ORAS)
        perm = rcm.rcm(*rcm.pattern_graph(P))
        lp_ = mx.local_problem(lm, Al, lp, l, "oras")
        assert np.array_equal(lp_["perm"], perm)


def test_errors_are_reported():
    with pytest.raises(mx.MxError) as ei:
        mx.Mesh(0, 2, 2)
    assert ei.value.code == mx.MX_EINVAL
    m = mx.Mesh(4, 4, 4)
    with pytest.raises(mx.MxError):
        mx.Partition(m, 2, 2, 2, 1, cx=[0, 3, 2])
    with pytest.raises(mx.MxError):
        mx.Partition(m, 5, 1, 1, 1)


def test_plan_needs_no_device():
    """The host half of the setup runs without a context (and so without a GPU): it returns the
    device footprint, is deterministic, and a planned preconditioner refuses to be used before it
    is materialised; bad schedule options are refused at planning time."""
    m = mx.Mesh(9, 8, 7)
    p = mx.Partition(m, 2, 2, 2, 2)
    A = mx.Matrix(None, m, 4.0, 16.0)
    sizes = set()
    for kind in ("oras", "as"):
        for prec in ("c128", "c64"):
            P1 = mx.Precond(None, A, m, p, kind, precision=prec, plan_only=True)
            P2 = mx.Precond(None, A, m, p, kind, precision=prec, plan_only=True)
            assert P1.device_bytes > 0 and P1.device_bytes == P2.device_bytes
            sizes.add(P1.device_bytes)
            with pytest.raises(mx.MxError):
                P1.apply(None, None)
    assert len(sizes) == 4  # kinds and precisions differ in footprint
    for bad in (dict(schedule=7), dict(schedule="lookahead", width=5)):
        with pytest.raises(mx.MxError) as ei:
            mx.Precond(None, A, m, p, "oras", plan_only=True, **bad)
        assert ei.value.code == mx.MX_EINVAL


def test_device_vectors_are_checked():
    """Device vectors are handed to kernels that index them up to the problem size, so the
    binding refuses anything but a contiguous GPU tensor of exactly complex128[n] bytes (a CPU
    tensor, a strided view, a short or long buffer) with MX_EINVAL; None reaches the library,
    which reports it."""
    import torch

    class GpuTensorStandIn:  # the attributes the check reads (there is no GPU here)
        is_cuda = True

        def __init__(self, numel, esize, contiguous=True):
            self._n, self._e, self._c = numel, esize, contiguous

        def is_contiguous(self):
            return self._c

        def numel(self):
            return self._n

        def element_size(self):
            return self._e

        def data_ptr(self):
            return 4096

    assert mx._dvec(None, 5, "v") is None
    assert mx._dvec(GpuTensorStandIn(5, 16), 5, "v") == 4096
    assert mx._dvec(GpuTensorStandIn(10, 8), 5, "v") == 4096  # any dtype of the right byte size
    bad = [GpuTensorStandIn(4, 16), GpuTensorStandIn(6, 16), GpuTensorStandIn(5, 8),
           GpuTensorStandIn(5, 16, contiguous=False), torch.zeros(5, dtype=torch.complex128)]
    for t in bad:
        with pytest.raises(mx.MxError) as ei:
            mx._dvec(t, 5, "v")
        assert ei.value.code == mx.MX_EINVAL


def test_export_sizes_are_checked():
    """A planned preconditioner exports each subdomain's reverse Cuthill-McKee order, equal to
    the host view of the same local problem; a buffer length other than the subdomain's DOF
    count is refused with MX_EINVAL before anything is written."""
    m = mx.Mesh(6, 5, 4)
    p = mx.Partition(m, 2, 2, 1, 2)
    A = mx.Matrix(None, m, 4.0, 16.0)
    for kind in ("oras", "as"):
        P = mx.Precond(None, A, m, p, kind, plan_only=True)
        for l in range(4):
            ref = mx.local_problem(m, A, p, l, kind)
            n = len(ref["perm"])
            perm, first = P.perm(l, n)
            assert np.array_equal(perm, ref["perm"]) and np.array_equal(first, ref["first"])
            for bad in (n - 1, n + 1):
                with pytest.raises(mx.MxError) as ei:
                    P.perm(l, bad)
                assert ei.value.code == mx.MX_EINVAL
            with pytest.raises(mx.MxError) as ei:
                P.diag(l, n)  # needs the factors on a device
            assert ei.value.code == mx.MX_EINVAL


def test_concurrent_host_threads():
    """Host halves of the library on several host threads at once (ctypes releases the GIL, so
    the calls overlap): each thread builds its own mesh, host matrix, partition and preconditioner
    plan, while all of them also plan from one shared mesh and partition, and every handle is
    destroyed on a thread other than the one that made it. Results equal a single-threaded run
    bit for bit."""
    import threading

    shared_m = mx.Mesh(7, 6, 5)
    shared_p = mx.Partition(shared_m, 2, 2, 1, 2)
    shared_A = mx.Matrix(None, shared_m, 3.0, 9.0)

    def work(seed):
        n = (5 + seed % 3, 4 + seed % 2, 6)
        m = mx.Mesh(*n)
        p = mx.Partition(m, 2, 1, 2, 1 + seed % 2)
        A = mx.Matrix(None, m, 2.0 + seed, (2.0 + seed) ** 2)
        out = {"own": (m, p, A)}
        for kind in ("oras", "as"):
            P = mx.Precond(None, A, m, p, kind, plan_only=True)
            Ps = mx.Precond(None, shared_A, shared_m, shared_p, kind, plan_only=True)
            ref = mx.local_problem(shared_m, shared_A, shared_p, 1, kind)
            perm, _ = Ps.perm(1, len(ref["perm"]))
            out[kind] = (P, Ps, P.device_bytes, Ps.device_bytes, perm, ref["perm"])
        return out

    serial = [work(s) for s in range(6)]
    results = [None] * 6
    errors = []

    def run(i):
        try:
            results[i] = work(i)
        except Exception as e:  # reported on the main thread
            errors.append(e)

    for _ in range(2):
        th = [threading.Thread(target=run, args=(i,)) for i in range(6)]
        for t in th:
            t.start()
        for t in th:
            t.join()
        assert not errors, errors
        for a, b in zip(serial, results):
            for kind in ("oras", "as"):
                assert a[kind][2] == b[kind][2] and a[kind][3] == b[kind][3]
                assert np.array_equal(a[kind][4], b[kind][4])
                assert np.array_equal(b[kind][4], b[kind][5])
        # destroy the handles made on the worker threads from other threads, concurrently
        doomed = results[:]
        results = [None] * 6

        def drop(i):
            doomed[i] = None

        th = [threading.Thread(target=drop, args=((i + 1) % 6,)) for i in range(6)]
        for t in th:
            t.start()
        for t in th:
            t.join()


def test_host_thread_pool_errors():
    """An error raised on one of the library's host worker threads (the per-subdomain host work of
    plans and setups) comes back as the entry point's status code on the calling thread, after
    every worker has been joined, instead of terminating the process; with no failure every item
    runs exactly once per pass."""
    for n in (0, 1, 7, 100, 5000):
        rc, ran = mx.selftest_host(n)
        assert rc == mx.MX_OK and ran == 2 * n
    for code in (mx.MX_EINVAL, mx.MX_ENOMEM):
        for n, at in ((1, 0), (64, 0), (64, 63), (5000, 2500)):
            rc, ran = mx.selftest_host(n, at, code)
            assert rc == code
            assert 0 <= ran < n  # the failing item never completes; the pass stops
            if code == mx.MX_EINVAL:
                assert "planted failure of item %d" % at in mx._lib.mx_last_error().decode()
    rc, _ = mx.selftest_host(10, -1, 123)
    assert rc == mx.MX_EINVAL


def test_medium_partition_and_orders_bit_exact():
    """The 32^3 problem with 4x4x4 subdomains and 2 layers: local DOF sets of both kinds and the
    owners of every subdomain, and the reverse Cuthill-McKee order and envelope of a corner, an
    edge, a face and an interior subdomain, equal the oracle's integer for integer."""
    from mx_inputs import config_medium
    w = config_medium()
    om, lm = OMesh(*w.n), mx.Mesh(*w.n)
    op = dd.Partition(om, *w.parts, w.layers)
    lp = mx.Partition(lm, *w.parts, w.layers)
    for kind, sets in (("oras", op.oras_sets), ("as", op.as_sets)):
        ex = lp.export(kind)
        assert len(ex["sets"]) == 64
        for l in range(64):
            assert np.array_equal(ex["sets"][l], sets[l]), (kind, l)
        assert np.array_equal(ex["owner"], op.owner)
    A = mx.Matrix(None, lm, w.k, w.xi)
    for l in (0, 1, 5, 21):  # corner, edge, face, interior box
        for kind in ("oras", "as"):
            lp_ = mx.local_problem(lm, A, lp, l, kind)
            g = rcm.pattern_graph(dd.local_pattern(op, l, {"oras": dd.ORAS, "as": dd.AS}[kind]))
            perm = rcm.rcm(*g)
            assert np.array_equal(lp_["perm"], perm), (kind, l)
            assert np.array_equal(lp_["first"], rcm.envelope(*g, perm)), (kind, l)


@pytest.mark.parametrize("n,ratio,bc", [((8, 8, 8), 2, mx.MX_BC_IMPEDANCE), ((8, 8, 8), 4, mx.MX_BC_PEC),
                                        ((12, 6, 9), 3, mx.MX_BC_IMPEDANCE), ((6, 4, 8), 2, mx.MX_BC_PEC)])
def test_coarse_operators_match_oracle(n, ratio, bc):
    """The library's coarse restriction R^0 (closed form on the Kuhn split) and coarse Galerkin
    matrix R^0 A R^0^T equal the oracle's (generic barycentric search) to rounding; with PEC the
    boundary coarse edges have empty R^0 rows and unit A^0 rows."""
    from oracle import coarse
    lengths = (1.0, 0.9, 1.2)
    om, lm = OMesh(*n, *lengths), mx.Mesh(*n, *lengths)
    for k, xi in ((4.0, 16.0), (3.0, -2.0)):
        A = mx.Matrix(None, lm, k, xi, bc)
        R, A0 = mx.coarse_operators(lm, A, ratio)
        oc = coarse.coarse_mesh(om, ratio)
        oR = coarse.restriction(om, oc, bc)
        keep = coarse.coarse_dofs(oc, bc)
        assert R.shape == (oc.n_edge, om.n_edge)
        assert abs(R[keep] - oR).max() <= 1e-14 * abs(oR).max()
        oA0 = (oR @ fem.assemble(om, k, xi, bc) @ oR.T).tocsr()
        assert abs(A0[keep][:, keep] - oA0).max() <= 1e-13 * abs(oA0).max()
        drop = np.setdiff1d(np.arange(oc.n_edge), keep)
        assert R[drop].count_nonzero() == 0
        assert abs(A0[drop] - sp.identity(oc.n_edge).tocsr()[drop]).max() == 0 if len(drop) else True
    with pytest.raises(mx.MxError):
        mx.coarse_operators(lm, A, 5)


@pytest.mark.parametrize("bc", [mx.MX_BC_IMPEDANCE, mx.MX_BC_PEC])
def test_weight_matrix_matches_oracle(bc):
    """D_k = K + k^2 M (eq:ip, eq:weight) assembled by the library equals the oracle's."""
    n = (5, 4, 6)
    om, lm = OMesh(*n), mx.Mesh(*n)
    for k in (0.0, 4.0, 9.5):
        D = mx.Matrix.weight(None, lm, k, bc)
        rp, col, val = D.export()
        L = sp.csr_matrix((val, col, rp), shape=(D.n, D.n))
        O = fem.weight_matrix(om, k, bc)
        assert not np.any(val.imag)
        assert abs(L - O).max() <= 1e-14 * abs(O).max()


@pytest.mark.parametrize("bc", [mx.MX_BC_IMPEDANCE, mx.MX_BC_PEC])
def test_coarse_operators_non_nested_match_oracle(bc):
    """Coarse box meshes that are not nested in the fine one: the library's R^0 (nq-point Gauss
    rule per fine edge, closed-form point location in the Kuhn split) and A^0 equal the oracle's
    (generic barycentric search); on a nested mesh the quadrature gives the midpoint values."""
    from oracle import coarse
    L = (1.0, 0.9, 1.2)
    n, cn = (7, 5, 6), (3, 2, 4)
    om, lm = OMesh(*n, *L), mx.Mesh(*n, *L)
    k, xi = 4.0, 4.0
    A = mx.Matrix(None, lm, k, xi, bc)
    oA = fem.assemble(om, k, xi, bc)
    oc = coarse.coarse_box_mesh(om, cn)
    keep = coarse.coarse_dofs(oc, bc)
    for nq in (3, 12):
        R, A0 = mx.coarse_operators(lm, A, box=cn, nq=nq)
        oR = coarse.restriction_quadrature(om, oc, bc, nq)
        assert R.shape == (oc.n_edge, om.n_edge)
        assert abs(R[keep] - oR).max() <= 1e-13 * abs(oR).max()
        oA0 = (oR @ oA @ oR.T).tocsr()
        assert abs(A0[keep][:, keep] - oA0).max() <= 1e-12 * abs(oA0).max()
    # nested mesh through the quadrature entry: the exact midpoint values
    n2 = (6, 4, 8)
    lm2 = mx.Mesh(*n2, *L)
    A2 = mx.Matrix(None, lm2, k, xi, bc)
    Rn, _ = mx.coarse_operators(lm2, A2, ratio=2)
    Rq, _ = mx.coarse_operators(lm2, A2, box=(3, 2, 4), nq=5)
    assert abs(Rq - Rn).max() <= 1e-14 * abs(Rn).max()
    # order 2 needs the nested mesh
    A3 = mx.Matrix(None, lm2, k, xi, bc, order=2)
    with pytest.raises(mx.MxError):
        mx.coarse_operators(lm2, A3, box=(3, 2, 4), nq=5)
    with pytest.raises(mx.MxError):
        mx.coarse_operators(lm, A, box=(3, 2, 4), nq=0)


@pytest.mark.parametrize("seed", range(4))
def test_randomised_coarse_box_operators(seed):
    """Seeded random fine and coarse boxes (coarser or finer, nested or not), quadrature orders
    and boundary conditions: the library's R^0 and A^0 equal the oracle's."""
    from oracle import coarse
    rng = np.random.default_rng(200 + seed)
    n = tuple(int(v) for v in rng.integers(2, 7, 3))
    cn = tuple(int(v) for v in rng.integers(1, 5, 3))
    L = tuple(float(v) for v in rng.uniform(0.5, 1.5, 3))
    nq = int(rng.integers(1, 13))
    bc = int(rng.integers(0, 2))
    k, xi = float(rng.uniform(1, 6)), float(rng.uniform(0.5, 20))
    om, lm = OMesh(*n, *L), mx.Mesh(*n, *L)
    A = mx.Matrix(None, lm, k, xi, bc)
    R, A0 = mx.coarse_operators(lm, A, box=cn, nq=nq)
    oc = coarse.coarse_box_mesh(om, cn)
    keep = coarse.coarse_dofs(oc, bc)
    oR = coarse.restriction_quadrature(om, oc, bc, nq)
    if oR.nnz == 0:
        assert R[keep].count_nonzero() == 0
        return
    assert abs(R[keep] - oR).max() <= 1e-13 * abs(oR).max()
    oA0 = (oR @ fem.assemble(om, k, xi, bc) @ oR.T).tocsr()
    assert abs(A0[keep][:, keep] - oA0).max() <= 1e-12 * max(abs(oA0).max(), 1e-300)
