"""GPU parity of the two-level Schwarz preconditioners (Sec. 3.2, Sec. 3.3, Sec. 6.3) through the
C ABI against the oracle (oracle/coarse.py) on the same seeded inputs:
* the coarse restriction R^0 (eq:restriction) and the coarse Galerkin matrix A^0 = R^0 A R^0^T
  exported by the library equal the oracle's to rounding (PEC: on the coarse DOFs that carry a
  basis function);
* single applications of every form -- AS2 (eq:defAS), RAS2 (eq:RAS2), ImpRAS2, hybrid (eq:HRAS)
  and deflated (eq:ADEF1ras) with RAS and ImpRAS -- to 1e-10 relative;
* GMRES with the two-level forms: iterations within +-1 of the oracle's, and after exactly the
  oracle's iteration count the solution within 1e-8 relative L2;
* the same with coarse box meshes that are not nested in the fine one (R^0 by a 12-point Gauss
  rule along each fine edge)."""
import sys

import numpy as np
import pytest
import scipy.sparse as sp

from mx_inputs import random_rhs
from oracle import coarse, dd, fem, gmres
from oracle.mesh import Mesh as OMesh

pytestmark = pytest.mark.gpu

OKIND = {"oras": dd.ORAS, "ras": dd.RAS, "as": dd.AS}
COMB = {"additive": coarse.ADDITIVE, "hybrid": coarse.HYBRID, "deflation": coarse.DEFLATION}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, np.complex128)).cuda()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    return gpu_lib.Context(0)


class Case:
    def __init__(self, mx, ctx, n, parts, layers, k, xi, kind, ratio, combine, bc=fem.BC_IMPEDANCE,
                 precision="c128"):
        self.om = OMesh(*n)
        self.oA = fem.assemble(self.om, k, xi, bc)
        self.op = dd.Partition(self.om, *parts, layers)
        self.oc = coarse.coarse_mesh(self.om, ratio)
        self.oR = coarse.restriction(self.om, self.oc, bc)
        self.oB = coarse.TwoLevel(dd.Schwarz(self.op, self.oA, OKIND[kind], k, xi, bc), self.oA,
                                  self.oR, COMB[combine])
        self.lm = mx.Mesh(*n)
        self.lA = mx.Matrix(ctx, self.lm, k, xi, bc)
        self.lp = mx.Partition(self.lm, *parts, layers)
        self.lP = mx.Precond(ctx, self.lA, self.lm, self.lp, kind, precision=precision)
        self.lP.add_coarse(ctx, self.lA, self.lm, ratio, combine)
        self.E = self.om.n_edge
        self.bc = bc


@pytest.mark.parametrize("bc", [fem.BC_IMPEDANCE, fem.BC_PEC])
def test_coarse_operators_match_oracle(gpu_lib, ctx, bc):
    say("coarse R0 and A0 export", bc)
    c = Case(gpu_lib, ctx, (8, 8, 8), (2, 2, 2), 2, 4.0, 16.0, "oras", 2, "additive", bc)
    R, A0 = c.lP.coarse_export()
    keep = coarse.coarse_dofs(c.oc, bc)
    assert R.shape == (c.oc.n_edge, c.E) and A0.shape == (c.oc.n_edge, c.oc.n_edge)
    assert abs(R[keep] - c.oR).max() <= 1e-14 * abs(c.oR).max()
    oA0 = c.oB.A0.tocsr()
    assert abs(A0[keep][:, keep] - oA0).max() <= 1e-13 * abs(oA0).max()
    if bc == fem.BC_PEC:
        drop = np.setdiff1d(np.arange(c.oc.n_edge), keep)
        assert R[drop].count_nonzero() == 0
        assert abs(A0[drop][:, drop] - sp.identity(len(drop))).max() == 0


CASES = [("as", "additive"), ("ras", "additive"), ("oras", "additive"), ("ras", "hybrid"),
         ("oras", "hybrid"), ("ras", "deflation"), ("oras", "deflation")]


@pytest.mark.parametrize("kind,combine", CASES)
def test_two_level_apply(gpu_lib, ctx, kind, combine):
    say("two-level apply", kind, combine)
    c = Case(gpu_lib, ctx, (12, 12, 12), (3, 3, 3), 2, 5.0, 5.0, kind, 3, combine)
    v = random_rhs(c.E, 11)
    vd, zd = dev(v), dev(np.zeros(c.E))
    c.lP.apply(vd, zd)
    c.lP.check()
    z = host(zd)
    ref = c.oB(v)
    err = np.linalg.norm(z - ref) / np.linalg.norm(ref)
    say("  rel err", err)
    assert err <= 1e-10
    zd2 = dev(np.zeros(c.E))
    c.lP.apply(vd, zd2)
    assert np.array_equal(host(zd2), z)


@pytest.mark.parametrize("kind,combine", CASES)
def test_two_level_gmres(gpu_lib, ctx, kind, combine):
    say("two-level GMRES", kind, combine)
    c = Case(gpu_lib, ctx, (16, 16, 16), (4, 4, 4), 2, 6.0, 6.0, kind, 2, combine)
    f = random_rhs(c.E, 12)
    ores = gmres.gmres(c.oA, f, c.oB, restart=100, rtol=1e-6)
    bd, xd = dev(f), dev(np.zeros(c.E))
    st = gpu_lib.gmres(ctx, c.lA, c.lP, bd, xd, restart=100, rtol=1e-6)
    say("  iterations gpu", st["iters"], "oracle", ores.iters)
    assert st["converged"] and abs(st["iters"] - ores.iters) <= 1
    xd2 = dev(np.zeros(c.E))
    gpu_lib.gmres(ctx, c.lA, c.lP, bd, xd2, restart=100, fixed_iters=ores.iters)
    err = np.linalg.norm(host(xd2) - ores.x) / np.linalg.norm(ores.x)
    say("  rel L2 at the oracle's count", err)
    assert err <= 1e-8


def test_two_level_refusals(gpu_lib, ctx):
    mx = gpu_lib
    lm = mx.Mesh(6, 6, 6)
    lA = mx.Matrix(ctx, lm, 4.0, 16.0)
    lp = mx.Partition(lm, 2, 2, 2, 1)
    P = mx.Precond(ctx, lA, lm, lp, "oras")
    other = mx.Matrix(ctx, lm, 4.0, 8.0)
    for args in ((lA, lm, 4, "additive"), (lA, lm, 0, "additive"), (other, lm, 2, "additive")):
        with pytest.raises(mx.MxError) as ei:
            P.add_coarse(ctx, *args)
        assert ei.value.code == mx.MX_EINVAL
    P.add_coarse(ctx, lA, lm, 2, "hybrid")
    with pytest.raises(mx.MxError):
        P.add_coarse(ctx, lA, lm, 3, "hybrid")


def test_two_level_planned_on_another_thread(gpu_lib, ctx):
    """The host half of the coarse level (mx_precond_plan_coarse), made on a planned one-level
    preconditioner on a second host thread, then completed by mx_precond_add_coarse, gives the
    same two-level preconditioner bit for bit as the one-call path; before completion the
    preconditioner is refused."""
    import threading
    mx = gpu_lib
    n, parts = (12, 12, 12), (3, 3, 3)
    lm = mx.Mesh(*n)
    lp = mx.Partition(lm, *parts, 2)
    A = mx.Matrix(ctx, lm, 5.0, 5.0)
    ref = mx.Precond(ctx, A, lm, lp, "oras")
    ref.add_coarse(ctx, A, lm, 3, "deflation")
    out = {}

    def prepare():
        try:
            P = mx.Precond(None, A, lm, lp, "oras", plan_only=True)
            P.plan_coarse(A, lm, 3, "deflation")
            out["P"] = P
        except Exception as e:
            out["err"] = e

    th = threading.Thread(target=prepare)
    th.start()
    th.join()
    assert "err" not in out, out.get("err")
    P = out["P"]
    P.materialize(ctx)
    v = random_rhs(lm.n_edge, 41)
    vd, z1, z2 = dev(v), dev(np.zeros(lm.n_edge)), dev(np.zeros(lm.n_edge))
    with pytest.raises(mx.MxError):
        P.apply(vd, z2)
    with pytest.raises(mx.MxError):
        P.add_coarse(ctx, A, lm, 3, "hybrid")  # differs from the plan
    P.add_coarse(ctx, A, lm, 3, "deflation")
    ref.apply(vd, z1)
    P.apply(vd, z2)
    assert np.array_equal(host(z1), host(z2))


class BoxCase:
    """Two-level with a coarse box mesh that is not nested in the fine one (R^0 by a 12-point
    Gauss rule per fine edge)."""

    def __init__(self, mx, ctx, n, parts, layers, k, xi, kind, cn, combine, nq=12):
        self.om = OMesh(*n)
        self.oA = fem.assemble(self.om, k, xi)
        op = dd.Partition(self.om, *parts, layers)
        oc = coarse.coarse_box_mesh(self.om, cn)
        oR = coarse.restriction_quadrature(self.om, oc, fem.BC_IMPEDANCE, nq)
        self.oB = coarse.TwoLevel(dd.Schwarz(op, self.oA, OKIND[kind], k, xi), self.oA, oR,
                                  COMB[combine])
        self.lm = mx.Mesh(*n)
        self.lA = mx.Matrix(ctx, self.lm, k, xi)
        self.lP = mx.Precond(ctx, self.lA, self.lm, mx.Partition(self.lm, *parts, layers), kind)
        self.lP.add_coarse(ctx, self.lA, self.lm, combine=combine, box=cn, nq=nq)
        self.E = self.om.n_edge


@pytest.mark.parametrize("combine", ["additive", "hybrid", "deflation"])
def test_two_level_non_nested_apply(gpu_lib, ctx, combine):
    say("two-level apply, non-nested coarse mesh", combine)
    c = BoxCase(gpu_lib, ctx, (12, 12, 12), (3, 3, 3), 2, 5.0, 5.0, "oras", (5, 5, 5), combine)
    v = random_rhs(c.E, 13)
    vd, zd = dev(v), dev(np.zeros(c.E))
    c.lP.apply(vd, zd)
    c.lP.check()
    z = host(zd)
    ref = c.oB(v)
    err = np.linalg.norm(z - ref) / np.linalg.norm(ref)
    say("  rel err", err)
    assert err <= 1e-10


@pytest.mark.parametrize("kind,combine", [("oras", "hybrid"), ("ras", "deflation")])
def test_two_level_non_nested_gmres(gpu_lib, ctx, kind, combine):
    say("two-level GMRES, non-nested coarse mesh", kind, combine)
    c = BoxCase(gpu_lib, ctx, (16, 16, 16), (4, 4, 4), 2, 6.0, 6.0, kind, (7, 7, 7), combine)
    f = random_rhs(c.E, 14)
    ores = gmres.gmres(c.oA, f, c.oB, restart=100, rtol=1e-6)
    bd, xd = dev(f), dev(np.zeros(c.E))
    st = gpu_lib.gmres(ctx, c.lA, c.lP, bd, xd, restart=100, rtol=1e-6)
    say("  iterations gpu", st["iters"], "oracle", ores.iters)
    assert st["converged"] and abs(st["iters"] - ores.iters) <= 1
    xd2 = dev(np.zeros(c.E))
    gpu_lib.gmres(ctx, c.lA, c.lP, bd, xd2, restart=100, fixed_iters=ores.iters)
    err = np.linalg.norm(host(xd2) - ores.x) / np.linalg.norm(ores.x)
    say("  rel L2 at the oracle's count", err)
    assert err <= 1e-8
