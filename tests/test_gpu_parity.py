"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle on the same seeded
inputs.  Tolerances: FP64 path 1e-8 relative L2 for GMRES solutions (at the oracle's iteration
count), iteration counts within +-1; single preconditioner applications and SpMV to rounding
(1e-10 / 1e-13); complex64 factors 1e-4 per application and 1e-5 for FGMRES solutions."""
import sys

import numpy as np
import pytest

from mx_inputs import config_small, jittered_cuts, random_rhs
from oracle import dd, fem, gmres
from oracle.mesh import Mesh as OMesh

pytestmark = pytest.mark.gpu

OKIND = {"oras": dd.ORAS, "ras": dd.RAS, "as": dd.AS}


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
    """A problem built on both sides from the same description."""

    def __init__(self, mx, ctx, n, parts, layers, k, xi, kind, cuts=(None, None, None),
                 bc=fem.BC_IMPEDANCE, precision="c128", lengths=(1.0, 1.0, 1.0), sweep_grid=0):
        self.om = OMesh(*n, *lengths)
        self.oA = fem.assemble(self.om, k, xi, bc)
        self.op = dd.Partition(self.om, *parts, layers, *cuts)
        self.oB = dd.Schwarz(self.op, self.oA, OKIND[kind], k, xi, bc)
        self.lm = mx.Mesh(*n, *lengths)
        self.lA = mx.Matrix(ctx, self.lm, k, xi, bc)
        self.lp = mx.Partition(self.lm, *parts, layers, *cuts)
        self.lP = mx.Precond(ctx, self.lA, self.lm, self.lp, kind, precision=precision,
                             sweep_grid=sweep_grid)
        self.E = self.om.n_edge


def test_selftest_matrix_cores(ctx):
    say("selftest")
    e64, e32 = ctx.selftest()
    say("mfma rel err", e64, e32)
    assert e64 < 1e-13 and e32 < 1e-5


@pytest.mark.parametrize("n", [(8, 8, 8), (5, 7, 3)])
def test_spmv(gpu_lib, ctx, n):
    say("spmv", n)
    om = OMesh(*n)
    A = fem.assemble(om, 4.0, 16.0)
    lm = gpu_lib.Mesh(*n)
    lA = gpu_lib.Matrix(ctx, lm, 4.0, 16.0)
    x = random_rhs(om.n_edge, 11)
    xd, yd = dev(x), dev(np.zeros(om.n_edge))
    lA.spmv(ctx, xd, yd)
    y = host(yd)
    ref = A @ x
    assert np.linalg.norm(y - ref) <= 1e-13 * np.linalg.norm(ref)


@pytest.mark.parametrize("kind,grid", [("oras", 0), ("ras", 0), ("as", 0), ("oras", 3), ("as", 1)])
def test_apply_config_small(gpu_lib, ctx, kind, grid):
    """grid 0: one sweep workgroup per compute unit; 3 and 1: few workgroups, so that most block
    rows are claimed late and a single workgroup walks the whole ticket order."""
    say("apply cfg small", kind, grid)
    c = Case(gpu_lib, ctx, (8, 8, 8), (2, 2, 2), 2, 4.0, 16.0, kind, sweep_grid=grid)
    v = random_rhs(c.E, 3)
    vd, zd = dev(v), dev(np.zeros(c.E))
    c.lP.apply(vd, zd)
    c.lP.check()
    z = host(zd)
    ref = c.oB(v)
    err = np.linalg.norm(z - ref) / np.linalg.norm(ref)
    say("  rel err", err)
    assert err <= 1e-10
    # repeated application is bitwise deterministic
    zd2 = dev(np.zeros(c.E))
    c.lP.apply(vd, zd2)
    assert np.array_equal(host(zd2), z)


@pytest.mark.parametrize("grid,precision", [(0, "c128"), (5, "c128"), (0, "c64"), (5, "c64")])
def test_apply_multi_tile_jittered(gpu_lib, ctx, grid, precision):
    """Uneven jittered boxes with several 64-row blocks per subdomain and ragged last blocks,
    two sweep grids and both factor precisions."""
    say("apply jittered", grid, precision)
    n = (16, 14, 12)
    cuts = (jittered_cuts(16, 3, 0.2, 7), jittered_cuts(14, 2, 0.2, 8), jittered_cuts(12, 2, 0.2, 9))
    c = Case(gpu_lib, ctx, n, (3, 2, 2), 2, 5.0, 5.0, "oras", cuts, precision=precision,
             sweep_grid=grid)
    info = c.lP.info()
    say("  info", info)
    assert info["max_blocks"] >= 20
    v = random_rhs(c.E, 4)
    vd, zd = dev(v), dev(np.zeros(c.E))
    c.lP.apply(vd, zd)
    c.lP.check()
    ref = c.oB(v)
    err = np.linalg.norm(host(zd) - ref) / np.linalg.norm(ref)
    say("  rel err", err)
    assert err <= (1e-10 if precision == "c128" else 1e-4)


def test_apply_pec_and_negative_xi(gpu_lib, ctx):
    say("apply pec")
    c = Case(gpu_lib, ctx, (6, 6, 6), (2, 2, 1), 1, 3.0, -9.0, "oras", bc=fem.BC_PEC)
    v = random_rhs(c.E, 5)
    vd, zd = dev(v), dev(np.zeros(c.E))
    c.lP.apply(vd, zd)
    c.lP.check()
    ref = c.oB(v)
    assert np.linalg.norm(host(zd) - ref) <= 1e-10 * np.linalg.norm(ref)


def test_apply_complex64(gpu_lib, ctx):
    say("apply c64")
    c = Case(gpu_lib, ctx, (8, 8, 8), (2, 2, 2), 2, 4.0, 16.0, "oras", precision="c64")
    v = random_rhs(c.E, 6)
    vd, zd = dev(v), dev(np.zeros(c.E))
    c.lP.apply(vd, zd)
    c.lP.check()
    ref = c.oB(v)
    err = np.linalg.norm(host(zd) - ref) / np.linalg.norm(ref)
    say("  rel err", err)
    assert err <= 1e-4


@pytest.mark.parametrize("kind", ["oras", "ras", "as"])
def test_gmres_config_small(gpu_lib, ctx, kind):
    """8^3, k = 4, xi = k^2, impedance, Gaussian source, 2x2x2 subdomains, 2 layers, GMRES(50)."""
    say("gmres cfg small", kind)
    w = config_small(kind)
    c = Case(gpu_lib, ctx, w.n, w.parts, w.layers, w.k, w.xi, kind)
    f = fem.load_vector(c.om, fem.gaussian_source(w.center, w.pol, w.sigma))
    fl = c.lm.rhs_gaussian(w.center, w.pol, w.sigma)
    assert np.abs(fl - f).max() <= 1e-14 * np.abs(f).max()
    ores = gmres.gmres(c.oA, f, c.oB, restart=w.restart, rtol=w.rtol)
    bd, xd = dev(f), dev(np.zeros(c.E))
    st = gpu_lib.gmres(ctx, c.lA, c.lP, bd, xd, restart=w.restart, rtol=w.rtol, history=True)
    say("  iters gpu", st["iters"], "oracle", ores.iters, "relres", st["relres_true"])
    assert st["converged"] and st["relres_true"] <= w.rtol
    assert abs(st["iters"] - ores.iters) <= 1
    # solution at the oracle's iteration count
    xd2 = dev(np.zeros(c.E))
    st2 = gpu_lib.gmres(ctx, c.lA, c.lP, bd, xd2, restart=w.restart, fixed_iters=ores.iters)
    x = host(xd2)
    err = np.linalg.norm(x - ores.x) / np.linalg.norm(ores.x)
    say("  fixed-iteration solution rel err", err)
    assert st2["iters"] == ores.iters
    assert err <= 1e-8


@pytest.mark.parametrize("kind", ["oras", "as"])
def test_gmres_absorption_only_in_preconditioner(gpu_lib, ctx, kind):
    """The problem without absorption (xi_prob = 0) preconditioned by the Schwarz method built
    with xi_prec = k (Sec. 1.2, eq. key_intro; Appendix B): the preconditioner is set up from the
    matrix assembled at xi_prec, GMRES multiplies by the matrix at xi_prob.  8^3, k = 4, 2x2x2
    subdomains, 2 layers, Gaussian source, GMRES(50): iterations within one of the oracle's, and
    the solution at the oracle's iteration count to 1e-8."""
    w = config_small(kind)
    k, xp = w.k, w.k
    say("gmres xi_prob 0, xi_prec k", kind)
    om = OMesh(*w.n, *w.lengths)
    oA0, oAp = fem.assemble(om, k, 0.0), fem.assemble(om, k, xp)
    op = dd.Partition(om, *w.parts, w.layers)
    oB = dd.Schwarz(op, oAp, OKIND[kind], k, xp)
    lm = gpu_lib.Mesh(*w.n, *w.lengths)
    lA0 = gpu_lib.Matrix(ctx, lm, k, 0.0)
    lAp = gpu_lib.Matrix(None, lm, k, xp)  # host only: the local problems are built from it
    lp = gpu_lib.Partition(lm, *w.parts, w.layers)
    lP = gpu_lib.Precond(ctx, lAp, lm, lp, kind, xi_prec=xp)
    f = fem.load_vector(om, fem.gaussian_source(w.center, w.pol, w.sigma))
    ores = gmres.gmres(oA0, f, oB, restart=w.restart, rtol=w.rtol)
    ores_same = gmres.gmres(oAp, f, oB, restart=w.restart, rtol=w.rtol)
    E = om.n_edge
    bd, xd = dev(f), dev(np.zeros(E))
    st = gpu_lib.gmres(ctx, lA0, lP, bd, xd, restart=w.restart, rtol=w.rtol)
    say("  iters gpu", st["iters"], "oracle", ores.iters, "(xi_prob = xi_prec:", ores_same.iters,
        ") relres", st["relres_true"])
    assert ores.converged and st["converged"] and st["relres_true"] <= w.rtol
    assert abs(st["iters"] - ores.iters) <= 1
    xd2 = dev(np.zeros(E))
    st2 = gpu_lib.gmres(ctx, lA0, lP, bd, xd2, restart=w.restart, fixed_iters=ores.iters)
    err = np.linalg.norm(host(xd2) - ores.x) / np.linalg.norm(ores.x)
    say("  fixed-iteration solution rel err", err)
    assert st2["iters"] == ores.iters and err <= 1e-8


@pytest.mark.parametrize("coarse_ratio", [0, 2])
def test_gmres_without_absorption_anywhere(gpu_lib, ctx, coarse_ratio):
    """xi_prob = xi_prec = 0, the setting of Table tab:EpsPrec0 (ImpRAS, and ImpHRAS with a
    coarse level): no coercivity bound guarantees the pivots of the unpivoted local
    factorisations here (a zero pivot would be reported as MX_EPIVOT), but the impedance
    condition on the subdomain boundaries keeps the ORAS local problems nonsingular.  8^3, k = 4,
    2x2x2 subdomains, 2 layers, Gaussian source, GMRES(50): iterations within one of the
    oracle's, the solution at the oracle's count to 1e-8."""
    from oracle import coarse
    w = config_small("oras")
    k = w.k
    say("gmres xi_prob = xi_prec = 0, coarse ratio", coarse_ratio)
    om = OMesh(*w.n, *w.lengths)
    oA = fem.assemble(om, k, 0.0)
    op = dd.Partition(om, *w.parts, w.layers)
    oB = dd.Schwarz(op, oA, dd.ORAS, k, 0.0)
    lm = gpu_lib.Mesh(*w.n, *w.lengths)
    lA = gpu_lib.Matrix(ctx, lm, k, 0.0)
    lp = gpu_lib.Partition(lm, *w.parts, w.layers)
    lP = gpu_lib.Precond(ctx, lA, lm, lp, "oras", xi_prec=0.0)
    if coarse_ratio:
        oB = coarse.TwoLevel(oB, oA, coarse.restriction(om, coarse.coarse_mesh(om, coarse_ratio)),
                             coarse.HYBRID)
        lP.add_coarse(ctx, lA, lm, coarse_ratio, "hybrid")
    f = fem.load_vector(om, fem.gaussian_source(w.center, w.pol, w.sigma))
    ores = gmres.gmres(oA, f, oB, restart=w.restart, rtol=w.rtol)
    E = om.n_edge
    bd, xd = dev(f), dev(np.zeros(E))
    st = gpu_lib.gmres(ctx, lA, lP, bd, xd, restart=w.restart, rtol=w.rtol)
    say("  iters gpu", st["iters"], "oracle", ores.iters, "relres", st["relres_true"])
    assert ores.converged and st["converged"] and st["relres_true"] <= w.rtol
    assert abs(st["iters"] - ores.iters) <= 1
    xd2 = dev(np.zeros(E))
    st2 = gpu_lib.gmres(ctx, lA, lP, bd, xd2, restart=w.restart, fixed_iters=ores.iters)
    err = np.linalg.norm(host(xd2) - ores.x) / np.linalg.norm(ores.x)
    say("  fixed-iteration solution rel err", err)
    assert st2["iters"] == ores.iters and err <= 1e-8


def test_gmres_restart_and_flexible(gpu_lib, ctx):
    """Small restart length (several cycles), flexible variant, nonzero initial guess."""
    say("gmres restart")
    c = Case(gpu_lib, ctx, (8, 6, 7), (2, 2, 1), 1, 3.0, 3.0, "ras")
    f = random_rhs(c.E, 9)
    x0 = random_rhs(c.E, 10) * 1e-3
    for flex in (False, True):
        ores = gmres.gmres(c.oA, f, c.oB, x0=x0, restart=5, rtol=1e-8, flexible=flex)
        xd = dev(x0)
        st = gpu_lib.gmres(ctx, c.lA, c.lP, dev(f), xd, restart=5, rtol=1e-8, flexible=flex)
        say("  flex", flex, "iters", st["iters"], ores.iters, "cycles", st["cycles"], ores.cycles)
        assert abs(st["iters"] - ores.iters) <= 1 and st["converged"]
        xd = dev(x0)
        gpu_lib.gmres(ctx, c.lA, c.lP, dev(f), xd, restart=5, fixed_iters=ores.iters, flexible=flex)
        err = np.linalg.norm(host(xd) - ores.x) / np.linalg.norm(ores.x)
        assert err <= 1e-8


def test_gmres_degenerate(gpu_lib, ctx):
    say("gmres degenerate")
    # one subdomain: B^-1 = A^-1, one iteration
    c = Case(gpu_lib, ctx, (5, 4, 4), (1, 1, 1), 2, 4.0, 4.0, "oras")
    f = random_rhs(c.E, 12)
    xd = dev(np.zeros(c.E))
    st = gpu_lib.gmres(ctx, c.lA, c.lP, dev(f), xd, restart=10, rtol=1e-10)
    assert st["iters"] == 1 and st["converged"]
    x = host(xd)
    assert np.linalg.norm(c.oA @ x - f) <= 1e-10 * np.linalg.norm(f)
    # zero right-hand side: converged with no iteration, x stays 0
    xd = dev(np.zeros(c.E))
    st = gpu_lib.gmres(ctx, c.lA, c.lP, dev(np.zeros(c.E)), xd)
    assert st["iters"] == 0 and st["converged"] and not host(xd).any()


def test_fgmres_mixed_precision_config(gpu_lib, ctx):
    """complex64 factors and complex64 SpMV values inside FP64 flexible GMRES: error against the
    FP64 oracle solution reported and bounded by 1e-5."""
    say("fgmres c64")
    w = config_small("oras", precision="c64")
    c = Case(gpu_lib, ctx, w.n, w.parts, w.layers, w.k, w.xi, "oras", precision="c64")
    f = fem.load_vector(c.om, fem.gaussian_source(w.center, w.pol, w.sigma))
    import scipy.sparse.linalg as spla
    x_exact = spla.spsolve(c.oA.tocsc(), f)
    ores = gmres.gmres(c.oA, f, c.oB, restart=w.restart, rtol=w.rtol)
    xd = dev(np.zeros(c.E))
    st = gpu_lib.gmres(ctx, c.lA, c.lP, dev(f), xd, restart=w.restart, rtol=w.rtol, flexible=True,
                       spmv_c64=True)
    x = host(xd)
    err = np.linalg.norm(x - ores.x) / np.linalg.norm(ores.x)
    say("  iters", st["iters"], "oracle", ores.iters, "err vs oracle", err,
        "err vs exact", np.linalg.norm(x - x_exact) / np.linalg.norm(x_exact))
    assert st["converged"] and st["relres_true"] <= w.rtol
    assert err <= 1e-5


def test_resident_share_and_autotune(gpu_lib, ctx):
    """A preconditioner built on a share of the subdomains returns the share's part of the sum
    (zero on DOFs owned elsewhere); the launch-shape tuner keeps the result bit-identical."""
    say("share")
    n = (14, 12, 16)
    cuts = (jittered_cuts(14, 2, 0.2, 21), jittered_cuts(12, 2, 0.2, 22), jittered_cuts(16, 3, 0.2, 23))
    k, xi = 4.0, 4.0
    om = OMesh(*n)
    oA = fem.assemble(om, k, xi)
    op = dd.Partition(om, 2, 2, 3, 2, *cuts)
    oB = dd.Schwarz(op, oA, dd.ORAS, k, xi)
    lm = gpu_lib.Mesh(*n)
    lA = gpu_lib.Matrix(ctx, lm, k, xi)
    lp = gpu_lib.Partition(lm, 2, 2, 3, 2, *cuts)
    s0, s1 = 4, 8  # the middle z-layer of boxes
    P = gpu_lib.Precond(ctx, lA, lm, lp, "oras", precision="c64", share=(s0, s1))
    v = random_rhs(om.n_edge, 31)
    ref = np.zeros(om.n_edge, np.complex128)
    for l in range(s0, s1):
        idx = op.oras_sets[l]
        ref[idx] += op.pou(l, dd.ORAS) * oB.lu[l].solve(v[idx])
    vd, zd = dev(v), dev(np.zeros(om.n_edge))
    P.apply(vd, zd)
    P.check()
    z = host(zd)
    err = np.linalg.norm(z - ref) / np.linalg.norm(ref)
    say("  share rel err (c64)", err)
    assert err <= 1e-4
    assert not z[(op.owner < s0) | (op.owner >= s1)].any()
    g, ms = P.autotune()
    say("  autotune grid", g, "ms", ms)
    zd2 = dev(np.zeros(om.n_edge))
    P.apply(vd, zd2)
    P.check()
    assert np.array_equal(host(zd2), z)


@pytest.mark.parametrize("kind,precision", [("oras", "c128"), ("as", "c128"), ("oras", "c64")])
def test_factor_pivots(gpu_lib, ctx, kind, precision):
    """The exported LDL^T pivots D of every local factor equal the pivots of an unpivoted LU
    (natural column order, no row exchanges) of the oracle's local matrix in the exported
    reverse Cuthill-McKee order: both are ratios of the same leading principal minors."""
    import scipy.sparse.linalg as spla
    say("factor pivots", kind, precision)
    c = Case(gpu_lib, ctx, (8, 8, 8), (2, 2, 2), 2, 4.0, 16.0, kind, precision=precision)
    tol = 1e-9 if precision == "c128" else 1e-4
    for l in range(c.op.N):
        Al = c.oB.local[l]
        n = Al.shape[0]
        perm, first = c.lP.perm(l, n)
        assert np.array_equal(np.sort(perm), np.arange(n))
        Ap = Al[perm][:, perm].tocsc()
        lu = spla.splu(Ap, permc_spec="NATURAL", diag_pivot_thresh=0.0,
                       options={"SymmetricMode": True})
        assert np.array_equal(lu.perm_r, np.arange(n)) and np.array_equal(lu.perm_c, np.arange(n))
        ref = lu.U.diagonal()
        d = c.lP.diag(l, n)
        err = np.max(np.abs(d - ref) / np.abs(ref))
        say("  sub", l, "n", n, "max rel pivot err", err)
        assert err <= tol
        # the envelope start of every row is its first nonzero column in the permuted matrix
        lower = sp_lower_first(Ap)
        assert np.array_equal(first, lower)


def sp_lower_first(Ap):
    """First nonzero column of each row of the lower triangle (diagonal included)."""
    C = Ap.tocsr()
    n = C.shape[0]
    out = np.arange(n, dtype=np.int32)
    for i in range(n):
        cols = C.indices[C.indptr[i]:C.indptr[i + 1]]
        if cols.size:
            out[i] = min(i, int(cols.min()))
    return out


def test_plan_then_materialize(gpu_lib, ctx):
    """The two halves of the setup (host plan on a host-only matrix, then device
    materialisation) give the same preconditioner, bit for bit, as the one-call setup; a planned
    preconditioner refuses to apply, and materialising twice is refused."""
    say("plan + materialize")
    n, parts = (9, 8, 7), (2, 2, 2)
    lm = gpu_lib.Mesh(*n)
    lp = gpu_lib.Partition(lm, *parts, 2)
    A_dev = gpu_lib.Matrix(ctx, lm, 4.0, 16.0)
    ref = gpu_lib.Precond(ctx, A_dev, lm, lp, "oras")
    A_host = gpu_lib.Matrix(None, lm, 4.0, 16.0)
    Pp = gpu_lib.Precond(ctx, A_host, lm, lp, "oras", plan_only=True)
    assert Pp.device_bytes > 0
    v = random_rhs(lm.n_edge, 21)
    vd, z1, z2 = dev(v), dev(np.zeros(lm.n_edge)), dev(np.zeros(lm.n_edge))
    with pytest.raises(gpu_lib.MxError):
        Pp.apply(vd, z2)
    Pp.materialize(ctx)
    with pytest.raises(gpu_lib.MxError):
        Pp.materialize(ctx)
    ref.apply(vd, z1)
    Pp.apply(vd, z2)
    ref.check()
    Pp.check()
    assert np.array_equal(host(z1), host(z2))
    A_host.upload(ctx)
    with pytest.raises(gpu_lib.MxError):
        A_host.upload(ctx)
    b = dev(random_rhs(lm.n_edge, 22))
    x1, x2 = dev(np.zeros(lm.n_edge)), dev(np.zeros(lm.n_edge))
    s1 = gpu_lib.gmres(ctx, A_dev, ref, b, x1, restart=30, rtol=1e-8)
    s2 = gpu_lib.gmres(ctx, A_host, Pp, b, x2, restart=30, rtol=1e-8)
    assert s1["iters"] == s2["iters"] and np.array_equal(host(x1), host(x2))


def test_plan_stage_materialize_threads(gpu_lib, ctx):
    """The staged setup (matrix upload and host-to-device copies of the plan made on a second
    host thread with its own context, while this thread keeps the device busy with another
    preconditioner) gives the same preconditioner, bit for bit; staging twice, or after
    materialising, is refused."""
    import threading
    say("plan + stage + materialize on two host threads")
    n, parts = (9, 8, 7), (2, 2, 2)
    lm = gpu_lib.Mesh(*n)
    lp = gpu_lib.Partition(lm, *parts, 2)
    A_dev = gpu_lib.Matrix(ctx, lm, 4.0, 16.0)
    ref = gpu_lib.Precond(ctx, A_dev, lm, lp, "oras")
    ctx2 = gpu_lib.Context(0)
    out = {}

    def prepare():
        try:
            A = gpu_lib.Matrix(None, lm, 4.0, 16.0)
            A.upload(ctx2)
            P = gpu_lib.Precond(ctx2, A, lm, lp, "oras", plan_only=True)
            P.stage(ctx2)
            out["A"], out["P"] = A, P
        except Exception as e:  # reported below, on this thread
            out["err"] = e

    v = random_rhs(lm.n_edge, 23)
    vd, z1, z2 = dev(v), dev(np.zeros(lm.n_edge)), dev(np.zeros(lm.n_edge))
    th = threading.Thread(target=prepare)
    th.start()
    for _ in range(20):  # device work on this thread meanwhile
        ref.apply(vd, z1)
    th.join()
    assert "err" not in out, out.get("err")
    P = out["P"]
    with pytest.raises(gpu_lib.MxError):
        P.stage(ctx2)
    P.materialize(ctx)
    with pytest.raises(gpu_lib.MxError):
        P.stage(ctx)
    P.apply(vd, z2)
    ref.check()
    P.check()
    assert np.array_equal(host(z1), host(z2))
    b = dev(random_rhs(lm.n_edge, 24))
    x1, x2 = dev(np.zeros(lm.n_edge)), dev(np.zeros(lm.n_edge))
    s1 = gpu_lib.gmres(ctx, A_dev, ref, b, x1, restart=30, rtol=1e-8)
    s2 = gpu_lib.gmres(ctx, out["A"], P, b, x2, restart=30, rtol=1e-8)
    assert s1["iters"] == s2["iters"] and np.array_equal(host(x1), host(x2))


@pytest.mark.parametrize("n,parts", [((1, 1, 1), (1, 1, 1)), ((2, 1, 1), (2, 1, 1)), ((3, 2, 1), (3, 2, 1))])
def test_tiny_meshes(gpu_lib, ctx, n, parts):
    """Subdomains far smaller than one 64-row tile (a single ragged block each), including the
    single-cube mesh (19 edges)."""
    say("tiny", n, parts)
    for kind in ("oras", "as"):
        c = Case(gpu_lib, ctx, n, parts, 1, 3.0, 9.0, kind)
        v = random_rhs(c.E, 30)
        vd, zd = dev(v), dev(np.zeros(c.E))
        c.lP.apply(vd, zd)
        c.lP.check()
        ref = c.oB(v)
        err = np.linalg.norm(host(zd) - ref) / np.linalg.norm(ref)
        say("  ", kind, "E", c.E, "rel err", err)
        assert err <= 1e-10
        f = random_rhs(c.E, 31)
        xd = dev(np.zeros(c.E))
        st = gpu_lib.gmres(ctx, c.lA, c.lP, dev(f), xd, restart=20, rtol=1e-10)
        ores = gmres.gmres(c.oA, f, c.oB, restart=20, rtol=1e-10)
        assert st["converged"] and abs(st["iters"] - ores.iters) <= 1


@pytest.mark.parametrize("precision", ["c128", "c64"])
def test_grouped_factorisation(gpu_lib, ctx, precision):
    """A tile-pool limit makes the setup factor consecutive subdomain groups one after another
    in a pool that holds one group; the factors, and so the applications, are bitwise those of
    the one-group setup, and they still match the oracle."""
    say("grouped factorisation", precision)
    n = (16, 14, 12)
    cuts = (jittered_cuts(16, 3, 0.2, 7), jittered_cuts(14, 2, 0.2, 8), jittered_cuts(12, 2, 0.2, 9))
    c = Case(gpu_lib, ctx, n, (3, 2, 2), 2, 5.0, 5.0, "oras", cuts, precision=precision)
    info = c.lP.info()
    assert info["factor_groups"] == 1
    limit = info["factor_bytes"] // 4
    Pg = gpu_lib.Precond(ctx, c.lA, c.lm, c.lp, "oras", precision=precision, pool_limit=limit)
    ig = Pg.info()
    say("  groups", ig["factor_groups"], "pool bytes", ig["factor_bytes"], "limit", limit)
    assert ig["factor_groups"] >= 4 and ig["factor_bytes"] <= limit
    v = random_rhs(c.E, 41)
    vd, z1, z2 = dev(v), dev(np.zeros(c.E)), dev(np.zeros(c.E))
    c.lP.apply(vd, z1)
    Pg.apply(vd, z2)
    Pg.check()
    assert np.array_equal(host(z1), host(z2))
    ref = c.oB(v)
    err = np.linalg.norm(host(z2) - ref) / np.linalg.norm(ref)
    assert err <= (1e-10 if precision == "c128" else 1e-4)
    with pytest.raises(gpu_lib.MxError):
        gpu_lib.Precond(ctx, c.lA, c.lm, c.lp, "oras", precision=precision, pool_limit=1024)


@pytest.mark.parametrize("precision", ["c128", "c64"])
def test_factor_schedules(gpu_lib, ctx, precision):
    """The launch orders of the blocked LDL^T (one stream; look-ahead with 1, 2, 3 or 4 block
    columns per pass of the trailing update) compute the same factors up to rounding: their
    applications agree with the oracle, and with each other to rounding.  Subdomains of unequal
    block counts (jittered cuts) cover groups cut short by a subdomain's last column."""
    say("factor schedules", precision)
    n = (16, 14, 12)
    cuts = (jittered_cuts(16, 3, 0.2, 7), jittered_cuts(14, 2, 0.2, 8), jittered_cuts(12, 2, 0.2, 9))
    c = Case(gpu_lib, ctx, n, (3, 2, 2), 2, 5.0, 5.0, "oras", cuts, precision=precision)
    v = random_rhs(c.E, 43)
    vd = dev(v)
    ref = c.oB(v)
    out = {}
    for sched, width in (("one_stream", 0), ("lookahead", 1), ("lookahead", 2), ("lookahead", 3),
                         ("lookahead", 4)):
        P = gpu_lib.Precond(ctx, c.lA, c.lm, c.lp, "oras", precision=precision, schedule=sched,
                            width=width)
        z = dev(np.zeros(c.E))
        P.apply(vd, z)
        P.check()
        out[(sched, width)] = host(z)
        err = np.linalg.norm(out[(sched, width)] - ref) / np.linalg.norm(ref)
        say("  ", sched, width, "rel err vs oracle", err)
        assert err <= (1e-10 if precision == "c128" else 1e-4)
    base = out[("one_stream", 0)]
    for key, z in out.items():
        d = np.linalg.norm(z - base) / np.linalg.norm(base)
        assert d <= (1e-12 if precision == "c128" else 1e-5), key
    for bad in (dict(schedule=7), dict(schedule="lookahead", width=5)):
        with pytest.raises(gpu_lib.MxError):
            gpu_lib.Precond(ctx, c.lA, c.lm, c.lp, "oras", precision=precision, **bad)


def test_factor_tuner(gpu_lib, ctx):
    """The factorisation tuner times the five launch shapes and returns one of them; the
    preconditioner built with its choice applies like the default one (same factors up to
    rounding)."""
    say("factor tuner")
    n, parts = (16, 14, 12), (3, 2, 2)
    cuts = (jittered_cuts(16, 3, 0.2, 7), jittered_cuts(14, 2, 0.2, 8), jittered_cuts(12, 2, 0.2, 9))
    lm = gpu_lib.Mesh(*n)
    lp = gpu_lib.Partition(lm, *parts, 2, *cuts)
    A = gpu_lib.Matrix(ctx, lm, 5.0, 5.0)
    sch, wid, best, each = gpu_lib.tune_factor(ctx, A, lm, lp, "oras")
    say("  choice", sch, wid, best, each)
    assert (sch, wid) in [(1, 1), (2, 1), (2, 2), (2, 3), (2, 4)]
    assert len(each) == 5 and min(each) > 0 and best == min(each)
    P1 = gpu_lib.Precond(ctx, A, lm, lp, "oras")
    P2 = gpu_lib.Precond(ctx, A, lm, lp, "oras", schedule=sch, width=wid)
    v = random_rhs(lm.n_edge, 51)
    vd, z1, z2 = dev(v), dev(np.zeros(lm.n_edge)), dev(np.zeros(lm.n_edge))
    P1.apply(vd, z1)
    P2.apply(vd, z2)
    a, b = host(z1), host(z2)
    assert np.linalg.norm(a - b) <= 1e-12 * np.linalg.norm(a)


@pytest.mark.parametrize("kind,flexible,restart", [("oras", False, 4), ("as", True, 5)])
def test_gmres_graph_replay(gpu_lib, ctx, kind, flexible, restart):
    """Arnoldi steps captured as HIP graphs and replayed (in later cycles and in later solves
    with the same matrix and preconditioner) give bitwise the solution, iteration count and
    residual history of the launched steps; checked over several solves with different right-hand
    sides, with eager work (launched solves, applications, synchronisations) between the
    replays, and again after a coarse level changes the preconditioner."""
    say("graph replay", kind, flexible, restart)
    c = Case(gpu_lib, ctx, (8, 8, 8), (2, 2, 2), 2, 4.0, 16.0, kind)
    for rnd in range(2):
        for seed in (61, 62, 63):
            b = dev(random_rhs(c.E, seed))
            xe, xg = dev(np.zeros(c.E)), dev(np.zeros(c.E))
            se = gpu_lib.gmres(ctx, c.lA, c.lP, b, xe, restart=restart, rtol=1e-8, flexible=flexible,
                               history=True)
            sg = gpu_lib.gmres(ctx, c.lA, c.lP, b, xg, restart=restart, rtol=1e-8, flexible=flexible,
                               history=True, graph=True)
            say("  round", rnd, "seed", seed, "iters", se["iters"], sg["iters"], "cycles", sg["cycles"])
            assert sg["cycles"] > 1  # later cycles replay the captured steps
            assert se["iters"] == sg["iters"] and np.array_equal(se["history"], sg["history"])
            assert np.array_equal(host(xe), host(xg))
            zd = dev(np.zeros(c.E))
            c.lP.apply(b, zd)  # eager work between replays
            host(zd)
        if rnd == 0:
            c.lP.add_coarse(ctx, c.lA, c.lm, 2, "deflation")  # the cached graphs no longer apply
