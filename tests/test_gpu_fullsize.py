"""Full-size checks on the 64^3 benchmark problem (1,872,064 DOFs, 4x4x4 subdomains, 2 layers,
k = 16), with the launch configuration the benchmark times: all 64 subdomains factored together
and applied with one sweep launch per direction, one sweep workgroup per CU.

The oracle cannot solve the whole problem in test time, so the checks are:
* integer work at full size: the local DOF sets of both kinds and the owners of all 64
  subdomains, and the reverse Cuthill-McKee order of an interior subdomain, bit-exact;
* sampled outputs at xi = k and xi = k^2 (the ends of the benchmark's range): the ORAS
  application restricted to the DOFs owned by a corner (0), an interior (42, the largest local
  problem) and the last subdomain (63, the highest tile and vector offsets) equals the oracle's
  local solve there (Boolean partition of unity: z_e = x_l[e] for owner(e) = l); the AS local
  solves of the same subdomains, through one-subdomain resident shares (output R_l^T x_l), equal
  the oracle's.  Bar: 1e-10 relative.  The oracle's local problems are factored in parallel on
  host worker processes;
* a property at full size: GMRES's reported convergence holds for the oracle's matrix, i.e. the
  true relative residual computed with the oracle's A is <= rtol (ORAS at xi = k^2, AS at xi = k
  through a restart, and the mixed-precision FGMRES);
* the two-level deflated form with the 16^3-cube coarse mesh: the oracle's coarse correction at
  full size plus sampled local solves against the library's application;
* weighted GMRES: the reported D-norm residual equals the one recomputed with the oracle's A and
  D_k."""
import sys
import time

import numpy as np
import pytest

from mx_inputs import random_rhs
from oracle import dd, fem, pool, rcm
from oracle.mesh import Mesh as OMesh

pytestmark = pytest.mark.gpu

N, P_, L, K = 64, 4, 2, 16.0
XIS = (K, K * K)
SAMPLED = (0, 42, 63)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def big(gpu_lib):
    t0 = time.time()
    ctx = gpu_lib.Context(0)
    lm = gpu_lib.Mesh(N, N, N)
    lp = gpu_lib.Partition(lm, P_, P_, P_, L)
    say("library objects", time.time() - t0)
    om = OMesh(N, N, N)
    op = dd.Partition(om, P_, P_, P_, L)
    say("oracle mesh + partition", time.time() - t0)
    Kg, Mg, Bg = fem.assemble_parts(om)
    say("oracle K, M, M_b", time.time() - t0)
    return {"ctx": ctx, "lm": lm, "lp": lp, "om": om, "op": op, "E": om.n_edge,
            "oA": lambda xi: fem.combine(Kg, Mg, Bg, K, xi, fem.BC_IMPEDANCE)}


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, np.complex128)).cuda()


def _host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _host_apply(P, v):
    vd = _dev(v)
    zd = _dev(np.zeros_like(v))
    P.apply(vd, zd)
    P.check()
    return _host(zd)


@pytest.mark.timeout(600)
def test_fullsize_partition_and_order_bit_exact(gpu_lib, big):
    say("full-size partition sets, owners, RCM order of subdomain 42")
    op, lp = big["op"], big["lp"]
    for kind, sets in (("oras", op.oras_sets), ("as", op.as_sets)):
        ex = lp.export(kind)
        assert len(ex["sets"]) == 64
        for l in range(64):
            assert np.array_equal(ex["sets"][l], sets[l]), (kind, l)
        assert np.array_equal(ex["owner"], op.owner)
    A = gpu_lib.Matrix(None, big["lm"], K, K)
    for kind, okind in (("oras", dd.ORAS), ("as", dd.AS)):
        g = rcm.pattern_graph(dd.local_pattern(op, 42, okind))
        perm = rcm.rcm(*g)
        lp_ = gpu_lib.local_problem(big["lm"], A, lp, 42, kind)
        say("  ", kind, "n", len(perm))
        assert np.array_equal(lp_["perm"], perm)
        assert np.array_equal(lp_["first"], rcm.envelope(*g, perm))


@pytest.mark.timeout(1200)
def test_fullsize_sampled_local_solves(gpu_lib, big):
    mx, b, op = gpu_lib, big, big["op"]
    E = b["E"]
    v = random_rhs(E, 5)
    tasks, keys, gpu = [], [], {}
    for xi in XIS:
        say("xi", xi)
        lA = mx.Matrix(b["ctx"], b["lm"], K, xi)
        P = mx.Precond(b["ctx"], lA, b["lm"], b["lp"], "oras")
        gpu[("oras", xi)] = _host_apply(P, v)
        del P
        for l in SAMPLED:
            S = mx.Precond(b["ctx"], lA, b["lm"], b["lp"], "as", share=(l, l + 1))
            gpu[("as", xi, l)] = _host_apply(S, v)
            del S
        oA = b["oA"](xi)
        for l in SAMPLED:
            tasks.append((dd.local_matrix(op, None, dd.ORAS, K, xi, l), v[op.oras_sets[l]]))
            keys.append(("oras", xi, l))
            tasks.append((dd.local_matrix(op, oA, dd.AS, K, xi, l), v[op.as_sets[l]]))
            keys.append(("as", xi, l))
        del oA
    t0 = time.time()
    res = pool.solve_many(tasks)
    say("oracle: %d local solves in %.1f s (longest factorisation %.1f s)"
        % (len(tasks), time.time() - t0, max(r[1] for r in res)))
    for key, (x, _, _) in zip(keys, res):
        kind, xi, l = key
        if kind == "oras":
            idx = op.oras_sets[l]
            own = op.pou(l, dd.ORAS) > 0
            z = gpu[("oras", xi)]
            err = np.max(np.abs(z[idx[own]] - x[own])) / np.max(np.abs(x[own]))
            say("  ORAS xi %g l %d owned %d: max rel err %.2e" % (xi, l, int(own.sum()), err))
        else:
            idx = op.as_sets[l]
            z = gpu[("as", xi, l)]
            err = np.max(np.abs(z[idx] - x)) / np.max(np.abs(x))
            rest = np.ones(E, bool)
            rest[idx] = False
            assert not np.any(z[rest])
            say("  AS xi %g l %d n %d: max rel err %.2e" % (xi, l, len(idx), err))
        assert err <= 1e-10, key


@pytest.mark.timeout(900)
@pytest.mark.parametrize("kind,xi", [("oras", K * K), ("as", K)])
def test_gmres_fullsize_true_residual(gpu_lib, big, kind, xi):
    """ORAS at xi = k^2 (13 iterations) and AS at xi = k (the batch's longest solve, over 100
    iterations, so GMRES(100) restarts)."""
    mx, b = gpu_lib, big
    say("full-size", kind, "xi", xi, "GMRES(100), true residual with the oracle's matrix")
    oA = b["oA"](xi)
    lA = mx.Matrix(b["ctx"], b["lm"], K, xi)
    P = mx.Precond(b["ctx"], lA, b["lm"], b["lp"], kind)
    f = random_rhs(b["E"], 2)
    x = _dev(np.zeros(b["E"]))
    st = mx.gmres(b["ctx"], lA, P, _dev(f), x, restart=100, rtol=1e-6)
    xs = _host(x)
    rel = np.linalg.norm(f - oA @ xs) / np.linalg.norm(f)
    say("  iterations", st["iters"], "reported", st["relres_true"], "oracle residual", rel)
    assert st["converged"] and rel <= 1e-6
    assert abs(rel - st["relres_true"]) <= 1e-9


@pytest.mark.timeout(900)
def test_fgmres_mixed_fullsize_true_residual(gpu_lib, big):
    """The mixed-precision path at full size (ORAS with complex64 factors and SpMV values, FP64
    FGMRES(100), xi = k): the true residual recomputed with the oracle's FP64 matrix is <= rtol and
    equals the reported one, so the FP64 stopping test is met for the oracle's problem."""
    mx, b = gpu_lib, big
    say("full-size mixed ORAS FGMRES(100), true residual with the oracle's matrix")
    oA = b["oA"](K)
    lA = mx.Matrix(b["ctx"], b["lm"], K, K)
    P = mx.Precond(b["ctx"], lA, b["lm"], b["lp"], "oras", precision="c64")
    f = random_rhs(b["E"], 3)
    x = _dev(np.zeros(b["E"]))
    st = mx.gmres(b["ctx"], lA, P, _dev(f), x, restart=100, rtol=1e-6, flexible=True, spmv_c64=True)
    xs = _host(x)
    rel = np.linalg.norm(f - oA @ xs) / np.linalg.norm(f)
    say("  iterations", st["iters"], "reported", st["relres_true"], "oracle residual", rel)
    assert st["converged"] and rel <= 1e-6
    assert abs(rel - st["relres_true"]) <= 1e-9


@pytest.mark.timeout(1200)
def test_fullsize_two_level_deflation_sampled(gpu_lib, big):
    """The two-level deflated form (eq:ADEF1ras) over ORAS at xi = k on the 64^3 problem, with the
    nested coarse mesh of 16^3 cubes, as `bench.py --coarse 4 --combine deflation` runs it.  With
    the Boolean partition of unity, B v = B1 t + G v with t = v - A G v and G v = R^0^T (A^0)^-1
    R^0 v, so on the DOFs owned by subdomain l, (B v)_e = x_l[e] + (G v)_e with x_l the local
    solve of t.  The oracle computes G v exactly at full size (its R^0, A^0 = R^0 A R^0^T and a
    sparse LU of A^0) and the local solves of a corner (0) and the last subdomain (63).
    Bar: 1e-10 relative."""
    from oracle import coarse
    mx, b, op, om = gpu_lib, big, big["op"], big["om"]
    xi = K
    v = random_rhs(b["E"], 9)
    lA = mx.Matrix(b["ctx"], b["lm"], K, xi)
    P = mx.Precond(b["ctx"], lA, b["lm"], b["lp"], "oras")
    P.add_coarse(b["ctx"], lA, b["lm"], 4, "deflation")
    z = _host_apply(P, v)
    del P
    t0 = time.time()
    oA = b["oA"](xi)
    R = coarse.restriction(om, coarse.coarse_mesh(om, 4))
    lu0 = dd.factor_local((R @ oA @ R.T).tocsc())
    Gv = R.T @ lu0.solve(R @ v)
    t = v - oA @ Gv
    say("oracle coarse correction at full size: %d coarse DOFs, %.1f s" % (R.shape[0], time.time() - t0))
    tasks = [(dd.local_matrix(op, None, dd.ORAS, K, xi, l), t[op.oras_sets[l]]) for l in (0, 63)]
    res = pool.solve_many(tasks)
    for l, (x, _, _) in zip((0, 63), res):
        idx = op.oras_sets[l]
        own = op.pou(l, dd.ORAS) > 0
        want = x[own] + Gv[idx[own]]
        err = np.max(np.abs(z[idx[own]] - want)) / np.max(np.abs(want))
        say("  ADEF1-ORAS xi %g l %d owned %d: max rel err %.2e" % (xi, l, int(own.sum()), err))
        assert err <= 1e-10


@pytest.mark.timeout(900)
def test_weighted_gmres_fullsize_true_residual(gpu_lib, big):
    """Weighted GMRES (Sec. 5.2, D_k = K + k^2 M) on the 64^3 ORAS problem at xi = k^2: the
    D-norm relative residual the library reports equals the one recomputed with the oracle's A
    and D_k, and is <= rtol (a property that holds at any size)."""
    mx, b = gpu_lib, big
    say("full-size weighted ORAS GMRES(100), D-norm true residual with the oracle's matrices")
    oA = b["oA"](K * K)
    oD = fem.weight_matrix(b["om"], K)
    lA = mx.Matrix(b["ctx"], b["lm"], K, K * K)
    lD = mx.Matrix.weight(b["ctx"], b["lm"], K)
    P = mx.Precond(b["ctx"], lA, b["lm"], b["lp"], "oras")
    f = random_rhs(b["E"], 3)
    x = _dev(np.zeros(b["E"]))
    st = mx.gmres(b["ctx"], lA, P, _dev(f), x, restart=100, rtol=1e-6, weight=lD)
    r = f - oA @ _host(x)
    dn = lambda v: np.sqrt(np.real(np.vdot(v, oD @ v)))
    rel = dn(r) / dn(f)
    say("  iterations", st["iters"], "reported", st["relres_true"], "oracle D-norm residual", rel)
    assert st["converged"] and rel <= 1e-6
    assert abs(rel - st["relres_true"]) <= 1e-9
