"""Solve server (continuous batching): results are the same alone and in the mix, with the
preconditioner applications of co-resident requests batched into shared sweep launches or each
on its own stream; requests that can never fit the HBM budget are refused, a served solution
matches the FP64 oracle, and the largest request of the serving configuration meets its stopping
test for the oracle's matrix."""
import numpy as np
import pytest

from oracle import dd, fem, gmres
from oracle.mesh import Mesh as OMesh

pytestmark = pytest.mark.gpu

REQ = dict(n=10, p=2, k=5.0, xi=25.0, center=(0.45, 0.5, 0.55), pol=(0.6, 0.8, 0.0), sigma=0.1)


def say(*a):
    print(*a, flush=True)


OTHERS = [dict(n=14, p=2, k=7.0, xi=7.0), dict(n=9, p=3, k=4.0, xi=16.0),
          dict(n=16, p=2, k=8.0, xi=64.0), dict(n=12, p=2, k=6.0, xi=6.0)]


def _mix(srv):
    tickets = [srv.submit(**o) for o in OTHERS[:2]]
    tm = srv.submit(**REQ)
    tickets += [srv.submit(**o) for o in OTHERS[2:]]
    rm = srv.wait(tm, 300.0)
    sols = []
    for tk in tickets:
        ro = srv.wait(tk, 300.0)
        assert ro["status"] == 0 and ro["converged"], ro
        sols.append(srv.solution(tk, ro["n_dof"]))
    return rm, srv.solution(tm, rm["n_dof"]), sols


def test_batched_and_unbatched_applications_agree(gpu_lib):
    """The same mix of requests served with batched preconditioner applications (one sweep
    launch per direction over the co-resident requests) and with one launch per request on its
    own stream: every solution bitwise equal; the batcher did batch."""
    say("serve batched vs per stream")
    res = {}
    for batched in (True, False):
        # a long window, so that co-resident requests' applications reliably meet in batches
        srv = gpu_lib.Server(slots=4, precision="c64", restart=50, batch_applies=batched,
                             batch_window_us=20000)
        res[batched] = _mix(srv)
        st = srv.stats()
        say("  batched" if batched else "  per stream", st)
        if batched:
            assert st["batched_applications"] >= 2 * st["batches"] > 0  # batches of 2 or more
        else:
            assert st["batches"] == 0
        srv.close()
    (ra, xa, sa), (rb, xb, sb) = res[True], res[False]
    assert ra["iters"] == rb["iters"] and np.array_equal(xa, xb)
    for u, w in zip(sa, sb):
        assert np.array_equal(u, w)


def test_alone_vs_in_the_mix(gpu_lib):
    say("serve alone")
    srv = gpu_lib.Server(slots=3, precision="c64", restart=50)
    t = srv.submit(**REQ)
    r = srv.wait(t, 120.0)
    assert r["status"] == 0 and r["converged"], r
    x_alone = srv.solution(t, r["n_dof"])
    say("  alone", r)
    # the same request among others of different sizes, k and xi, all in flight together
    rm, x_mix, _ = _mix(srv)
    st = srv.stats()
    say("  mix", rm, st)
    assert rm["iters"] == r["iters"]
    assert np.array_equal(x_mix, x_alone)
    assert st["max_admitted"] >= 2  # work of several requests overlapped on the device
    srv.close()


def test_budget_refusal(gpu_lib):
    say("serve budget")
    srv = gpu_lib.Server(slots=1, hbm_budget=1 << 20, precision="c64")
    t = srv.submit(**REQ)
    r = srv.wait(t, 60.0)
    assert r["status"] == gpu_lib.MX_EHBM and r["footprint_bytes"] > (1 << 20)
    srv.close()


def test_served_solution_vs_oracle(gpu_lib):
    say("serve vs oracle")
    srv = gpu_lib.Server(slots=2, precision="c64", restart=50)
    t = srv.submit(**REQ)
    r = srv.wait(t, 120.0)
    x = srv.solution(t, r["n_dof"])
    srv.close()
    n = REQ["n"]
    om = OMesh(n, n, n)
    A = fem.assemble(om, REQ["k"], REQ["xi"])
    f = fem.load_vector(om, fem.gaussian_source(REQ["center"], REQ["pol"], REQ["sigma"]))
    part = dd.Partition(om, 2, 2, 2, 2)
    B = dd.Schwarz(part, A, dd.ORAS, REQ["k"], REQ["xi"])
    ores = gmres.gmres(A, f, B, restart=50, rtol=1e-6)
    err = np.linalg.norm(x - ores.x) / np.linalg.norm(ores.x)
    say("  served err vs oracle", err, "iters", r["iters"], ores.iters)
    assert err <= 1e-5


@pytest.mark.timeout(600)
def test_largest_served_request_true_residual(gpu_lib):
    """The largest request of the serving configuration (k = 16: n = ceil(16^1.5) + 4 = 68 cubes
    per side, 4x4x4 subdomains, about 2.3 M DOFs, xi = k, mixed precision): the true relative
    residual recomputed with the oracle's FP64 matrix and the oracle's Gaussian load vector is
    <= rtol and equals the one the server reports."""
    say("largest served request vs the oracle's matrix")
    req = dict(n=68, p=4, k=16.0, xi=16.0, center=(0.4, 0.55, 0.5), pol=(0.0, 0.6, 0.8), sigma=0.1)
    srv = gpu_lib.Server(slots=1, precision="c64", restart=50)
    t = srv.submit(**req)
    r = srv.wait(t, 300.0)
    assert r["status"] == 0 and r["converged"], r
    x = srv.solution(t, r["n_dof"])
    srv.close()
    om = OMesh(req["n"], req["n"], req["n"])
    A = fem.assemble(om, req["k"], req["xi"])
    f = fem.load_vector(om, fem.gaussian_source(req["center"], req["pol"], req["sigma"]))
    rel = np.linalg.norm(f - A @ x) / np.linalg.norm(f)
    say("  n_dof", r["n_dof"], "iters", r["iters"], "reported", r["relres_true"], "oracle residual", rel)
    assert rel <= 1e-6 and abs(rel - r["relres_true"]) <= 1e-9


def test_retry_after_late_allocation_failure(gpu_lib):
    """Requests whose device phase fails after their preconditioner has been set up (MX_ENOMEM,
    injected through the server's test hook) are retried from the same host plan: every request
    of the mix still converges, and each solution equals the one served without failures, bit
    for bit."""
    say("serve with injected late allocation failures")
    srv = gpu_lib.Server(slots=3, precision="c64", restart=50)
    r0, x0, s0 = _mix(srv)
    srv.inject_enomem(3)
    r1, x1, s1 = _mix(srv)
    say("  without", r0["iters"], "with injected failures", r1["iters"], srv.stats())
    srv.close()
    assert r1["status"] == 0 and r1["converged"] and r1["iters"] == r0["iters"]
    assert np.array_equal(x1, x0)
    for u, w in zip(s0, s1):
        assert np.array_equal(u, w)
