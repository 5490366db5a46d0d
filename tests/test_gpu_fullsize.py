"""Full-size checks on the 64^3 benchmark problem (1,872,064 DOFs, 4x4x4 subdomains, 2 layers,
k = 16, xi = k^2), with the launch configuration the benchmark times: all 64 subdomains factored
together and applied with one sweep launch per direction, one sweep workgroup per CU.

The oracle cannot solve the whole problem in test time, so the checks are:
* sampled outputs: the ORAS application restricted to the DOFs owned by subdomain 0 equals the
  oracle's local solve there (Boolean partition of unity: z_e = x_l[e] for owner(e) = l). The
  bar is 1e-10 relative.
* the same for AS, through a one-subdomain resident share, whose output is R_l^T x_l.
* a property at full size: GMRES's reported convergence holds for the oracle's matrix, i.e. the
  true relative residual computed with the oracle's A is <= rtol."""
import sys

import numpy as np
import pytest

from mx_inputs import random_rhs
from oracle import dd, fem
from oracle.mesh import Mesh as OMesh

pytestmark = pytest.mark.gpu

N, P_, L, K, XI = 64, 4, 2, 16.0, 256.0


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def big(gpu_lib):
    import time
    t0 = time.time()
    ctx = gpu_lib.Context(0)
    lm = gpu_lib.Mesh(N, N, N)
    lp = gpu_lib.Partition(lm, P_, P_, P_, L)
    lA = gpu_lib.Matrix(ctx, lm, K, XI)
    say("library objects", time.time() - t0)
    om = OMesh(N, N, N)
    op = dd.Partition(om, P_, P_, P_, L)
    say("oracle mesh + partition", time.time() - t0)
    return {"ctx": ctx, "lm": lm, "lp": lp, "lA": lA, "om": om, "op": op, "E": om.n_edge}


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, np.complex128)).cuda()


def _host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _local_solve(Al, r):
    import scipy.sparse.linalg as spla
    return spla.splu(Al).solve(r)


@pytest.mark.timeout(900)
def test_oras_fullsize_sampled_subdomain(gpu_lib, big):
    mx, b = gpu_lib, big
    say("full-size ORAS application, sampled subdomain 0")
    P = mx.Precond(b["ctx"], b["lA"], b["lm"], b["lp"], "oras")
    v = random_rhs(b["E"], 5)
    z = _host_apply(P, v)
    l = 0
    idx = b["op"].oras_sets[l]
    Al = dd.local_matrix(b["op"], None, dd.ORAS, K, XI, l)
    say("  local n", Al.shape[0])
    x = _local_solve(Al, v[idx])
    own = b["op"].pou(l, dd.ORAS) > 0
    err = np.max(np.abs(z[idx[own]] - x[own])) / np.max(np.abs(x[own]))
    say("  max rel err on owned DOFs", err, "owned", int(own.sum()))
    assert err <= 1e-10


def _host_apply(P, v):
    vd = _dev(v)
    zd = _dev(np.zeros_like(v))
    P.apply(vd, zd)
    P.check()
    return _host(zd)


@pytest.mark.timeout(900)
def test_as_fullsize_share_subdomain(gpu_lib, big):
    """AS local solve of subdomain 0 at full size: its resident share returns R_0^T x_0."""
    mx, b = gpu_lib, big
    say("full-size AS local solve of subdomain 0 (share)")
    oA = fem.assemble(b["om"], K, XI)
    P = mx.Precond(b["ctx"], b["lA"], b["lm"], b["lp"], "as", share=(0, 1))
    v = random_rhs(b["E"], 6)
    z = _host_apply(P, v)
    idx = b["op"].as_sets[0]
    x = _local_solve(dd.local_matrix(b["op"], oA, dd.AS, K, XI, 0), v[idx])
    err = np.max(np.abs(z[idx] - x)) / np.max(np.abs(x))
    say("  max rel err", err)
    assert err <= 1e-10
    rest = np.ones(b["E"], bool)
    rest[idx] = False
    assert not np.any(z[rest])
    b["oA"] = oA


@pytest.mark.timeout(900)
def test_gmres_fullsize_true_residual(gpu_lib, big):
    mx, b = gpu_lib, big
    say("full-size ORAS GMRES(100), true residual with the oracle's matrix")
    oA = b.get("oA")
    if oA is None:
        oA = fem.assemble(b["om"], K, XI)
    P = mx.Precond(b["ctx"], b["lA"], b["lm"], b["lp"], "oras")
    f = random_rhs(b["E"], 2)
    x = _dev(np.zeros(b["E"]))
    st = mx.gmres(b["ctx"], b["lA"], P, _dev(f), x, restart=100, rtol=1e-6)
    xs = _host(x)
    rel = np.linalg.norm(f - oA @ xs) / np.linalg.norm(f)
    say("  iterations", st["iters"], "reported", st["relres_true"], "oracle residual", rel)
    assert st["converged"] and rel <= 1e-6
    assert abs(rel - st["relres_true"]) <= 1e-9
