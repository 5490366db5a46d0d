"""End-to-end parity on the intermediate unit-cube problem: 32^3 cubes (238,688 DOFs), k = 8,
xi in {k, k^1.5, k^2}, 4x4x4 subdomains with 2 layers (corner, edge, face and interior boxes,
several 64-row tiles per subdomain), AS and ORAS, GMRES(100), rtol 1e-6.

For each case the oracle (its local problems factored and solved on a pool of host processes,
bitwise equal to the one-process oracle) runs GMRES to the tolerance; the library must
* stop within +-1 iteration of the oracle (Sec. 6.1 stopping rule),
* after exactly the oracle's iteration count, return a solution within 1e-8 relative L2 of the
  oracle's (Sec. 5.2 minimal-residual iterate; rounding decides nothing else),
(The integer work of the same problem -- local DOF sets, owners, RCM orders -- is checked
bit-exact on the CPU, in test_abi_host.py.)"""
import sys

import numpy as np
import pytest

from mx_inputs import config_medium, random_rhs
from oracle import dd, fem, gmres, pool
from oracle.mesh import Mesh as OMesh

pytestmark = pytest.mark.gpu

OKIND = {"oras": dd.ORAS, "as": dd.AS}


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
def med(gpu_lib):
    w = config_medium()
    ctx = gpu_lib.Context(0)
    lm = gpu_lib.Mesh(*w.n)
    lp = gpu_lib.Partition(lm, *w.parts, w.layers)
    om = OMesh(*w.n)
    op = dd.Partition(om, *w.parts, w.layers)
    return {"ctx": ctx, "lm": lm, "lp": lp, "om": om, "op": op, "E": om.n_edge}


@pytest.mark.timeout(900)
@pytest.mark.parametrize("kind", ["oras", "as"])
@pytest.mark.parametrize("xi_exp", [1.0, 1.5, 2.0])
def test_medium_gmres_parity(gpu_lib, med, kind, xi_exp):
    mx = gpu_lib
    w = config_medium(kind, xi_exp, seed=int(2 * xi_exp))
    say("32^3 GMRES(100)", kind, "xi = k^%g" % xi_exp)
    oA = fem.assemble(med["om"], w.k, w.xi)
    f = random_rhs(med["E"], w.seed)
    with pool.PooledSchwarz(med["op"], oA, OKIND[kind], w.k, w.xi) as oB:
        say("  oracle setup %.1f s on %d workers" % (oB.t_setup, len(oB.procs)))
        ores = gmres.gmres(oA, f, oB, restart=w.restart, rtol=w.rtol)
    say("  oracle iterations", ores.iters, "relres", ores.relres_true)
    assert ores.converged
    lA = mx.Matrix(med["ctx"], med["lm"], w.k, w.xi)
    lP = mx.Precond(med["ctx"], lA, med["lm"], med["lp"], kind)
    bd = dev(f)
    xd = dev(np.zeros(med["E"]))
    st = mx.gmres(med["ctx"], lA, lP, bd, xd, restart=w.restart, rtol=w.rtol)
    say("  gpu iterations", st["iters"], "relres", st["relres_true"])
    assert st["converged"] and abs(st["iters"] - ores.iters) <= 1
    rel = np.linalg.norm(f - oA @ host(xd)) / np.linalg.norm(f)
    assert rel <= w.rtol
    xd2 = dev(np.zeros(med["E"]))
    mx.gmres(med["ctx"], lA, lP, bd, xd2, restart=w.restart, fixed_iters=ores.iters)
    x2 = host(xd2)
    err = np.linalg.norm(x2 - ores.x) / np.linalg.norm(ores.x)
    say("  rel L2 vs oracle at %d iterations: %.2e" % (ores.iters, err))
    assert err <= 1e-8
