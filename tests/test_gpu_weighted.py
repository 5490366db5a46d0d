"""GPU parity of weighted GMRES (Sec. 5.2, eq:ip: residual minimised in the D_k-norm with
D_k = K + k^2 M) through the C ABI against the oracle on the same seeded inputs: iterations
within +-1, and after exactly the oracle's iteration count the solution within 1e-8 relative L2;
restarted and flexible variants; the D-norm true residual reported by the library equals the one
recomputed with the oracle's matrices."""
import sys

import numpy as np
import pytest

from mx_inputs import random_rhs
from oracle import dd, fem, gmres
from oracle.mesh import Mesh as OMesh

pytestmark = pytest.mark.gpu


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


@pytest.mark.parametrize("kind,restart,flexible,bc", [("oras", 50, False, fem.BC_IMPEDANCE),
                                                      ("as", 50, False, fem.BC_IMPEDANCE),
                                                      ("oras", 6, True, fem.BC_IMPEDANCE),
                                                      ("as", 8, False, fem.BC_PEC)])
def test_weighted_gmres_parity(gpu_lib, kind, restart, flexible, bc):
    mx = gpu_lib
    say("weighted GMRES", kind, restart, flexible, bc)
    n, parts, k, xi = (8, 8, 8), (2, 2, 2), 4.0, 4.0
    om = OMesh(*n)
    oA = fem.assemble(om, k, xi, bc)
    oD = fem.weight_matrix(om, k, bc)
    oB = dd.Schwarz(dd.Partition(om, *parts, 2), oA, {"oras": dd.ORAS, "as": dd.AS}[kind], k, xi, bc)
    f = random_rhs(om.n_edge, 31)
    if bc == fem.BC_PEC:
        f[om.boundary_edge_mask()] = 0
    ores = gmres.gmres(oA, f, oB, restart=restart, rtol=1e-6, flexible=flexible, D=oD)
    std = gmres.gmres(oA, f, oB, restart=restart, rtol=1e-6, flexible=flexible)
    say("  oracle iterations weighted", ores.iters, "standard", std.iters)
    ctx = mx.Context(0)
    lm = mx.Mesh(*n)
    lA = mx.Matrix(ctx, lm, k, xi, bc)
    lD = mx.Matrix.weight(ctx, lm, k, bc)
    lP = mx.Precond(ctx, lA, lm, mx.Partition(lm, *parts, 2), kind)
    bd, xd = dev(f), dev(np.zeros(om.n_edge))
    st = mx.gmres(ctx, lA, lP, bd, xd, restart=restart, rtol=1e-6, flexible=flexible, weight=lD)
    say("  gpu iterations", st["iters"], "relres_D", st["relres_true"])
    assert st["converged"] and abs(st["iters"] - ores.iters) <= 1
    r = f - oA @ host(xd)
    dn = lambda v: np.sqrt(np.real(np.vdot(v, oD @ v)))
    assert abs(dn(r) / dn(f) - st["relres_true"]) <= 1e-10 and st["relres_true"] <= 1e-6
    xd2 = dev(np.zeros(om.n_edge))
    mx.gmres(ctx, lA, lP, bd, xd2, restart=restart, fixed_iters=ores.iters, flexible=flexible,
             weight=lD)
    err = np.linalg.norm(host(xd2) - ores.x) / np.linalg.norm(ores.x)
    say("  rel L2 at the oracle's count", err)
    assert err <= 1e-8
