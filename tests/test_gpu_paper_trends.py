"""The trends of Tables tab:1 and tab:lowAbs (Sec. 6.2) through the C ABI, against the oracle on
the same seeded inputs: one-level AS with its PEC local problems, PEC on the global boundary, a
16^3 mesh in 4x4x4 boxes with 2 layers, k = 8 and 10, xi_prob = xi_prec = k^2 and = k.  Each GPU
solve takes the oracle's iteration count within +-1 (up to 120 iterations, GMRES(200)), and the
GPU counts show the paper's trend (flat at xi = k^2, larger and growing with k at xi = k).

After exactly the oracle's iteration count the solutions agree to 1e-8 relative L2 at xi = k^2.
At xi = k the iterates themselves are sensitive at rounding level: the oracle's own solution
moves by s of the order of 1e-8 (k = 8) and 1e-6 (k = 10) when b is perturbed by 1e-15 relative
(seeded), and the GPU's differs from it by about as much (measured 9.6e-9 and 1.8e-6).  So there
the bar is max(1e-8, 10 s), with s measured in the test."""
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


@pytest.mark.timeout(900)
def test_low_absorption_trend_matches_oracle(gpu_lib):
    mx = gpu_lib
    n, parts, layers = (16, 16, 16), (4, 4, 4), 2
    om = OMesh(*n)
    opart = dd.Partition(om, *parts, layers)
    f = random_rhs(om.n_edge, 53)
    f[om.boundary_edge_mask()] = 0
    ctx = mx.Context(0)
    lm = mx.Mesh(*n)
    lpart = mx.Partition(lm, *parts, layers)
    bd = dev(f)
    its = {}
    for k in (8.0, 10.0):
        for xi in (k * k, k):
            say("AS, PEC, 16^3, k", k, "xi", xi)
            oA = fem.assemble(om, k, xi, fem.BC_PEC)
            oB = dd.Schwarz(opart, oA, dd.AS, k, xi, fem.BC_PEC)
            ores = gmres.gmres(oA, f, oB, restart=200, rtol=1e-6, max_iters=400)
            assert ores.converged
            lA = mx.Matrix(ctx, lm, k, xi, mx.MX_BC_PEC)
            lP = mx.Precond(ctx, lA, lm, lpart, "as")
            xd = dev(np.zeros(om.n_edge))
            st = mx.gmres(ctx, lA, lP, bd, xd, restart=200, rtol=1e-6, max_iters=400)
            xd2 = dev(np.zeros(om.n_edge))
            mx.gmres(ctx, lA, lP, bd, xd2, restart=200, fixed_iters=ores.iters)
            err = np.linalg.norm(host(xd2) - ores.x) / np.linalg.norm(ores.x)
            say("  oracle", ores.iters, "gpu", st["iters"], "relres", st["relres_true"],
                "err at the oracle's count %.2e" % err)
            assert st["converged"] and abs(st["iters"] - ores.iters) <= 1
            bar = 1e-8
            if xi == k:  # the oracle's own rounding-level sensitivity at this iteration count
                g = f * (1 + 1e-15 * np.random.default_rng(7).standard_normal(len(f)))
                pert = gmres.gmres(oA, g, oB, restart=200, fixed_iters=ores.iters)
                sens = np.linalg.norm(pert.x - ores.x) / np.linalg.norm(ores.x)
                bar = max(bar, 10 * sens)
                say("  oracle sensitivity to a 1e-15 perturbation of b: %.2e" % sens)
            assert err <= bar, (err, bar)
            its[k, xi] = st["iters"]
            del lP, lA
    assert abs(its[10.0, 100.0] - its[8.0, 64.0]) <= 5, its
    assert its[8.0, 8.0] >= 1.5 * its[8.0, 64.0] and its[10.0, 10.0] >= 2.5 * its[10.0, 100.0], its
    assert its[10.0, 10.0] >= 1.4 * its[8.0, 8.0], its
