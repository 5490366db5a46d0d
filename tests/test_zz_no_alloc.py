"""GMRES without device allocation (mx_gmres_noalloc) against mx_gmres through the C ABI: two
calls in a row on one context, the second on a smaller problem, each bitwise equal to the
allocating entry point (same kernels, same order); the device's free memory does not shrink
across the calls; a problem whose workspace exceeds the fixed scratch is refused; and an order-2
matrix with a two-level preconditioner."""
import sys

import numpy as np
import pytest

from mx_inputs import random_rhs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, np.complex128)).cuda()


def _case(mx, ctx, n, parts, kind, k, xi):
    lm = mx.Mesh(*n)
    lA = mx.Matrix(ctx, lm, k, xi)
    lp = mx.Partition(lm, *parts, 2)
    return lm, lA, mx.Precond(ctx, lA, lm, lp, kind)


def test_gmres_noalloc_matches_gmres(gpu_lib):
    import torch
    mx = gpu_lib
    ctx = mx.Context(0)
    cases = [((16, 16, 16), (2, 2, 2), "oras", 6.0, 36.0, 50, False),
             ((8, 8, 8), (2, 2, 2), "as", 4.0, 16.0, 30, True)]
    built = []
    for n, parts, kind, k, xi, m, flex in cases:
        lm, lA, P = _case(mx, ctx, n, parts, kind, k, xi)
        b = _dev(random_rhs(lm.n_edge, 7))
        x_ref, x_na = _dev(np.zeros(lm.n_edge)), _dev(np.zeros(lm.n_edge))
        built.append((n, kind, lA, P, b, x_ref, x_na, m, flex))
    refs = []
    for n, kind, lA, P, b, x_ref, x_na, m, flex in built:
        say("reference mx_gmres", n, kind)
        refs.append(mx.gmres(ctx, lA, P, b, x_ref, restart=m, rtol=1e-8, flexible=flex, history=True))
        say("  iterations", refs[-1]["iters"])
    # between the two readings of free device memory only the no-allocation calls touch the
    # device (comparisons of device tensors would allocate their results)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    stats = []
    for n, kind, lA, P, b, x_ref, x_na, m, flex in built:
        say("mx_gmres_noalloc", n, kind)
        stats.append(mx.gmres(ctx, lA, P, b, x_na, restart=m, rtol=1e-8, flexible=flex,
                              history=True, noalloc=True))
        torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    say("free device memory before / after the no-allocation calls", free0, free1)
    assert free1 >= free0 - (1 << 20)
    for (n, kind, lA, P, b, x_ref, x_na, m, flex), ref, st in zip(built, refs, stats):
        say("  iterations", st["iters"], "vs", ref["iters"])
        assert st["converged"] and st["iters"] == ref["iters"] and st["cycles"] == ref["cycles"]
        assert np.array_equal(st["history"], ref["history"])
        assert st["relres_true"] == ref["relres_true"]
        assert np.array_equal(x_na.cpu().numpy(), x_ref.cpu().numpy())
    # a workspace beyond the fixed scratch is refused before any work is enqueued
    n, kind, lA, P, b, x_ref, x_na, m, flex = built[0]
    with pytest.raises(mx.MxError) as ei:
        mx.gmres(ctx, lA, P, b, x_na, restart=400, rtol=1e-8, flexible=True, noalloc=True)
    assert ei.value.code == mx.MX_EINVAL and "fixed scratch" in str(ei.value)


def test_gmres_noalloc_two_level_order2(gpu_lib):
    """The no-allocation entry point with an order-2 matrix and a two-level (hybrid) preconditioner,
    whose coarse level holds its own buffers: bitwise equal to mx_gmres, no device allocation."""
    import torch
    mx = gpu_lib
    ctx = mx.Context(0)
    lm = mx.Mesh(8, 8, 8)
    lA = mx.Matrix(ctx, lm, 4.0, 16.0, order=2)
    P = mx.Precond(ctx, lA, lm, mx.Partition(lm, 2, 2, 2, 1), "oras")
    P.add_coarse(ctx, lA, lm, 2, "hybrid")
    b = _dev(random_rhs(lA.n, 8))
    x_ref, x_na = _dev(np.zeros(lA.n)), _dev(np.zeros(lA.n))
    ref = mx.gmres(ctx, lA, P, b, x_ref, restart=40, rtol=1e-8, history=True)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    st = mx.gmres(ctx, lA, P, b, x_na, restart=40, rtol=1e-8, history=True, noalloc=True)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    say("order-2 two-level noalloc iterations", st["iters"], "vs", ref["iters"], "free", free0, free1)
    assert free1 >= free0 - (1 << 20)
    assert st["converged"] and st["iters"] == ref["iters"]
    assert np.array_equal(st["history"], ref["history"])
    assert np.array_equal(x_na.cpu().numpy(), x_ref.cpu().numpy())
