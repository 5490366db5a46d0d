"""Full-size checks on the 96x96x192 jittered-box problem (box [0,1]x[0,1]x[0,2], 12,524,928
DOFs, k = xi = 24, 6x6x12 subdomains with cut planes jittered by +-20 %, 2 layers, ORAS,
complex64 factors), in the launch configuration the benchmark times: one preconditioner over all
432 subdomains, factored in the subdomain groups that fit beside the trimmed factors, one sweep
launch per direction.

The oracle cannot build the whole problem's preconditioner in test time.  An ORAS local problem
reaches only `layers` cubes past its box, and on the boundary of the overlapped subdomain it
carries the impedance term with coefficient k, on the boundary of the domain (eq:imp) as on the
interface (ImpRAS, Sec. 6.3).  So the oracle assembles it on the sub-box around the subdomain
(its box of cubes extended by the layers, clipped to the domain), cut so that the subdomain is
one box of that partition (dd.sub_box); up to numbering it is the whole problem's local problem.
Sub-box vertices map to the whole mesh through integer coordinates; both numberings order
vertices, and so edges, lexicographically by (z, y, x), so the local sets keep their order.

Sampled: the first subdomain (a corner), an interior one and the last (highest tile and vector
offsets).  Checked per sample:
* the library's local DOF set equals the oracle's, mapped to global edges (bit-exact), and the
  library's owner of every edge interior to the box (all its tetrahedra in the box) is the box;
* the library's local matrix equals the oracle's (1e-13 relative), and its reverse Cuthill-McKee
  order and envelope starts equal the oracle's (bit-exact);
* the application z = B v on the edges interior to the box equals the oracle's local solve there
  (Boolean partition of unity), to 1e-4 relative L2: the bar of the complex64 application tests
  on small meshes.
A property of the whole solve: the FGMRES true residual recomputed with the oracle's matrix."""
import gc
import sys
import time

import numpy as np
import pytest
import scipy.sparse as sp

from mx_inputs import config_batching, random_rhs
from oracle import dd, pool, rcm
from oracle.mesh import Mesh as OMesh

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.timeout(1500)
def test_batching_fullsize_sampled(gpu_lib):
    import torch
    mx = gpu_lib
    w = config_batching(0)
    px, py, pz = w.parts
    sampled = (0, 2 + px * (3 + py * 6), px * py * pz - 1)
    t0 = time.time()
    ctx = mx.Context(0)
    lm = mx.Mesh(*w.n, *w.lengths)
    E = lm.n_edge
    lA = mx.Matrix(ctx, lm, w.k, w.xi)
    lp = mx.Partition(lm, *w.parts, w.layers, *w.cuts)
    ex = lp.export("oras")
    loc = {l: mx.local_problem(lm, lA, lp, l, "oras") for l in sampled}
    v = random_rhs(E, 13)
    P = mx.Precond(ctx, lA, lm, lp, "oras", precision="c64")
    info = P.info()
    say("library: %d DOFs, %d subdomains, %d factor groups, setup done at %.1f s"
        % (E, info["n_sub"], info["factor_groups"], time.time() - t0))
    vd = torch.from_numpy(v).cuda()
    zd = torch.zeros_like(vd)
    P.apply(vd, zd)
    P.check()
    torch.cuda.synchronize()
    z = zd.cpu().numpy()
    del P, lA, vd, zd, ctx
    gc.collect()
    torch.cuda.empty_cache()
    say("library application done at %.1f s" % (time.time() - t0))

    og = OMesh(*w.n, *w.lengths)  # the oracle's numbering of the whole mesh's edges
    assert og.n_edge == E
    say("oracle whole-mesh numbering at %.1f s" % (time.time() - t0))
    h = np.array([L / n for L, n in zip(w.lengths, w.n)])
    nx, ny, _ = w.n
    tasks, keep = [], []
    for l in sampled:
        om, part, lr, lo, hi, rlo = dd.sub_box(w.n, w.lengths, w.parts, w.layers, w.cuts, l)
        ijk = np.rint(om.xyz / h).astype(np.int64) + np.array(rlo)
        gv = ijk[:, 0] + (nx + 1) * (ijk[:, 1] + (ny + 1) * ijk[:, 2])
        a, b = gv[om.edge_vert[:, 0]], gv[om.edge_vert[:, 1]]
        assert np.all(a < b)  # the same orientation in both numberings
        gid = og.edge_index(a, b)
        s = part.oras_sets[lr]
        assert np.all(np.diff(gid[s]) > 0)
        assert np.array_equal(ex["sets"][l], gid[s]), l
        inner = np.ones(len(s), bool)
        for end in (0, 1):
            c = ijk[om.edge_vert[s, end]]
            inner &= np.all((c > np.array(lo)) & (c < np.array(hi)), axis=1)
        assert inner.sum() > 0 and np.all(ex["owner"][gid[s][inner]] == l), l
        Al = dd.local_matrix(part, None, dd.ORAS, w.k, w.xi, lr).tocsr()
        L = loc[l]
        Ll = sp.csr_matrix((L["val"], L["col"], L["rowptr"]), shape=Al.shape)
        assert abs(Ll - Al).max() <= 1e-13 * abs(Al).max(), l
        g = rcm.pattern_graph(dd.local_pattern(part, lr, dd.ORAS))
        perm = rcm.rcm(*g)
        assert np.array_equal(L["perm"], perm) and np.array_equal(L["first"], rcm.envelope(*g, perm)), l
        say("  subdomain %d: n = %d, %d interior edges; sets, owners, matrix, order equal (%.1f s)"
            % (l, len(s), int(inner.sum()), time.time() - t0))
        tasks.append((Al.tocsc(), v[gid[s]]))
        keep.append((l, gid[s][inner], inner))
    res = pool.solve_many(tasks)
    for (l, gi, inner), (x, t_lu, _) in zip(keep, res):
        err = np.linalg.norm(z[gi] - x[inner]) / np.linalg.norm(x[inner])
        say("  subdomain %d: application vs oracle local solve, rel L2 %.2e (oracle LU %.1f s)"
            % (l, err, t_lu))
        assert err <= 1e-4, (l, err)


@pytest.mark.timeout(1500)
def test_batching_fullsize_fgmres_true_residual(gpu_lib):
    """The whole 96x96x192 solve as the benchmark runs it (ORAS with complex64 factors,
    FGMRES(50) with complex64 SpMV values and FP64 Krylov vectors, rtol 1e-6), on a seeded random
    right-hand side: the library's reported convergence holds for the oracle's matrix, i.e. the
    true relative residual recomputed with the oracle's A at full size is <= rtol and equals the
    reported one to 1e-9."""
    import torch
    from oracle import fem
    mx = gpu_lib
    w = config_batching(0)
    t0 = time.time()
    ctx = mx.Context(0)
    lm = mx.Mesh(*w.n, *w.lengths)
    E = lm.n_edge
    lA = mx.Matrix(ctx, lm, w.k, w.xi)
    lp = mx.Partition(lm, *w.parts, w.layers, *w.cuts)
    P = mx.Precond(ctx, lA, lm, lp, "oras", precision="c64")
    f = random_rhs(E, 17)
    fd = torch.from_numpy(f).cuda()
    xd = torch.zeros_like(fd)
    st = mx.gmres(ctx, lA, P, fd, xd, restart=50, rtol=1e-6, max_iters=1000, flexible=True,
                  spmv_c64=True)
    torch.cuda.synchronize()
    x = xd.cpu().numpy()
    say("library: %d iterations, reported relres %.4e, at %.1f s"
        % (st["iters"], st["relres_true"], time.time() - t0))
    del P, lA, fd, xd, ctx
    gc.collect()
    torch.cuda.empty_cache()
    oA = fem.assemble(OMesh(*w.n, *w.lengths), w.k, w.xi)
    rel = np.linalg.norm(f - oA @ x) / np.linalg.norm(f)
    say("oracle residual %.4e at %.1f s" % (rel, time.time() - t0))
    assert st["converged"] and rel <= 1e-6
    assert abs(rel - st["relres_true"]) <= 1e-9
