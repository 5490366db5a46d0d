"""Oracle: the whole path for one problem (mesh -> assembly -> partition -> local factors ->
preconditioned GMRES), for tests and the CPU baseline.

Test infrastructure only (see oracle/__init__.py).
"""
import time

import numpy as np

from . import dd, fem, gmres
from .mesh import Mesh


class Problem:
    def __init__(self, n=(8, 8, 8), lengths=(1.0, 1.0, 1.0), k=4.0, xi=16.0,
                 bc=fem.BC_IMPEDANCE, parts=(2, 2, 2), layers=2, kind=dd.ORAS, cuts=None):
        self.n, self.lengths, self.k, self.xi, self.bc = n, lengths, k, xi, bc
        self.parts, self.layers, self.kind, self.cuts = parts, layers, kind, cuts


def setup(prob, timings=None):
    t = time.perf_counter()
    mesh = Mesh(*prob.n, *prob.lengths)
    A = fem.assemble(mesh, prob.k, prob.xi, prob.bc)
    cx, cy, cz = prob.cuts if prob.cuts is not None else (None, None, None)
    part = dd.Partition(mesh, *prob.parts, prob.layers, cx, cy, cz)
    t1 = time.perf_counter()
    B = dd.Schwarz(part, A, prob.kind, prob.k, prob.xi, prob.bc)
    t2 = time.perf_counter()
    if timings is not None:
        timings["assemble_partition"] = t1 - t
        timings["local_factor"] = t2 - t1
    return mesh, A, part, B


def gaussian_rhs(mesh, prob, center=None, pol=(1.0, 0.0, 0.0), sigma=0.1):
    if center is None:
        center = tuple(0.5 * L for L in prob.lengths)
    return fem.load_vector(mesh, fem.gaussian_source(center, pol, sigma), prob.bc)


def solve(prob, f=None, restart=50, rtol=1e-6, max_iters=1000, flexible=False, fixed_iters=0):
    mesh, A, part, B = setup(prob)
    if f is None:
        f = gaussian_rhs(mesh, prob)
    res = gmres.gmres(A, f, B, restart=restart, rtol=rtol, max_iters=max_iters,
                      flexible=flexible, fixed_iters=fixed_iters)
    return mesh, A, part, B, f, res
