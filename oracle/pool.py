"""Oracle: the one-level Schwarz preconditioner of dd.Schwarz with its local factorisations and
solves spread over a pool of worker processes.

Test infrastructure only (see oracle/__init__.py).

The local problems are independent, and the paper solves each one on its own core (Sec. 6.1,
one subdomain per processor).  PooledSchwarz does the same on the host's cores: the caller builds
the local matrices A^l exactly as dd.Schwarz does, the workers factor them (dd.factor_local) and
return the local solutions (A^l)^-1 R_l v on request, and the caller forms
z = sum_l R_l^T D_l x_l in subdomain order with the same operations as dd.Schwarz.apply.  The
result equals dd.Schwarz bit for bit (tested); only the wall-clock time differs.

Workers are started with the "spawn" method: they share no memory or device state with the
caller, which may already hold a GPU.
"""
import multiprocessing as mp
import os
import time

import numpy as np

from . import dd, fem


def _worker(conn):
    from threadpoolctl import threadpool_limits
    threadpool_limits(1)  # one core per worker: BLAS threads of many workers would oversubscribe
    lus, sets = {}, {}
    while True:
        msg = conn.recv()
        if msg is None:
            break
        if msg[0] == "factor":
            _, l, Al, idx = msg
            t = time.perf_counter()
            lus[l] = dd.factor_local(Al)
            sets[l] = idx
            conn.send(time.perf_counter() - t)
        else:
            v = msg[1]
            conn.send({l: lu.solve(v[sets[l]]) for l, lu in lus.items()})
    conn.close()


def _solve_one(task):
    from threadpoolctl import threadpool_limits
    threadpool_limits(1)
    Al, r = task
    t = time.perf_counter()
    lu = dd.factor_local(Al)
    t_lu = time.perf_counter() - t
    x = lu.solve(r)
    return x, t_lu, time.perf_counter() - t - t_lu


def solve_many(tasks, workers=None):
    """[(A^l, r), ...] -> [((A^l)^-1 r, seconds of the factorisation, seconds of the solve), ...],
    each pair on a worker process (the same exact local solve as dd.Schwarz.local_solve)."""
    nw = max(1, min(len(tasks), workers or default_workers()))
    with mp.get_context("spawn").Pool(nw) as p:
        return p.map(_solve_one, tasks, chunksize=1)


def default_workers():
    return max(1, min(16, os.cpu_count() or 1))


class PooledSchwarz:
    """z = sum_l R_l^T D_l (A^l)^-1 R_l v (D_l = I for AS), arguments as dd.Schwarz, with the
    factorisations and local solves on `workers` processes (subdomains dealt round-robin, largest
    first).  Use as a context manager, or call close().  t_lu holds each subdomain's factorisation
    time as measured in its worker; t_setup the wall-clock time of all of them."""

    def __init__(self, part, A, kind, k, xi, bc=fem.BC_IMPEDANCE, workers=None, local=None):
        self.kind = kind
        self.sets = part.local_set(kind)
        self.D = [part.pou(l, kind) if kind in (dd.RAS, dd.ORAS) else None for l in range(part.N)]
        self.n = A.shape[0]
        loc = local if local is not None else dd.local_matrices(part, A, kind, k, xi, bc)
        N = part.N
        nw = min(N, workers or default_workers())
        ctx = mp.get_context("spawn")
        self.conns, self.procs = [], []
        for _ in range(nw):
            a, b = ctx.Pipe()
            p = ctx.Process(target=_worker, args=(b,), daemon=True)
            p.start()
            b.close()
            self.conns.append(a)
            self.procs.append(p)
        order = sorted(range(N), key=lambda l: -loc[l].shape[0])
        self.owner = {l: i % nw for i, l in enumerate(order)}
        t0 = time.perf_counter()
        for l in order:
            self.conns[self.owner[l]].send(("factor", l, loc[l], self.sets[l]))
        self.t_lu = {}
        for l in order:
            self.t_lu[l] = self.conns[self.owner[l]].recv()
        self.t_setup = time.perf_counter() - t0

    def local_solves(self, v):
        v = np.ascontiguousarray(v, np.complex128)
        for c in self.conns:
            c.send(("solve", v))
        local = {}
        for c in self.conns:
            local.update(c.recv())
        return local

    def apply(self, v):
        local = self.local_solves(v)
        z = np.zeros(self.n, dtype=np.complex128)
        for l, idx in enumerate(self.sets):
            x = local[l]
            if self.D[l] is not None:
                x = self.D[l] * x
            np.add.at(z, idx, x)
        return z

    __call__ = apply

    def close(self):
        for c in self.conns:
            try:
                c.send(None)
                c.close()
            except (OSError, BrokenPipeError):
                pass
        for p in self.procs:
            p.join(timeout=30)
            if p.is_alive():
                p.kill()
        self.conns, self.procs = [], []

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        if getattr(self, "procs", None):
            self.close()
