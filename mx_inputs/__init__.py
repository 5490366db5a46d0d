"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle's callers.

Holds no arithmetic of the method: only random draws and the workload descriptions (mesh sizes,
wavenumbers, subdomain counts) of the unit-cube experiments of the paper's Sec. 6, so that the
oracle and the GPU library receive identical inputs.
"""
import math

import numpy as np

ORAS, RAS, AS = "oras", "ras", "as"


def random_rhs(n_dof, seed):
    """Per-DOF complex Gaussian load b_e = (N(0,1) + i N(0,1)) / sqrt(2), PCG64(seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    re = rng.standard_normal(n_dof)
    im = rng.standard_normal(n_dof)
    return (re + 1j * im) / math.sqrt(2.0)


def jittered_cuts(n_cubes, n_parts, rel, seed):
    """Cut planes of n_parts boxes along an axis of n_cubes cubes: the interior planes are moved
    from the even position by round(U(-rel, rel) * box width)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w = n_cubes / n_parts
    cuts = [0]
    for i in range(1, n_parts):
        c = int(round(i * w + round(rng.uniform(-rel, rel) * w)))
        c = max(cuts[-1] + 1, min(c, n_cubes - (n_parts - i)))
        cuts.append(c)
    cuts.append(n_cubes)
    return cuts


class Workload:
    """One solve: box of n cubes per axis, wavenumber k, absorption xi, px*py*pz subdomains."""

    def __init__(self, name, n, lengths, k, xi, parts, layers, kind, restart, rtol=1e-6,
                 rhs="gaussian", seed=0, cuts=None, center=None, pol=(1.0, 0.0, 0.0),
                 sigma=0.1, precision="c128"):
        self.name, self.n, self.lengths, self.k, self.xi = name, tuple(n), tuple(lengths), k, xi
        self.parts, self.layers, self.kind, self.restart, self.rtol = tuple(parts), layers, kind, restart, rtol
        self.rhs, self.seed, self.cuts, self.pol, self.sigma = rhs, seed, cuts, pol, sigma
        self.center = center if center is not None else tuple(0.5 * L for L in self.lengths)
        self.precision = precision

    def describe(self):
        return {"workload": self.name, "cubes": list(self.n), "lengths": list(self.lengths),
                "k": self.k, "xi": self.xi, "subdomains": list(self.parts),
                "overlap_layers": self.layers, "kind": self.kind, "restart": self.restart,
                "rtol": self.rtol, "rhs": self.rhs, "seed": self.seed, "precision": self.precision}


def config_small(kind=ORAS, xi=None, precision="c128"):
    """Unit cube 8^3 cubes x 6 tets, k = 4, xi = k^2, impedance, Gaussian (sigma 0.1)
    x-polarised source at the centre, 2x2x2 subdomains, 2 layers, GMRES(50)."""
    k = 4.0
    return Workload("unit-cube 8^3, k=4", (8, 8, 8), (1, 1, 1), k, k * k if xi is None else xi,
                    (2, 2, 2), 2, kind, 50, precision=precision)


def config_scale(kind=ORAS, xi_exp=2.0, seed=0):
    """Unit cube 64^3 cubes x 6 tets (1,872,064 DOFs), k = 16, xi = k^xi_exp (1, 1.5 or 2),
    4x4x4 subdomains, 2 layers, GMRES(100), seeded complex Gaussian per-DOF load."""
    k = 16.0
    return Workload("unit-cube 64^3, k=16, xi=k^%g" % xi_exp, (64, 64, 64), (1, 1, 1), k,
                    k ** xi_exp, (4, 4, 4), 2, kind, 100, rhs="random", seed=seed)


def config_medium(kind=ORAS, xi_exp=2.0, seed=0, n=32, parts=4):
    """Unit cube 32^3 cubes x 6 tets (238,688 DOFs), k = 8, xi = k^xi_exp, 4x4x4 subdomains
    (every class of box: corner, edge, face, interior), 2 layers, GMRES(100), seeded complex
    Gaussian per-DOF load: the 64^3 benchmark problem at half the resolution and wavenumber."""
    k = 8.0
    return Workload("unit-cube %d^3, k=8, xi=k^%g" % (n, xi_exp), (n, n, n), (1, 1, 1), k,
                    k ** xi_exp, (parts, parts, parts), 2, kind, 100, rhs="random", seed=seed)


def config_order2(kind=ORAS, xi_exp=2.0, seed=0):
    """Unit cube 24^3 cubes x 6 tets with second-order Nedelec elements (542,736 DOFs), k = 12
    (about 12.6 cubes, 25 DOFs per direction, per wavelength), xi = k^xi_exp, 4x4x4 subdomains,
    1 layer (minimal overlap), GMRES(100), seeded complex Gaussian per-DOF load; the coarse mesh
    of 4^3 cubes (ratio 6: about two coarse cubes per wavelength)."""
    k = 12.0
    return Workload("unit-cube 24^3 order 2, k=12, xi=k^%g" % xi_exp, (24, 24, 24), (1, 1, 1), k,
                    k ** xi_exp, (4, 4, 4), 1, kind, 100, rhs="random", seed=seed)


def config_batching(seed=0):
    """Box [0,1]x[0,1]x[0,2], 96x96x192 cubes, k = xi = 24, 6x6x12 subdomains with cut planes
    jittered by +-20 % of the box width, complex64 factors."""
    cx = jittered_cuts(96, 6, 0.2, seed)
    cy = jittered_cuts(96, 6, 0.2, seed + 1)
    cz = jittered_cuts(192, 12, 0.2, seed + 2)
    return Workload("box 96x96x192, k=24", (96, 96, 192), (1, 1, 2), 24.0, 24.0, (6, 6, 12), 2,
                    ORAS, 50, cuts=(cx, cy, cz), center=(0.5, 0.5, 1.0), precision="c64")


def serving_requests(n_requests, rate, seed):
    """Poisson arrivals at `rate` per second; each request draws k ~ U[4,16], xi in {k, k^2},
    n = ceil(k^1.5) + 4 cubes per side, p = clamp(ceil(n/17), 2, 4) subdomains per side, a Gaussian
    source with centre in [0.35, 0.65]^3 and a random unit polarisation."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    for i in range(n_requests):
        t += rng.exponential(1.0 / rate)
        k = rng.uniform(4.0, 16.0)
        xi = k if rng.uniform() < 0.5 else k * k
        n = int(math.ceil(k ** 1.5)) + 4
        p = min(4, max(2, int(math.ceil(n / 17))))
        c = rng.uniform(0.35, 0.65, size=3)
        pol = rng.standard_normal(3)
        pol /= np.linalg.norm(pol)
        out.append({"id": i, "arrival": t, "k": k, "xi": xi, "n": n, "p": p,
                    "center": tuple(c), "pol": tuple(pol)})
    return out
