"""Host-side checks of bench.py: the one-GPU guard and the headline workload's description."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    """--gpus 2 exits with status 2 and a message, before any device is touched."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one MI355X" in r.stderr and r.stdout == ""


def test_headline_batch_instances():
    """Six solves: ORAS and AS, each at xi = k, k^1.5 and k^2 (exponents of k); each xi has one
    right-hand side seed, shared by ORAS and AS."""
    inst = bench.instances("scale")
    assert sorted((k, e) for k, e, _ in inst) == sorted(
        (k, e) for k in ("oras", "as") for e in (1.0, 1.5, 2.0))
    assert sorted({s for _, _, s in inst}) == [0, 1, 2]
    assert all(len({s for _, e2, s in inst if e2 == e}) == 1 for _, e, _ in inst)
    with pytest.raises(SystemExit):
        bench.instances("no-such-workload")


def test_headline_dof_count_matches_mesh():
    """The DOF count quoted in the workload description is the library mesh's edge count, and
    both equal the closed form for n^3 cubes split into 6 tetrahedra each: axis edges
    3n(n+1)^2, face diagonals 3n^2(n+1) and body diagonals n^3."""
    from paper_1711_03789_amd import mx
    w, cfg = bench.workload_desc("scale")
    n = w.n[0]
    assert w.n == (n, n, n)
    closed = 3 * n * (n + 1) ** 2 + 3 * n * n * (n + 1) + n ** 3
    assert "{:,} complex DOFs".format(closed) in cfg["workload"]
    assert mx.Mesh(*w.n, *w.lengths).n_edge == closed
