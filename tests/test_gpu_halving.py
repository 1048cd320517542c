"""Sec. 4.3: a move that reverses a Delaunay edge is discarded and the step
redone in halves (max_dt_halvings levels), with Brownian-bridge noise keyed
like the step's own draws.  The library (host-driven halves on the device)
against the oracle: positions, angles, triangulations and every counter."""
import numpy as np
import pytest

import oracle
from paper_1703_02484_amd import binding, synth
from tests._checks import rel_err, tri_set
from tests.conftest import gpu_available
from tests.test_oracle import reversal_case

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

COUNTERS = ("reversals", "dt_halvings", "overlap_rounds_total", "overlap_edges_total", "cap_hits", "noise_clamps")


def _compare(g, o, tol):
    xg, tg, sg, stg = g.state()
    xo, to, so, sto = o.state()
    assert sg == so
    assert rel_err(xg, xo) <= tol
    assert np.abs(tg - to).max() <= max(tol, 1e-12)
    assert tri_set(g.triangles()) == tri_set(o.triangles())
    for k in COUNTERS:
        assert stg[k] == sto[k], (k, stg[k], sto[k])
    return stg


@pytest.mark.parametrize("levels", [1, 3])
@pytest.mark.parametrize("graph", [False, True])
def test_reversal_case_halved(levels, graph):
    xy, th, kw = reversal_case()
    n = xy.shape[0]
    args = (xy, np.ones(n), np.zeros(n, np.int32), th, np.zeros((1, 1)))
    g = binding.Sim(*args, max_dt_halvings=levels, **kw)
    g.set_graph_mode(graph)
    o = oracle.OracleSim(*args, max_dt_halvings=levels, **kw)
    g.step(1)
    o.step(1)
    st = _compare(g, o, 1e-12)
    assert st["dt_halvings"] >= 1


@pytest.mark.parametrize("graph", [False, True])
def test_huge_noise_steps_halved(graph):
    # noise amplitude ~2.8 per step: disks swap places often; up to 3 halvings per step, with
    # self-propulsion and rotational noise in the bridge
    n = 30
    # a slightly jittered lattice: an exact one has cocircular cells, whose Delaunay triangulation is not
    # unique, and the first step's reversal count would depend on the diagonals each side chose
    jitter = np.random.default_rng(6).uniform(-0.05, 0.05, size=(n, 2))
    xy = np.array([[50.0 + 2.2 * (i % 15), 50.0 + 2.3 * (i // 15)] for i in range(n)]) + jitter
    th = np.linspace(0.0, 6.0, n)
    kw = dict(L=200.0, D=1.0, dt=4.0, seed=1, v0=0.3, Dr=0.5, max_dt_halvings=3)
    args = (xy, np.ones(n), np.zeros(n, np.int32), th, np.zeros((1, 1)))
    g = binding.Sim(*args, **kw)
    g.set_graph_mode(graph)
    o = oracle.OracleSim(*args, **kw)
    for _ in range(4):
        g.step(1)
        o.step(1)
        st = _compare(g, o, 1e-9)
    assert st["dt_halvings"] >= 2 and st["reversals"] >= 2


def test_halving_dense_workload_matches_oracle():
    # a dense box with a time step large enough for occasional reversals among many disks
    n = 600
    L = synth.box_side(n, 0.45)
    xy = synth.rsa(n, L, 1.0, seed=4)
    w = synth.Workload("dense", xy, np.ones(n), np.zeros(n, np.int32), np.zeros(n), 1, np.array([[1e-2]]), L=L,
                       D=1.0, dt=0.2, seed=9, max_dt_halvings=4)
    g = binding.Sim.from_workload(w)
    g.set_graph_mode(True)
    o = oracle.OracleSim.from_workload(w)
    for _ in range(3):
        g.step(2)
        o.step(2)
        st = _compare(g, o, 1e-9)
    assert st["dt_halvings"] >= 1


def test_halving_off_is_bitwise_unchanged():
    w = synth.make("C1", n=700)
    a = binding.Sim.from_workload(w)
    b = binding.Sim.from_workload(w, max_dt_halvings=5)
    a.step(15)
    b.step(15)
    assert np.array_equal(a.state()[0], b.state()[0])
    assert b.state()[3]["dt_halvings"] == 0


def test_halving_rejections():
    w = synth.make("C1", n=300)
    with pytest.raises(binding.BDError):
        binding.Sim.from_workload(w, max_dt_halvings=13)
    g = binding.Sim.from_workload(w, max_dt_halvings=2)
    with pytest.raises(binding.BDError):
        g.adjoint_begin(2, 1)
