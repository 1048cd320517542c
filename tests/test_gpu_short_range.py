"""The paper's short-range algorithm (Sec. 5): forces and overlap correction
both through the Verlet neighbour lists, no triangulation (overlap method
"verlet"), against the oracle, whose overlap rounds test every pair by brute
force.  Also the FP32 evaluation of the list force (positions, separations
and the cutoff test stay FP64)."""
import numpy as np
import pytest

import oracle
from paper_1703_02484_amd import binding, synth
from tests._checks import count_overlaps, rel_err
from tests.conftest import gpu_available

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _scale(f):
    return np.abs(f).max()


@pytest.mark.parametrize("n", [50, 3000])
def test_forces_verlet_fp32(n):
    w = synth.make("C3", n=n)
    g = binding.Sim.from_workload(w, fp32=True)
    fo = oracle.forces(w.xy, w.species, w.K, kind="screened", A=w.A, lam=w.lam, cutoff=w.cutoff)
    assert np.abs(g.forces() - fo).max() <= 1e-4 * _scale(fo)


def test_forces_verlet_fp32_power_two_species():
    w = synth.make("C3", n=4000)
    sp = (np.arange(w.n) % 2).astype(np.int32)
    K = np.array([[1.0, -0.3], [0.2, 0.7]])
    g = binding.Sim(w.xy, w.radii, sp, None, K, L=w.L, kind="power", q=6.0, cutoff=2.5, skin=0.5, fp32=True)
    fo = oracle.forces(w.xy, sp, K, kind="power", q=6.0, cutoff=2.5)
    assert np.abs(g.forces() - fo).max() <= 1e-4 * _scale(fo)


def _run(w, steps, tol, graph=False, check_every=10, **over):
    g = binding.Sim.from_workload(w, **over)
    o = oracle.OracleSim.from_workload(w, **over)
    g.set_graph_mode(graph)
    done = 0
    while done < steps:
        k = min(check_every, steps - done)
        g.step(k)
        o.step(k)
        done += k
        xg, tg, sg, stg = g.state()
        xo, to, so, sto = o.state()
        assert rel_err(xg, xo) <= tol, done
        assert sg == so
    for k in ("overlap_rounds_total", "overlap_rounds_max", "overlap_edges_total", "cap_hits", "noise_clamps"):
        assert stg[k] == sto[k], (k, stg[k], sto[k])
    return stg


@pytest.mark.parametrize("graph", [False, True])
def test_trajectory_c3_verlet_overlap_fp64(graph):
    st = _run(synth.make("C3", n=6000), 60, 1e-9, graph=graph, overlap="verlet", fp32=False)
    assert st["overlap_rounds_total"] > 0 and st["verlet_rebuilds"] >= 2


def test_trajectory_c3_verlet_overlap_fp32():
    st = _run(synth.make("C3", n=6000), 60, 1e-4, graph=True, overlap="verlet", fp32=True)
    assert st["overlap_rounds_total"] > 0


def test_trajectory_c3_delaunay_overlap_fp32_forces():
    # the Delaunay overlap method with the FP32 list force, against the FP64 oracle at 1e-4
    st = _run(synth.make("C3", n=6000), 40, 1e-4, graph=True, fp32=True)
    assert st["overlap_rounds_total"] > 0


def test_verlet_overlap_rebuilds_stale_lists_inside_a_step():
    # cutoff 2.0 + skin 0.1 leaves a margin of 0.05: strong noise moves disks farther inside one
    # step, so detections find the lists possibly incomplete; the library rebuilds them mid-step
    n = 800
    L = synth.box_side(n, 0.5)
    xy = synth.rsa(n, L, 1.0, seed=8)
    w = synth.Workload("dense", xy, np.ones(n), np.zeros(n, np.int32), np.zeros(n), 1, np.array([[1.0]]), L=L,
                       D=1.0, dt=2e-3, seed=2, kind="screened", A=1.0, lam=0.5, cutoff=2.0, skin=0.1,
                       overlap="verlet")
    st = _run(w, 10, 1e-9, check_every=1, graph=True)
    assert st["host_continued"] > 0 and st["verlet_rebuilds"] > 10 and st["overlap_rounds_max"] >= 2


def _list_run(w, steps, mode, graph=True, **over):
    g = binding.Sim.from_workload(w, overlap="verlet", **over)
    g.set_tail_mode(mode)
    g.set_graph_mode(graph)
    g.step(steps)
    x, th, step, st = g.state()
    g.close()
    return x, st


def test_verlet_overlap_launch_forms_agree_with_the_oracle():
    # the later list rounds as launches over every disk (form 0), in one workgroup over the disks near
    # those the round before moved (form 1), or the library's mix (form 2): the same positions bit for
    # bit, and the oracle's
    w = synth.make("C3", n=6000)
    runs = {m: _list_run(w, 30, m, fp32=False) for m in (0, 1, 2)}
    o = oracle.OracleSim.from_workload(w, overlap="verlet", fp32=False)
    o.step(30)
    xo = o.state()[0]
    for m, (x, st) in runs.items():
        assert np.array_equal(x, runs[0][0]), m
        assert st["overlap_edges_total"] == runs[0][1]["overlap_edges_total"], m
        assert st["overlap_rounds_total"] > 0
        assert rel_err(x, xo) <= 1e-9, m


def test_verlet_overlap_launch_forms_agree_at_200k():
    # large enough that the library's form launches the first rounds over all disks and runs the rest
    # in one workgroup (it picks the split from the previous steps' rounds)
    w = synth.make("C3", n=200000)
    x0, st0 = _list_run(w, 12, 0)
    x2, st2 = _list_run(w, 12, 2)
    assert np.array_equal(x0, x2)
    assert st0["overlap_edges_total"] == st2["overlap_edges_total"]
    assert st0["overlap_rounds_max"] >= 3 and st0["host_continued"] == st2["host_continued"]
    assert count_overlaps(x2) == 0


def test_verlet_overlap_has_no_triangulation():
    w = synth.make("C3", n=500)
    g = binding.Sim.from_workload(w, overlap="verlet")
    with pytest.raises(binding.BDError):
        g.triangles()
    with pytest.raises(binding.BDError):
        binding.Sim.from_workload(synth.make("C1", n=300), overlap="verlet")   # needs a cutoff


def test_full_size_c3_verlet_overlap():
    # N = 1,048,576: three steps in graph mode, then no pair of disks overlaps (brute force over a k-d
    # tree) and every disk is inside the walls
    w = synth.make("C3")
    g = binding.Sim.from_workload(w, overlap="verlet")
    g.set_graph_mode(True)
    g.step(3)
    x, th, step, st = g.state()
    assert step == 3 and np.all(x >= 1.0) and np.all(x <= w.L - 1.0)
    assert count_overlaps(x) == 0
    assert st["overlap_rounds_total"] > 0
