"""Parity of the HIP path (through the C-ABI) with the CPU oracle.

Tolerances: positions |x_gpu - x_orc| / max(|x_orc|, 1) <= 1e-9 with FP64
forces and <= 1e-4 with FP32 forces; the triangulation is compared exactly
(same triangle set as the oracle's Delaunay triangulation).
"""
import math
import os

import numpy as np
import pytest
from scipy.spatial import Delaunay as QhullDelaunay

import oracle
from paper_1703_02484_amd import binding, synth
from tests._checks import check_delaunay, count_overlaps, rel_err, tri_set
from tests.conftest import gpu_available

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _pair(w, **over):
    return binding.Sim.from_workload(w, **over), oracle.OracleSim.from_workload(w, **over)


def _force_scale(f):
    return np.abs(f).max()


# ------------------------------------------------------------------ forces
def test_forces_fp64_c1():
    w = synth.make("C1")
    g = binding.Sim.from_workload(w)
    fo = oracle.forces(w.xy, w.species, w.K)
    fg = g.forces()
    assert np.abs(fg - fo).max() <= 1e-12 * _force_scale(fo)


@pytest.mark.parametrize("n", [3, 100, 1000, 4099])
def test_forces_fp32_ragged(n):
    w = synth.make("C2", n=n)
    g = binding.Sim.from_workload(w)
    fo = oracle.forces(w.xy, w.species, w.K)
    fg = g.forces()
    assert np.abs(fg - fo).max() <= 1e-4 * _force_scale(fo)


def test_forces_fp64_general_power_and_screened():
    w = synth.make("C1", n=777)
    for kw in (dict(kind="power", q=6.0), dict(kind="screened", A=1.0, lam=0.5, cutoff=2.5)):
        g = binding.Sim.from_workload(w, **kw)
        fo = oracle.forces(w.xy, w.species, w.K, **kw)
        fg = g.forces()
        assert np.abs(fg - fo).max() <= 1e-11 * max(_force_scale(fo), 1e-300)


def test_forces_full_size_c2_sampled():
    w = synth.make("C2")
    g = binding.Sim.from_workload(w)
    fg = g.forces()
    rng = np.random.default_rng(0)
    idx = np.sort(rng.choice(w.n, 512, replace=False))
    fo = oracle.forces(w.xy, w.species, w.K, idx=idx)
    scale = np.abs(fo).max()
    assert np.abs(fg[idx] - fo).max() <= 1e-4 * scale


# ------------------------------------------------------------------ triangulation
def test_frame_matches_oracle():
    for w in (synth.make("C1"), synth.make("C3", n=3000)):
        g = binding.Sim.from_workload(w)
        assert np.array_equal(g.frame(), oracle.frame(w.L, 1.0))


def test_initial_triangulation_matches_oracle():
    for w in (synth.make("C1"), synth.make("C2", n=5000), synth.make("C3", n=3000)):
        g = binding.Sim.from_workload(w)
        assert tri_set(g.triangles()) == tri_set(oracle.delaunay_with_frame(w.xy, w.L, 1.0))


FIG_L = 60.0


def _load_fig(name):
    pts, moved = {}, {}
    for ln in open(os.path.join(GOLDEN, name)):
        f = ln.split()
        if not f or f[0].startswith("#"):
            continue
        if f[0] == "point":
            pts[f[1]] = (float(f[2]), float(f[3]))
        elif f[0] == "moved":
            moved[f[1]] = (float(f[2]), float(f[3]))
    names = "".join(sorted(pts))
    # centred in a 60-box, far from the wall frame, so the figure's own
    # triangles are Delaunay with the frame present
    xy = np.array([pts[k] for k in names]) + 27.0
    xy2 = xy.copy()
    for k, v in moved.items():
        xy2[names.index(k)] = np.array(v) + 27.0
    return names, xy, xy2


def _small_sim(xy):
    n = xy.shape[0]
    return binding.Sim(xy, np.full(n, 0.1), np.zeros(n, np.int32), None, np.array([[0.0]]), L=FIG_L)


def _fig_tris(g, names):
    # triangles among the figure's own points
    return {"".join(sorted(names[i] for i in t)) for t in g.triangles().tolist() if max(t) < len(names)}


def _fig_dt(xy, names):
    return {"".join(sorted(names[i] for i in t)) for t in oracle.delaunay_with_frame(xy, FIG_L, 0.1).tolist()
            if max(t) < len(names)}


def test_fig5_single_inversion_then_lawson():
    names, xy, xy2 = _load_fig("fig5_inverted_tri1.txt")
    g = _small_sim(xy)
    assert tri_set(g.triangles()) == tri_set(oracle.delaunay_with_frame(xy, FIG_L, 0.1))
    assert _fig_tris(g, names) == {"acd", "bcd", "bce", "bde"}      # panel (a)
    g.set_positions(xy2)
    st = g.state()[3]
    assert tri_set(g.triangles()) == tri_set(oracle.delaunay_with_frame(xy2, FIG_L, 0.1))
    assert _fig_tris(g, names) == {"abc", "abd", "bcd", "cde"}      # panel (d)
    assert st["inversion_flips"] >= 1 and st["flips_total"] >= 2
    assert st["kinetic_repairs"] == 0 and st["host_rebuilds"] == 0


def test_fig6_two_edge_crossing_is_replayed_on_device():
    names, xy, xy2 = _load_fig("fig6_inverted_tri2.txt")
    g = _small_sim(xy)
    g.set_positions(xy2)
    st = g.state()[3]
    assert tri_set(g.triangles()) == tri_set(oracle.delaunay_with_frame(xy2, FIG_L, 0.1))
    assert _fig_tris(g, names) == {"abe", "bef", "bcf", "cdf", "def"}
    assert st["kinetic_repairs"] == 1 and st["host_rebuilds"] == 0


# ------------------------------------------------------------------ trajectories
def _run_parity(w, steps, tol, check_every=10, graph=False, tail_mode=-1, gpu_over=None, **over):
    """Steps the library and the oracle side by side; every check_every steps the positions, angles,
    step counter and triangle sets are compared.  graph: the library replays captured steps (queued
    check_every at a time); tail_mode: how its overlap rounds are launched; gpu_over: options for the
    library only (e.g. a pinned force form)."""
    g = binding.Sim.from_workload(w, **over, **(gpu_over or {}))
    o = oracle.OracleSim.from_workload(w, **over)
    g.set_tail_mode(tail_mode)
    g.set_graph_mode(graph)
    worst = 0.0
    done = 0
    while done < steps:
        k = min(check_every, steps - done)
        if graph:
            g.step(k)
        else:
            for _ in range(k):
                g.step(1)
        o.step(k)
        done += k
        xg, tg, sg, stg = g.state()
        xo, to, so, sto = o.state()
        worst = max(worst, rel_err(xg, xo))
        assert worst <= tol, (done, worst)
        assert np.abs(tg - to).max() <= max(tol, 1e-12)
        assert sg == so
        assert tri_set(g.triangles()) == tri_set(o.triangles()), done
    stg, sto = g.state()[3], o.state()[3]
    for k in ("overlap_rounds_total", "overlap_rounds_max", "overlap_edges_total", "reversals", "noise_clamps"):
        assert stg[k] == sto[k], (k, stg[k], sto[k])
    assert stg["host_rebuilds"] == 0
    return worst, stg


def test_trajectory_c1_fp64_100_steps():
    worst, st = _run_parity(synth.make("C1"), 100, 1e-9)
    assert st["overlap_rounds_total"] > 0


def test_trajectory_c2_fp32_reduced_100_steps():
    worst, st = _run_parity(synth.make("C2", n=4096), 100, 1e-4)
    assert st["flips_total"] > 0


@pytest.mark.parametrize("tail_mode", [0, 1, 2])
def test_trajectory_c1_fp64_100_steps_graph(tail_mode):
    # graph replay (the benchmark's mode) against the oracle directly, both overlap-round launch forms
    worst, st = _run_parity(synth.make("C1"), 100, 1e-9, graph=True, tail_mode=tail_mode)
    assert st["overlap_rounds_total"] > 0


@pytest.mark.parametrize("tail_mode", [0, 1, 2])
def test_trajectory_c2_fp32_reduced_100_steps_graph(tail_mode):
    worst, st = _run_parity(synth.make("C2", n=4096), 100, 1e-4, graph=True, tail_mode=tail_mode)
    assert st["flips_total"] > 0


@pytest.mark.parametrize("pin", [-1, -2, -3])
def test_trajectory_c2_fp32_symmetric_graph_launch_per_phase(pin):
    # the timed C2 path at reduced size: symmetric force, graph replay, overlap rounds launched per phase
    worst, st = _run_parity(synth.make("C2", n=3000), 100, 1e-4, graph=True, tail_mode=0,
                            gpu_over=dict(force_chunk=pin))
    assert st["overlap_rounds_total"] > 0


def test_reversal_count_exact_for_a_disk_driven_through_its_neighbour():
    # the oracle's pinned case (one Delaunay edge reverses; Sec. 4.3 criterion) through the library
    from tests.test_oracle import reversal_case

    xy, th, kw = reversal_case()
    n = xy.shape[0]
    g = binding.Sim(xy, np.ones(n), np.zeros(n, np.int32), th, np.zeros((1, 1)), **kw)
    o = oracle.OracleSim(xy, np.ones(n), np.zeros(n, np.int32), th, np.zeros((1, 1)), **kw)
    g.step(1)
    o.step(1)
    assert g.state()[3]["reversals"] == 1 == o.state()[3]["reversals"]
    assert rel_err(g.state()[0], o.state()[0]) <= 1e-12
    assert tri_set(g.triangles()) == tri_set(o.triangles())


def test_trajectory_c5_contact_factor_fp64():
    _run_parity(synth.make("C5", n=2048), 50, 1e-9)


def test_trajectory_dense_strong_noise():
    # dense box, noise amplitude ~0.2 per step: many overlap rounds and cap truncations
    n = 600
    L = synth.box_side(n, 0.5)
    xy = synth.rsa(n, L, 1.0, seed=8)
    w = synth.Workload("dense", xy, np.ones(n), np.zeros(n, np.int32), np.zeros(n), 1, np.array([[0.0]]), L=L,
                       D=1.0, dt=2e-2, seed=2)
    worst, st = _run_parity(w, 12, 1e-9, check_every=1)
    assert st["cap_hits"] > 0 and st["overlap_rounds_max"] >= 3


def test_large_moves_repaired_on_device():
    # in a dilute box, 2% of the disks jump 1.5-3 units: some cross more than
    # one edge, which the device resolves by replaying the move in sub-steps
    rng = np.random.default_rng(3)
    n = 3000
    L = synth.box_side(n, 0.15)
    xy = synth.rsa(n, L, 1.0, seed=3)
    g = binding.Sim(xy, np.ones(n), np.zeros(n, np.int32), None, np.array([[0.0]]), L=L)
    moved = xy.copy()
    pick = rng.choice(n, n // 50, replace=False)
    ang = rng.uniform(0, 2 * np.pi, pick.size)
    rad = rng.uniform(1.5, 3.0, pick.size)
    target = moved[pick] + np.column_stack([rad * np.cos(ang), rad * np.sin(ang)])
    inside = np.all((target > 1.0) & (target < L - 1.0), axis=1)   # jumps leaving the box are skipped
    moved[pick[inside]] = target[inside]
    g.set_positions(moved)
    st = g.state()[3]
    assert tri_set(g.triangles()) == tri_set(oracle.delaunay_with_frame(moved, L, 1.0))
    assert st["kinetic_repairs"] >= 1 and st["host_rebuilds"] == 0


def test_full_size_c2_bench_configuration():
    # the configuration the benchmark times: 3 steps, then properties at full size
    w = synth.make("C2")
    g = binding.Sim.from_workload(w)
    g.step(3)
    x, th, step, st = g.state()
    assert step == 3
    assert np.all(x >= 1.0) and np.all(x <= w.L - 1.0)
    tris = g.triangles()
    pts = np.concatenate([x, g.frame()])
    check_delaunay(pts, tris)
    assert tri_set(tris) == tri_set(QhullDelaunay(pts).simplices)
    assert count_overlaps(x) == 0
    assert st["host_rebuilds"] == 0


def test_full_size_c2_bench_path_matches_oracle():
    # the timed path itself at full size (N = 65,536): the force form the autotuner picks there (the symmetric
    # form), graph replay with steps queued together, the default overlap-round launch form (the large
    # phases launched one by one, the rest in one workgroup, above 16,384 disks); 3 steps against the
    # oracle, element by element
    w = synth.make("C2")
    g = binding.Sim.from_workload(w)
    cfg = g.force_config()
    assert cfg["persistent"] == 2 and cfg["tuned"] in (1, 2), cfg
    g.set_graph_mode(True)
    g.step(3)
    o = oracle.OracleSim.from_workload(w)
    o.step(3)
    xg, tg, sg, stg = g.state()
    xo, to, so, sto = o.state()
    assert sg == so == 3
    assert rel_err(xg, xo) <= 1e-4
    assert np.abs(tg - to).max() <= 1e-12     # angles do not depend on forces
    assert tri_set(g.triangles()) == tri_set(o.triangles())
    for k in ("overlap_rounds_total", "overlap_rounds_max", "overlap_edges_total", "reversals", "noise_clamps"):
        assert stg[k] == sto[k], (k, stg[k], sto[k])
    assert stg["overlap_rounds_total"] > 0 and stg["host_rebuilds"] == 0


# ------------------------------------------------------------------ determinism, resume, errors
def test_bitwise_run_to_run():
    w = synth.make("C2", n=3000)
    a = binding.Sim.from_workload(w)
    b = binding.Sim.from_workload(w)
    a.step(15)
    b.step(15)
    assert np.array_equal(a.state()[0], b.state()[0])
    assert tri_set(a.triangles()) == tri_set(b.triangles())


def test_resume_from_state():
    w = synth.make("C1", n=800)
    a = binding.Sim.from_workload(w)
    a.step(20)
    full = a.state()[0]
    b = binding.Sim.from_workload(w)
    b.step(10)
    xy, th, step, _ = b.state()
    c = binding.Sim(xy, w.radii, w.species, th, w.K, L=w.L, D=w.D, dt=w.dt, seed=w.seed, step0=step)
    c.step(10)
    assert rel_err(c.state()[0], full) <= 1e-12


def test_round_cap_reports_no_convergence_and_rolls_back():
    n = 400
    L = synth.box_side(n, 0.5)
    xy = synth.rsa(n, L, 1.0, seed=8)
    g = binding.Sim(xy, np.ones(n), np.zeros(n, np.int32), None, np.array([[0.0]]), L=L, D=1.0, dt=2e-3, seed=2,
                    max_overlap_rounds=1)
    before = None
    with pytest.raises(binding.BDError) as e:
        for _ in range(20):
            before = g.state()[0]
            g.step(1)
    assert e.value.code == -3
    after, _, _, _ = g.state()
    assert np.array_equal(after, before)
    check_delaunay(np.concatenate([after, g.frame()]), g.triangles())


# ------------------------------------------------------------------ short-range (Verlet) path
@pytest.mark.parametrize("n", [50, 3000])
def test_forces_verlet_screened(n):
    w = synth.make("C3", n=n)
    g = binding.Sim.from_workload(w, fp32=False)
    fo = oracle.forces(w.xy, w.species, w.K, kind="screened", A=w.A, lam=w.lam, cutoff=w.cutoff)
    fg = g.forces()
    assert np.abs(fg - fo).max() <= 1e-12 * max(_force_scale(fo), 1e-300)


def test_forces_verlet_power_two_species():
    # the paper's short-range law r/r^7 with a cutoff and a non-reciprocal 2x2 K
    w = synth.make("C3", n=4000)
    sp = (np.arange(w.n) % 2).astype(np.int32)
    K = np.array([[1.0, -0.3], [0.2, 0.7]])
    g = binding.Sim(w.xy, w.radii, sp, None, K, L=w.L, kind="power", q=6.0, cutoff=2.5, skin=0.5)
    fo = oracle.forces(w.xy, sp, K, kind="power", q=6.0, cutoff=2.5)
    assert np.abs(g.forces() - fo).max() <= 1e-12 * _force_scale(fo)


def test_trajectory_c3_verlet_reduced():
    worst, st = _run_parity(synth.make("C3", n=6000), 60, 1e-9, gpu_over=dict(fp32=False))
    assert st["verlet_rebuilds"] >= 2


def test_full_size_c3_verlet():
    # the short-range workload at full size (N = 1,048,576): sampled forces
    # against the oracle, then 2 steps and the properties of the result
    w = synth.make("C3")
    g = binding.Sim.from_workload(w)   # FP32 list force, as the workload asks
    rng = np.random.default_rng(1)
    idx = np.sort(rng.choice(w.n, 256, replace=False))
    fo = oracle.forces(w.xy, w.species, w.K, kind="screened", A=w.A, lam=w.lam, cutoff=w.cutoff, idx=idx)
    fg = g.forces()
    assert np.abs(fg[idx] - fo).max() <= 1e-4 * _force_scale(fo)
    g.step(2)
    x, th, step, st = g.state()
    assert step == 2 and np.all(x >= 1.0) and np.all(x <= w.L - 1.0)
    check_delaunay(np.concatenate([x, g.frame()]), g.triangles())
    assert count_overlaps(x) == 0
    assert st["host_rebuilds"] == 0


def test_verlet_list_capacity_grows():
    # cutoff 7 + skin 1 at phi = 0.5: about 32 neighbours per disk, more than the
    # initial list capacity; the build grows the lists once and forces stay exact
    w = synth.make("C3", n=3000)
    g = binding.Sim.from_workload(w, cutoff=7.0, skin=1.0, fp32=False)
    fo = oracle.forces(w.xy, w.species, w.K, kind="screened", A=w.A, lam=w.lam, cutoff=7.0)
    fg = g.forces()
    assert np.abs(fg - fo).max() <= 1e-12 * _force_scale(fo)
    g.step(5)
    o = oracle.OracleSim.from_workload(w, cutoff=7.0)
    o.step(5)
    assert rel_err(g.state()[0], o.state()[0]) <= 1e-9


def test_verlet_list_capacity_exceeded_is_an_error(capfd):
    # cutoff 15: over 96 neighbours per disk, beyond the largest list capacity
    w = synth.make("C3", n=3000)
    with pytest.raises(binding.BDError) as e:
        binding.Sim.from_workload(w, cutoff=15.0, skin=1.0)
    assert e.value.code == -1
    assert "capacity" in capfd.readouterr().err
