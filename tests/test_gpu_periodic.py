"""The periodic box of the paper's own domain (Sec. 2.1).  Short-range path
of Sec. 5: minimum-image list forces, neighbour lists whose cell grid wraps
around, overlap rounds over the lists.  Delaunay path: the triangulation of
the flat torus (2n triangles, no infinite vertex), repaired by flips whose
predicates read every quad at its nearest images, overlap rounds over its
edges, minimum-image all-pairs forces.  Positions are folded into [0, L)
after every move.  Against the oracle (brute-force minimum-image forces, the
torus triangulation rebuilt from scratch after every move), element by
element, then the full-size workloads on sampled forces and by brute-force
properties."""
import numpy as np
import pytest
from scipy.spatial import cKDTree

import oracle
from paper_1703_02484_amd import binding, synth
from tests.conftest import gpu_available

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _per_err(a, b, L):
    # positions folded into [0, L): compare through the nearest image, relative to max(|x|, 1)
    d = a - b
    d -= L * np.rint(d / L)
    return float(np.max(np.abs(d) / np.maximum(np.abs(b), 1.0)))


def _workload(n, fp32):
    w = synth.make("C3", n=n, periodic=True)
    w.overlap = "verlet"
    w.fp32_forces = fp32
    return w


@pytest.mark.parametrize("fp32", [False, True])
def test_periodic_list_forces_match_oracle(fp32):
    w = _workload(3000, fp32)
    g = binding.Sim.from_workload(w)
    fo = oracle.forces(w.xy, w.species, w.K, kind="screened", A=w.A, lam=w.lam, cutoff=w.cutoff, period=w.L)
    fg = g.forces()
    assert np.abs(fg - fo).max() <= (1e-4 if fp32 else 1e-12) * np.abs(fo).max()
    # pairs across the boundary contribute: the walls' forces differ there
    fw = oracle.forces(w.xy, w.species, w.K, kind="screened", A=w.A, lam=w.lam, cutoff=w.cutoff)
    assert np.abs(fw - fo).max() > 1e-3 * np.abs(fo).max()


@pytest.mark.parametrize("fp32,graph", [(False, False), (False, True), (True, True)])
def test_periodic_trajectory_matches_oracle(fp32, graph):
    w = _workload(5000, fp32)
    g = binding.Sim.from_workload(w)
    o = oracle.OracleSim.from_workload(w)
    g.set_graph_mode(graph)
    tol = 1e-4 if fp32 else 1e-9
    for done in range(10, 61, 10):
        g.step(10)
        o.step(10)
        xg, tg, sg, stg = g.state()
        xo, to, so, sto = o.state()
        assert sg == so == done
        assert _per_err(xg, xo, w.L) <= tol, done
        assert xg.min() >= 0.0 and xg.max() < w.L
    for k in ("overlap_rounds_total", "overlap_rounds_max", "overlap_edges_total", "cap_hits", "noise_clamps"):
        assert stg[k] == sto[k], (k, stg[k], sto[k])
    assert stg["overlap_rounds_total"] > 0 and stg["verlet_rebuilds"] >= 2
    # disks did cross the boundary
    x0 = w.xy
    assert np.any(np.abs(xg - x0) > 0.5 * w.L)


def test_periodic_full_size_properties():
    w = _workload(1048576, True)
    g = binding.Sim.from_workload(w)
    g.set_graph_mode(True)
    g.step(5)
    xg, _, step, st = g.state()
    assert step == 5 and st["host_rebuilds"] == 0
    assert xg.min() >= 0.0 and xg.max() < w.L
    # no two disks closer than contact, through the boundary too
    tree = cKDTree(xg, boxsize=w.L)
    assert len(tree.query_pairs(2.0 * (1.0 - 1e-9))) == 0
    rng = np.random.default_rng(11)
    idx = rng.choice(w.n, 300, replace=False).astype(np.int32)
    fo = oracle.forces(xg, w.species, w.K, kind="screened", A=w.A, lam=w.lam, cutoff=w.cutoff, period=w.L,
                       idx=idx)
    assert np.abs(g.forces()[idx] - fo).max() <= 1e-4 * np.abs(fo).max()


def test_periodic_box_limits():
    w = _workload(500, False)
    c = synth.make("C1", n=500, periodic=True)
    with pytest.raises(binding.BDError):   # all pairs in a periodic box: the one-workgroup-per-tile form only
        binding.Sim.from_workload(c, force_chunk=-1)
    with pytest.raises(binding.BDError):   # no adjoint in a periodic box
        binding.Sim.from_workload(c).adjoint_begin(5, 5)
    with pytest.raises(binding.BDError):   # position outside [0, L)
        xy = w.xy.copy()
        xy[0, 0] = w.L
        binding.Sim(xy, w.radii, w.species, None, w.K, L=w.L, kind="screened", cutoff=2.5, skin=0.5,
                    overlap="verlet", periodic=True)


def _tris(tris):
    return {tuple(sorted(map(int, t))) for t in tris}


def _delaunay_run(w, steps, tol, graph, check_every=10):
    g = binding.Sim.from_workload(w)
    o = oracle.OracleSim.from_workload(w)
    g.set_graph_mode(graph)
    done = 0
    while done < steps:
        k = min(check_every, steps - done)
        g.step(k)
        o.step(k)
        done += k
        xg, tg, sg, stg = g.state()
        xo, to, so, sto = o.state()
        assert sg == so == done
        assert _per_err(xg, xo, w.L) <= tol, done
        assert xg.min() >= 0.0 and xg.max() < w.L
        tri = g.triangles()
        assert len(tri) == 2 * w.n
        assert _tris(tri) == _tris(o.triangles()), done
    for k in ("overlap_rounds_total", "overlap_rounds_max", "overlap_edges_total", "cap_hits", "noise_clamps",
              "reversals"):
        assert stg[k] == sto[k], (k, stg[k], sto[k])
    assert stg["host_rebuilds"] == 0
    return xg, stg


@pytest.mark.parametrize("graph", [False, True])
def test_periodic_delaunay_c1_matches_oracle(graph):
    w = synth.make("C1", n=1000, periodic=True)
    xg, st = _delaunay_run(w, 100, 1e-9, graph)
    assert st["overlap_rounds_total"] > 0 and st["flips_total"] > 0


def test_periodic_delaunay_c2_fp32_matches_oracle():
    w = synth.make("C2", n=4096, periodic=True)
    xg, st = _delaunay_run(w, 40, 1e-4, True)
    assert st["overlap_rounds_total"] > 0
    assert np.any(np.abs(xg - w.xy) > 0.5 * w.L)   # self-propelled disks went through the boundary


def test_periodic_delaunay_short_range_matches_oracle():
    w = synth.make("C3", n=3000, periodic=True)
    w.fp32_forces = False
    _delaunay_run(w, 30, 1e-9, True)


def test_periodic_forces_all_pairs_match_oracle():
    for fp32 in (False, True):
        w = synth.make("C2", n=3001, periodic=True)
        g = binding.Sim.from_workload(w, fp32=fp32)
        fo = oracle.forces(w.xy, w.species, w.K, period=w.L)
        assert np.abs(g.forces() - fo).max() <= (1e-4 if fp32 else 1e-12) * np.abs(fo).max()


def test_periodic_delaunay_full_size_c2_properties():
    w = synth.make("C2", periodic=True)
    g = binding.Sim.from_workload(w)
    g.set_graph_mode(True)
    g.step(3)
    xg, _, step, st = g.state()
    assert step == 3 and st["host_rebuilds"] == 0
    assert xg.min() >= 0.0 and xg.max() < w.L
    tree = cKDTree(xg, boxsize=w.L)
    assert len(tree.query_pairs(2.0 * (1.0 - 1e-9))) == 0
    tri = g.triangles()
    assert len(tri) == 2 * w.n
    # every triangle counter-clockwise at its nearest images and its circumcircle empty of other disks
    a = xg[tri[:, 0]]
    b = a + _mi(xg[tri[:, 1]] - a, w.L)
    c = a + _mi(xg[tri[:, 2]] - a, w.L)
    o = (b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0])
    assert np.all(o > 0)
    bx, by, cx, cy = b[:, 0] - a[:, 0], b[:, 1] - a[:, 1], c[:, 0] - a[:, 0], c[:, 1] - a[:, 1]
    d = 2.0 * (bx * cy - by * cx)
    ux = (cy * (bx * bx + by * by) - by * (cx * cx + cy * cy)) / d
    uy = (bx * (cx * cx + cy * cy) - cx * (bx * bx + by * by)) / d
    r = np.sqrt(ux * ux + uy * uy)
    centre = np.mod(a + np.stack([ux, uy], axis=1), w.L)
    inside = tree.query_ball_point(centre, r * (1.0 - 1e-9))
    for t, hits in enumerate(inside):
        assert set(hits) <= set(tri[t].tolist()), t
    idx = np.random.default_rng(3).choice(w.n, 200, replace=False).astype(np.int32)
    fo = oracle.forces(xg, w.species, w.K, period=w.L, idx=idx)
    assert np.abs(g.forces()[idx] - fo).max() <= 1e-4 * np.abs(fo).max()


def _mi(v, L):
    return v - L * np.rint(v / L)
