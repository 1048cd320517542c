"""Batched systems (``bd_batch_init``): parity with one handle per system and with the oracle.

A batch advances R independent systems; each must follow exactly the
trajectory a handle of its own would (same noise keys, same Delaunay
triangulation), so batched and single-handle positions are compared
bit for bit when both cut the all-pairs sums the same way (fixed
``force_chunk``), and against the FP64 oracle within 1e-9 relative.
"""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
from paper_1703_02484_amd import binding, synth
from tests._checks import check_delaunay, count_overlaps, rel_err, tri_set
from tests.conftest import gpu_available

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _split(xy, off):
    return [xy[off[r]:off[r + 1]] for r in range(len(off) - 1)]


def _local_tris(tris, r, doff, foff, n):
    """Triangles of system r in its own numbering (disks 0..n_r-1, then its frame points)."""
    d0, d1 = doff[r], doff[r + 1]
    f0, f1 = n + foff[r], n + foff[r + 1]
    nr = d1 - d0
    out = []
    for t in tris:
        if all(d0 <= v < d1 or f0 <= v < f1 for v in t):
            out.append([v - d0 if v < d1 else nr + (v - f0) for v in t])
        else:
            assert all(not (d0 <= v < d1 or f0 <= v < f1) for v in t), "triangle mixes systems"
    return np.array(out, dtype=np.int64)


def test_batch_layout_and_frames():
    ws = synth.make_batch(4, lo=60, hi=400)
    b = binding.Sim.from_workloads(ws)
    R, doff, foff = b.layout()
    assert R == 4
    assert list(np.diff(doff)) == [w.n for w in ws]
    fr = b.frame()
    for r, w in enumerate(ws):
        assert np.array_equal(fr[foff[r]:foff[r + 1]], oracle.frame(w.L, 1.0))
    tris = b.triangles()
    for r, w in enumerate(ws):
        lt = _local_tris(tris, r, doff, foff, b.n)
        assert tri_set(lt) == tri_set(oracle.delaunay_with_frame(w.xy, w.L, 1.0))


@pytest.mark.parametrize("fp32", [False, True])
def test_batch_equals_single_handles_bitwise(fp32):
    ws = synth.make_batch(5, seed=1, lo=100, hi=1500)
    b = binding.Sim.from_workloads(ws, force_chunk=128, fp32=fp32)
    singles = [binding.Sim.from_workload(w, force_chunk=128, fp32=fp32) for w in ws]
    _, doff, foff = b.layout()
    fb = b.forces()
    for r, s in enumerate(singles):
        assert np.array_equal(fb[doff[r]:doff[r + 1]], s.forces())
    for _ in range(3):
        b.step(10)
        for s in singles:
            s.step(10)
        xb, thb, stepb, _ = b.state()
        tris = b.triangles()
        for r, s in enumerate(singles):
            xs, ths, steps, _ = s.state()
            assert np.array_equal(xb[doff[r]:doff[r + 1]], xs), r
            assert np.array_equal(thb[doff[r]:doff[r + 1]], ths), r
            assert stepb == steps
            assert tri_set(_local_tris(tris, r, doff, foff, b.n)) == tri_set(s.triangles())
    sb = b.state()[3]
    tot = {k: sum(s.state()[3][k] for s in singles) for k in ("overlap_edges_total", "reversals", "noise_clamps")}
    for k, v in tot.items():
        assert sb[k] == v, k


def test_batch_matches_oracle_fp64():
    ws = synth.make_batch(4, seed=2, lo=150, hi=1200)
    b = binding.Sim.from_workloads(ws)
    orcs = [oracle.OracleSim.from_workload(w) for w in ws]
    _, doff, foff = b.layout()
    for step in range(30):
        b.step(1)
        for o in orcs:
            o.step(1)
        if (step + 1) % 10 == 0:
            xb, thb, stb, _ = b.state()
            tris = b.triangles()
            for r, o in enumerate(orcs):
                xo, tho, so, _ = o.state()
                assert rel_err(xb[doff[r]:doff[r + 1]], xo) <= 1e-9, (step, r)
                assert stb == so
                assert tri_set(_local_tris(tris, r, doff, foff, b.n)) == tri_set(o.triangles()), (step, r)


def test_batch_dense_and_dilute_mix():
    # systems at both ends of the area-fraction range, strong noise: overlap rounds
    # in some systems while others are already clean must not disturb them
    xs, Ls = [], []
    for r, (n, phi) in enumerate([(300, 0.5), (200, 0.05), (450, 0.45)]):
        L = synth.box_side(n, phi)
        xs.append(synth.rsa(n, L, 1.0, seed=40 + r))
        Ls.append(L)
    K = np.array([[0.0]])
    kw = dict(dt=1e-2, force_chunk=64)
    b = binding.Sim.batch(xs, [np.ones(len(x)) for x in xs], [np.zeros(len(x), np.int32) for x in xs], None, Ls,
                          [7, 8, 9], K, **kw)
    singles = [binding.Sim(x, np.ones(len(x)), np.zeros(len(x), np.int32), None, K, L=L, seed=sd, **kw)
               for x, L, sd in zip(xs, Ls, [7, 8, 9])]
    _, doff, _ = b.layout()
    b.step(8)
    for s in singles:
        s.step(8)
    xb = b.state()[0]
    for r, s in enumerate(singles):
        assert np.array_equal(xb[doff[r]:doff[r + 1]], s.state()[0]), r
    assert b.state()[3]["overlap_rounds_max"] >= 2


def test_batch_full_size_c4():
    # 256 systems, N_r log-uniform in [2048, 32768]: sampled forces against the
    # oracle, then two steps and the properties of every system
    ws = synth.make_batch(256)
    b = binding.Sim.from_workloads(ws)
    cfg = b.force_config()
    assert cfg["tuned"] in (1, 2) and cfg["tiles"] > 0
    _, doff, foff = b.layout()
    fb = b.forces()
    rng = np.random.default_rng(5)
    for r in rng.choice(len(ws), 6, replace=False):
        w = ws[r]
        idx = np.sort(rng.choice(w.n, 64, replace=False))
        fo = oracle.forces(w.xy, w.species, w.K, idx=idx)
        assert np.abs(fb[doff[r] + idx] - fo).max() <= 1e-12 * np.abs(fo).max(), r
    b.step(2)
    x, _, step, st = b.state()
    assert step == 2 and st["host_rebuilds"] == 0
    tris = b.triangles()
    fr = b.frame()
    for r in rng.choice(len(ws), 4, replace=False):
        w = ws[r]
        xr = x[doff[r]:doff[r + 1]]
        assert np.all(xr >= 1.0) and np.all(xr <= w.L - 1.0)
        assert count_overlaps(xr) == 0
        check_delaunay(np.concatenate([xr, fr[foff[r]:foff[r + 1]]]), _local_tris(tris, r, doff, foff, b.n))


_TUNE_CHILD = r"""
import json, sys
sys.path.insert(0, {root!r})
from paper_1703_02484_amd import binding, synth
w = synth.make("C2", n=12000)
s = binding.Sim.from_workload(w)
print(json.dumps(s.force_config()))
"""


def test_tuning_cache_file(tmp_path):
    # the first process times the candidate tilings and writes the cache; the
    # second takes the same tiling from the file without timing
    cache = tmp_path / "tune.json"
    env = dict(os.environ, BD_TUNE_CACHE=str(cache))
    code = _TUNE_CHILD.format(root=ROOT)
    outs = []
    for _ in range(2):
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
        assert r.returncode == 0, r.stderr
        outs.append(json.loads(r.stdout.strip().splitlines()[-1]))
    assert outs[0]["tuned"] == 1 and outs[1]["tuned"] == 2
    for k in ("chunk", "per_lane", "persistent"):
        assert outs[0][k] == outs[1][k]
    assert cache.exists() and len(json.loads(cache.read_text())) == 1


def test_same_shape_handles_share_tiling():
    w = synth.make("C2", n=12000)
    a = binding.Sim.from_workload(w)
    b = binding.Sim.from_workload(w)
    ca, cb = a.force_config(), b.force_config()
    assert ca["tuned"] in (1, 2) and cb["tuned"] == 2
    assert (ca["chunk"], ca["per_lane"], ca["persistent"]) == (cb["chunk"], cb["per_lane"], cb["persistent"])
    a.step(5)
    b.step(5)
    assert np.array_equal(a.state()[0], b.state()[0])


def test_batch_of_one_equals_plain_handle():
    w = synth.make("C1", n=700)
    a = binding.Sim.from_workload(w)
    b = binding.Sim.from_workloads([w])
    a.step(12)
    b.step(12)
    assert np.array_equal(a.state()[0], b.state()[0])
    assert tri_set(a.triangles()) == tri_set(b.triangles())
    assert a.force_config() == b.force_config()


def test_batch_of_tiny_systems():
    # three disks per system (the smallest allowed), boxes of different sides
    xs, Ls = [], []
    for r in range(6):
        L = 8.0 + r
        xs.append(synth.rsa(3, L, 1.0, seed=100 + r))
        Ls.append(L)
    K = np.array([[1e-2]])
    kw = dict(dt=1e-3)
    b = binding.Sim.batch(xs, [np.ones(3)] * 6, [np.zeros(3, np.int32)] * 6, None, Ls, list(range(6)), K, **kw)
    b.step(20)
    xb = b.state()[0]
    _, doff, _ = b.layout()
    for r in range(6):
        o = oracle.OracleSim(xs[r], np.ones(3), np.zeros(3, np.int32), None, K, L=Ls[r], seed=r, **kw)
        o.step(20)
        assert rel_err(xb[doff[r]:doff[r + 1]], o.state()[0]) <= 1e-9, r
