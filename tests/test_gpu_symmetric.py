"""The symmetric form of the all-pairs force (``force_chunk = -1``): every
pair of chunks of a system evaluated once by one workgroup, which writes the
partial sums of both chunks (the pair's geometric factor is the same for both
orders; K weights each side in the reduction).  Checked against the oracle
like the ordinary form: forces, trajectories, a batch, the adjoint, and
run-to-run determinism.  Chunks are cut to at most 1024 disks, so the sizes
below give ragged last chunks and several chunk pairs per system."""
import numpy as np
import pytest

import oracle
from paper_1703_02484_amd import binding, synth
from tests._checks import rel_err, tri_set
from tests.conftest import gpu_available

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _scale(f):
    return np.abs(f).max()


@pytest.mark.parametrize("pin", [-1, -2, -3])
@pytest.mark.parametrize("n", [3, 65, 1000, 1025, 4099])
def test_symmetric_forces_fp32(n, pin):
    w = synth.make("C2", n=n)
    g = binding.Sim.from_workload(w, force_chunk=pin)
    cfg = g.force_config()
    assert cfg["persistent"] == 2 and cfg["per_lane"] == {-1: 4, -2: 2, -3: 8}[pin]
    fo = oracle.forces(w.xy, w.species, w.K)
    assert np.abs(g.forces() - fo).max() <= 1e-4 * _scale(fo)


@pytest.mark.parametrize("pin", [-1, -2, -3])
@pytest.mark.parametrize("n", [700, 2500])
def test_symmetric_forces_fp64(n, pin):
    w = synth.make("C1", n=n)
    g = binding.Sim.from_workload(w, force_chunk=pin)
    fo = oracle.forces(w.xy, w.species, w.K)
    assert np.abs(g.forces() - fo).max() <= 1e-12 * _scale(fo)


@pytest.mark.parametrize("pin", [-1, -3])
def test_symmetric_full_size_c2_sampled(pin):
    w = synth.make("C2")
    g = binding.Sim.from_workload(w, force_chunk=pin)
    fg = g.forces()
    idx = np.sort(np.random.default_rng(0).choice(w.n, 512, replace=False))
    fo = oracle.forces(w.xy, w.species, w.K, idx=idx)
    assert np.abs(fg[idx] - fo).max() <= 1e-4 * _scale(fo)


def test_symmetric_trajectory_c2_fp32():
    w = synth.make("C2", n=3000)
    g = binding.Sim.from_workload(w, force_chunk=-1)
    o = oracle.OracleSim.from_workload(w)
    for _ in range(5):
        g.step(10)
        o.step(10)
        assert rel_err(g.state()[0], o.state()[0]) <= 1e-4
        assert tri_set(g.triangles()) == tri_set(o.triangles())


def test_symmetric_batch_fp64_matches_oracle():
    ws = synth.make_batch(5, seed=4, lo=300, hi=2600)
    b = binding.Sim.from_workloads(ws, force_chunk=-1)
    _, doff, _ = b.layout()
    f = b.forces()
    for r, w in enumerate(ws):
        fo = oracle.forces(w.xy, w.species, w.K)
        assert np.abs(f[doff[r]:doff[r + 1]] - fo).max() <= 1e-12 * _scale(fo)


def test_symmetric_bitwise_run_to_run():
    w = synth.make("C2", n=5000)
    a = binding.Sim.from_workload(w, force_chunk=-1)
    b = binding.Sim.from_workload(w, force_chunk=-1)
    a.step(8)
    b.step(8)
    assert np.array_equal(a.state()[0], b.state()[0])


@pytest.mark.parametrize("pin", [-1, -2, -3])
def test_symmetric_adjoint_matches_oracle_jvp(pin):
    w = synth.make("C5", n=1500)
    steps = 8
    g = binding.Sim.from_workload(w, force_chunk=pin)
    g.adjoint_begin(steps, 3)
    o = oracle.OracleSim.from_workload(w)
    rng = np.random.default_rng(2)
    v = rng.normal(size=(w.n, 2))
    tK = rng.normal(size=w.K.shape)
    o.set_tangent(v, tK)
    o.step(steps)
    assert np.abs(g.state()[0] - o.state()[0]).max() <= 1e-9 * w.L
    lam = rng.normal(size=(w.n, 2))
    g0, gK = g.adjoint_backward(lam)
    lhs = np.sum(g0 * v) + np.sum(gK * tK)
    rhs = np.sum(lam * o.tangent())
    assert abs(lhs - rhs) <= 1e-10 * abs(rhs)


def test_symmetric_form_needs_the_inverse_square_law():
    w = synth.make("C1", n=300)
    with pytest.raises(binding.BDError):
        binding.Sim.from_workload(w, force_chunk=-1, kind="power", q=6.0)
