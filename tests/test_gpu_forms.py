"""Every form of the all-pairs force kernel that the autotuner can choose,
pinned through bd_params (chunk length, particles per lane, launch form) and
checked element by element against the oracle's brute-force forces, for the
inverse-square fast path and the general laws, in FP32 and FP64, at ragged
sizes (several tiles and a short last tile).  Then the benchmark's own
configuration at full size: N = 65,536, tuned force, graph replay, default
overlap-round launches, three steps against the oracle."""
import numpy as np
import pytest

import oracle
from paper_1703_02484_amd import binding, synth
from tests._checks import rel_err, tri_set
from tests.conftest import gpu_available

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

LAWS = {
    "q2": dict(kind="power", q=2.0),
    "q6": dict(kind="power", q=6.0),
    "screened": dict(kind="screened", A=1.0, lam=0.5),
}


def _scale(f):
    return np.abs(f).max()


@pytest.mark.parametrize("law", sorted(LAWS))
@pytest.mark.parametrize("fp32", [False, True])
@pytest.mark.parametrize("per_lane", [2, 4])
@pytest.mark.parametrize("launch", [0, 1])
@pytest.mark.parametrize("n", [1000, 4099])
def test_pinned_force_form_matches_oracle(law, fp32, per_lane, launch, n):
    w = synth.make("C2", n=n)
    kw = dict(LAWS[law])
    g = binding.Sim.from_workload(w, fp32=fp32, force_chunk=512, force_per_lane=per_lane, force_launch=launch, **kw)
    cfg = g.force_config()
    assert (cfg["chunk"], cfg["per_lane"], cfg["persistent"], cfg["tuned"]) == (512, per_lane, launch, 0)
    fo = oracle.forces(w.xy, w.species, w.K, **kw)
    tol = 1e-4 if fp32 else 1e-12
    assert np.abs(g.forces() - fo).max() <= tol * _scale(fo)


@pytest.mark.parametrize("fp32", [False, True])
@pytest.mark.parametrize("per_lane", [2, 4])
@pytest.mark.parametrize("n", [1000, 4099])
def test_lds_staged_form_matches_oracle_and_scalar_form(fp32, per_lane, n):
    # j staged through LDS (the shared-memory broadcast of the paper's n-body kernel): same tiles and
    # summation order as the scalar-load form, so the forces are bitwise equal to it
    w = synth.make("C2", n=n)
    g = binding.Sim.from_workload(w, fp32=fp32, force_chunk=512, force_per_lane=per_lane, force_launch=2)
    assert g.force_config()["persistent"] == 3
    h = binding.Sim.from_workload(w, fp32=fp32, force_chunk=512, force_per_lane=per_lane, force_launch=0)
    fo = oracle.forces(w.xy, w.species, w.K)
    fg = g.forces()
    assert np.abs(fg - fo).max() <= (1e-4 if fp32 else 1e-12) * _scale(fo)
    assert np.array_equal(fg, h.forces())
    g.step(3)
    h.step(3)
    assert np.array_equal(g.state()[0], h.state()[0])


def test_pinned_force_form_rejects_bad_values():
    w = synth.make("C1", n=100)
    with pytest.raises(binding.BDError):
        binding.Sim.from_workload(w, force_chunk=512, force_per_lane=3)
    with pytest.raises(binding.BDError):
        binding.Sim.from_workload(w, force_chunk=512, force_launch=3)
    with pytest.raises(binding.BDError):   # the LDS form is written for the inverse-square law only
        binding.Sim.from_workload(w, force_chunk=512, force_launch=2, kind="power", q=6.0)


def test_full_size_c2_bench_path_matches_oracle():
    # exactly what bench.py times: the tuned force (the symmetric form on MI355X), graph replay,
    # the large overlap and flip rounds launched per phase and the rest in one workgroup (the library's choice
    # above 16,384 disks)
    w = synth.make("C2")
    g = binding.Sim.from_workload(w)
    cfg = g.force_config()
    print("force configuration", cfg, flush=True)
    assert cfg["tuned"] in (1, 2) and cfg["persistent"] == 2
    g.set_graph_mode(True)
    o = oracle.OracleSim.from_workload(w)
    g.step(3)
    o.step(3)
    xg, tg, sg, stg = g.state()
    xo, to, so, sto = o.state()
    assert sg == so == 3
    assert rel_err(xg, xo) <= 1e-4
    assert np.abs(tg - to).max() <= 1e-12
    assert tri_set(g.triangles()) == tri_set(o.triangles())
    for k in ("overlap_rounds_total", "overlap_rounds_max", "overlap_edges_total", "reversals", "noise_clamps",
              "cap_hits"):
        assert stg[k] == sto[k], (k, stg[k], sto[k])
    assert stg["host_rebuilds"] == 0 and stg["overlap_rounds_total"] > 0
