"""The stateless pair-force call bd_pair_forces_dev (device arrays in, device
forces out, no handle) against the oracle's brute-force forces, element by
element: every law, FP64 and FP32, non-reciprocal two-species K, ragged sizes
that span several workgroups and j splits with a short last one, the
single-particle and two-particle edge cases, and the full 65,536-disk
two-species workload on sampled rows."""
import numpy as np
import pytest

import oracle
from paper_1703_02484_amd import binding, synth
from tests.conftest import gpu_available

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

LAWS = {
    "q2": dict(kind="power", q=2.0),
    "q6": dict(kind="power", q=6.0),
    "screened_cut": dict(kind="screened", A=1.0, lam=0.5, cutoff=2.5),
    "q2_cut": dict(kind="power", q=2.0, cutoff=6.0),
}


def _dev(w):
    import torch

    xy = torch.from_numpy(np.ascontiguousarray(w.xy)).cuda()
    sp = torch.from_numpy(np.ascontiguousarray(w.species, dtype=np.int32)).cuda()
    return xy, sp


@pytest.mark.parametrize("law", sorted(LAWS))
@pytest.mark.parametrize("fp32", [False, True])
@pytest.mark.parametrize("n", [1, 2, 513, 3001])
def test_pair_forces_dev_matches_oracle(law, fp32, n):
    import torch

    w = synth.make("C2", n=max(n, 3))
    if n < 3:   # the workload generator's smallest system; keep its first n disks
        w.xy, w.species = w.xy[:n].copy(), w.species[:n].copy()
    kw = LAWS[law]
    xy, sp = _dev(w)
    f = binding.pair_forces_dev(xy, sp, w.K, fp32=fp32, **kw)
    torch.cuda.synchronize()
    fo = oracle.forces(w.xy, w.species, w.K, **kw)
    got = f.cpu().numpy()
    scale = max(np.abs(fo).max(), 1e-300)
    tol = 1e-4 if fp32 else 1e-12
    assert np.abs(got - fo).max() <= tol * scale
    if n == 1:
        assert np.all(got == 0.0)


def test_pair_forces_dev_full_size_sampled():
    import torch

    w = synth.make("C2")
    xy, sp = _dev(w)
    f = binding.pair_forces_dev(xy, sp, w.K, fp32=True).cpu().numpy()
    torch.cuda.synchronize()
    rng = np.random.default_rng(5)
    idx = np.concatenate([[0, w.n - 1], rng.choice(w.n, 510, replace=False)]).astype(np.int32)
    fo = oracle.forces(w.xy, w.species, w.K, idx=idx)
    assert np.abs(f[idx] - fo).max() <= 1e-4 * np.abs(fo).max()


def test_pair_forces_dev_rejects_bad_arguments():
    import torch

    w = synth.make("C1", n=100)
    xy, sp = _dev(w)
    with pytest.raises(ValueError):
        binding.pair_forces_dev(xy.float(), sp, w.K)
    with pytest.raises(binding.BDError):
        binding.pair_forces_dev(xy, sp, np.zeros((9, 9)))   # S above BD_MAX_SPECIES
    with pytest.raises(binding.BDError):
        binding.pair_forces_dev(xy, sp, w.K, kind="screened", lam=-1.0)
