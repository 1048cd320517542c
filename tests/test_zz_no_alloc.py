"""bd_pair_forces_dev_noalloc (no device allocation; fixed per-GPU scratch
array) against bd_pair_forces_dev on the same inputs: bitwise equal forces,
within the oracle's tolerance, on two calls in a row with the second on a
smaller input (the scratch keeps the first call's contents), FP64 and FP32,
then the size limit."""
import numpy as np
import pytest

import oracle
from paper_1703_02484_amd import binding, synth
from tests.conftest import gpu_available

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _dev(w):
    import torch

    xy = torch.from_numpy(np.ascontiguousarray(w.xy)).cuda()
    sp = torch.from_numpy(np.ascontiguousarray(w.species, dtype=np.int32)).cuda()
    return xy, sp


@pytest.mark.parametrize("fp32", [False, True])
def test_noalloc_matches_allocating_call_twice(fp32):
    import torch

    print("noalloc vs allocating call, fp32 =", fp32, flush=True)
    for n in (70001, 3001):   # second call smaller than the first
        w = synth.make("C2", n=n)
        xy, sp = _dev(w)
        ref = binding.pair_forces_dev(xy, sp, w.K, fp32=fp32)
        got = binding.pair_forces_dev(xy, sp, w.K, fp32=fp32, noalloc=True)
        torch.cuda.synchronize()
        a, b = ref.cpu().numpy(), got.cpu().numpy()
        assert np.array_equal(a, b), (n, np.abs(a - b).max())
        idx = np.arange(0, n, max(1, n // 400), dtype=np.int32)
        fo = oracle.forces(w.xy, w.species, w.K, idx=idx)
        assert np.abs(b[idx] - fo).max() <= (1e-4 if fp32 else 1e-12) * np.abs(fo).max()


def test_noalloc_rejects_sizes_beyond_its_scratch():
    import torch

    n = 2_097_153   # one split of FP64 sums needs 16 n bytes > 32 MiB
    xy = torch.zeros((n, 2), dtype=torch.float64, device="cuda")
    sp = torch.zeros(n, dtype=torch.int32, device="cuda")
    with pytest.raises(binding.BDError) as e:
        binding.pair_forces_dev(xy, sp, np.array([[1.0]]), noalloc=True)
    assert e.value.code == -1
