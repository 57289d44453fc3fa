"""The measurement helper: the atomic-rate microbenchmark adds exactly 1.0 per pass to
every element (small integers are exact in FP32), so its launch does the work its
rate is computed from."""
import pytest
import torch

pytestmark = pytest.mark.gpu

pm = pytest.importorskip("paper_2404_02783_amd")


def test_microbench_atomics_adds_one_per_pass():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    buf = torch.zeros((1 << 20) + 37, dtype=torch.float32, device="cuda")
    pm.pm_microbench_atomics(buf, passes=3)
    torch.cuda.synchronize()
    assert bool((buf == 3.0).all())


def test_microbench_atomics_rejects_bad_arguments():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    with pytest.raises(pm.PMError):
        pm.pm_microbench_atomics(torch.zeros(16, dtype=torch.float64, device="cuda"))
    with pytest.raises(pm.PMError):
        pm.pm_microbench_atomics(torch.zeros(16, dtype=torch.float32, device="cuda"), passes=0)
