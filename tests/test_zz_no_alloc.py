"""elocal_eval_noalloc (the allocation-free variant of elocal_eval, scratch in a fixed
per-GPU device array) against elocal_eval: bitwise equal local energies and log psi on two
calls in a row, the second with a smaller batch (the scratch keeps the first call's
contents), and a clear error past the scratch size."""
import numpy as np
import pytest
import torch

from paper_2506_07430_amd import elocal, synth
from tests.gpu_common import make_ham, theta_for, words_to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    torch.cuda.set_device(0)


@pytest.mark.parametrize("cfg,precision", [(0, elocal.BF16), (0, elocal.FP64), (1, elocal.BF16)])
def test_noalloc_equals_eval_on_two_calls(cfg, precision):
    p = synth.make_problem(cfg, samples=None if cfg == 0 else 2048)
    s = p.system
    ham = make_ham(p)
    th_dev, _ = theta_for(p.theta, precision)
    ans = elocal.Ansatz(s.widths, th_dev, precision)
    for rows in (p.x.shape[0], p.x.shape[0] // 3 + 1):
        x = words_to_dev(p.x[:rows])
        print(f"workload {cfg} precision {precision}: {rows} samples", flush=True)
        want, want_lp = ham.eval(ans, x)
        got_lp = torch.empty_like(want_lp)
        got, _ = ham.eval_noalloc(ans, x, logpsi=got_lp)
        torch.cuda.synchronize()
        assert torch.equal(got, want)
        assert torch.equal(got_lp, want_lp)


def test_noalloc_rejects_batches_beyond_its_scratch():
    p = synth.make_problem(1, samples=64)
    s = p.system
    ham = make_ham(p)
    th_dev, _ = theta_for(p.theta, elocal.BF16)
    ans = elocal.Ansatz(s.widths, th_dev, elocal.BF16)
    limit = elocal.NOALLOC_SCRATCH_MIB << 20
    # the smallest batch of this system whose workspace exceeds the scratch (no data needed:
    # the size check comes before any device work)
    B = 1
    while ham.workspace_bytes(elocal.OP_EVAL, B, ans) <= limit:
        B *= 2
    x = torch.zeros((B, ham.W), dtype=torch.int64, device="cuda")
    with pytest.raises(elocal.ElocalError) as e:
        ham.eval_noalloc(ans, x)
    assert e.value.status == 3
