"""Full-size workloads on the GPU, in the launch configuration of the benchmark.

The whole batch of each workload is evaluated in one call; sampled outputs are
compared with oracle values stored in tests/golden/full_size_eloc.json (written by
tests/golden/make_full_size_eloc.py from the oracle alone; the stored determinant
words confirm the inputs were regenerated identically). Properties that hold at any
size are checked too: a sample's local energy does not depend on the rest of the
batch (the first rows of the full call equal a call on those rows alone, bitwise).
Bars: FP64 mode within 1e-8 relative. Both BF16 modes within 1e-5 Ha of the oracle run
on the same BF16-rounded parameters, at every size (with hidden activations carried as
two fp16 terms, 2^-22 relative, the rounding summed over the 1.15 million connected
determinants of the 60-orbital workload stays a few 1e-6 Ha).
"""
import json
import os

import numpy as np
import pytest
import torch

from paper_2506_07430_amd import elocal, synth
from tests.gpu_common import make_ham, theta_for, words_to_dev

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "full_size_eloc.json")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    torch.cuda.set_device(0)


def _gold(cfg, precision, system=0):
    with open(GOLD) as f:
        entries = json.load(f)["entries"]
    tag = "fp64" if precision == elocal.FP64 else "bf16"   # both BF16 modes use bf16 parameters
    return [e for e in entries if e["workload"] == cfg and e["system"] == system and e["precision"] == tag]


def _c(e):
    e = e.cpu().numpy()
    return e[:, 0] + 1j * e[:, 1]


def _check_gold(p, eloc, gold, precision, bar=1e-5):
    assert gold, "no stored oracle values"
    for g in gold:
        assert g["samples"] == p.x.shape[0]
        assert [f"{int(v):016x}" for v in p.x[g["index"]]] == g["x"], "regenerated input differs"
        ref = g["re"] + 1j * g["im"]
        got = eloc[g["index"]]
        err = abs(got - ref)
        print(f"  sample {g['index']}: |dE_loc| = {err:.3e}", flush=True)
        if precision != elocal.FP64:
            assert err <= bar
        else:
            assert err <= 1e-8 * abs(ref)


@pytest.mark.parametrize("cfg,precision,bar", [(1, elocal.BF16, 1e-5), (3, elocal.BF16, 1e-5),
                                               (4, elocal.BF16X3, 1e-5), (4, elocal.BF16, 1e-5)])
def test_full_batch_bf16(cfg, precision, bar):
    p = synth.make_problem(cfg)
    s = p.system
    print(f"workload {cfg}: n={s.n} widths={s.widths} B={p.x.shape[0]} (precision {precision}, full batch)",
          flush=True)
    ham = make_ham(p)
    th_dev, _ = theta_for(p.theta, precision)
    ans = elocal.Ansatz(s.widths, th_dev, precision)
    x = words_to_dev(p.x)
    ham.timing(True)
    eloc, _ = ham.eval(ans, x, want_logpsi=False)
    ms, _ = ham.kernel_time(reset=True)
    print(f"  fused kernel {ms:.1f} ms", flush=True)
    full = _c(eloc)
    assert np.all(np.isfinite(full))
    _check_gold(p, full, _gold(cfg, precision), precision, bar)
    head, _ = ham.eval(ans, x[:5].contiguous(), want_logpsi=False)
    torch.cuda.synchronize()
    assert torch.equal(head, eloc[:5])


@pytest.mark.parametrize("cfg", [1, 3, 4])
def test_full_size_fp64_first_sample(cfg):
    p = synth.make_problem(cfg)
    s = p.system
    print(f"workload {cfg}: n={s.n} widths={s.widths} (FP64, first sample)", flush=True)
    ham = make_ham(p)
    th_dev, _ = theta_for(p.theta, elocal.FP64)
    ans = elocal.Ansatz(s.widths, th_dev, elocal.FP64)
    eloc, _ = ham.eval(ans, words_to_dev(p.x[:1]), want_logpsi=False)
    torch.cuda.synchronize()
    _check_gold(p, _c(eloc), _gold(cfg, elocal.FP64), elocal.FP64)


def test_eight_systems_one_launch_bf16():
    """The eight-system workload at full size through elocal_eval_multi."""
    wl = synth.WORKLOADS[2]
    probs = [synth.make_problem(2, si) for si in range(len(wl.systems))]
    print("eight systems: samples " + str([p.x.shape[0] for p in probs]), flush=True)
    hams = [make_ham(p) for p in probs]
    ans = [elocal.Ansatz(p.system.widths, theta_for(p.theta, elocal.BF16)[0], elocal.BF16) for p in probs]
    xs = [words_to_dev(p.x) for p in probs]
    hams[0].timing(True)
    outs, _ = elocal.MultiEval()(hams, ans, xs)
    ms, _ = hams[0].kernel_time(reset=True)
    pairs = sum(p.x.shape[0] * h.C for p, h in zip(probs, hams))
    print(f"  one launch: {ms:.1f} ms, {pairs / (ms * 1e-3):.3e} H elements/s", flush=True)
    for si, (p, out) in enumerate(zip(probs, outs)):
        print(f" system {si} (n={p.system.n})", flush=True)
        _check_gold(p, _c(out), _gold(2, elocal.BF16, si), elocal.BF16)
    for si in (0, 5, 7):
        head, _ = hams[si].eval(ans[si], xs[si][:3].contiguous(), want_logpsi=False)
        torch.cuda.synchronize()
        assert torch.equal(head, outs[si][:3])
