"""Launch shapes and the autotuner on the GPU.

Tiles per pass, waves per block and the grid change only which wave computes which work
item, not the arithmetic of an item: local energies must be bitwise equal across them
(groups per item change the per-item summation order, so those are held to rounding).
The autotuner's JSON cache must be written, and a second tuning of the same problem must
reuse it without timing and still give local energies that match the oracle."""
import json

import numpy as np
import pytest
import torch

from oracle import energy as oen
from paper_2506_07430_amd import autotune, elocal, synth
from tests.gpu_common import ansatz_samples, make_ham, theta_for, words_to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    torch.cuda.set_device(0)


@pytest.mark.parametrize("n,na,nb,widths", [(12, 6, 5, (64, 32)), (33, 8, 9, (32, 32)), (24, 12, 12, (128, 128)),
                                             (40, 14, 14, (256, 256, 256))])
def test_launch_shapes_give_bitwise_equal_local_energies(n, na, nb, widths):
    p = synth.random_problem(n, na, nb, widths, seed=500 + n, n_chol=4, decay=5.0, samples=40)
    ham = make_ham(p)
    th_dev, th = theta_for(p.theta, elocal.BF16)
    ans = elocal.Ansatz(widths, th_dev, elocal.BF16)
    x = words_to_dev(p.x)
    ham.tune()
    ref, _ = ham.eval(ans, x, want_logpsi=False)
    base = ham.launch_info(ans, x.shape[0])
    ran = []
    for cols in (1, 2):
        for waves in (0, base["max_waves"] // 2, 1):
            for grid in (0, 7):
                ham.tune(grid=grid, waves=waves, cols=cols)
                info = ham.launch_info(ans, x.shape[0])
                got, _ = ham.eval(ans, x, want_logpsi=False)
                torch.cuda.synchronize()
                ran.append((info["cols"], info["waves"], info["grid"]))
                assert torch.equal(got, ref), (cols, waves, grid, info)
    ham.tune()
    print(f"n={n} {widths}: {len(set(ran))} distinct launch shapes, all bitwise equal", flush=True)
    if max(widths) <= 128:
        assert any(r[0] == 2 for r in ran)         # the two-tile variant exists and ran
    e = ref.cpu().numpy()
    assert np.max(np.abs(e[:, 0] + 1j * e[:, 1] - oen.local_energies(p.h1e, p.eri, n, na, nb, widths, th, p.x))) <= 1e-5


def test_autotuner_cache_is_written_and_reused(tmp_path, monkeypatch):
    cache = tmp_path / "tune.json"
    monkeypatch.setenv(autotune.CACHE_ENV, str(cache))
    p = synth.make_problem(0)
    s = p.system
    x_np = ansatz_samples(p, 512, seed=3)
    th_dev, th = theta_for(p.theta, elocal.BF16)
    ans = elocal.Ansatz(s.widths, th_dev, elocal.BF16)
    x = words_to_dev(x_np)
    ham = make_ham(p)
    table = autotune.tune_eval(ham, ans, x, reps=1, budget_s=5.0)
    assert len(table) > 1 and not any(r.get("cached") for r in table)
    data = json.loads(cache.read_text())
    key = autotune.problem_key(ham, ans, x.shape[0])
    assert key in data
    best = data[key]
    # a new handle for the same problem: the cached shape is applied, nothing is timed
    ham2 = make_ham(p)
    rows = autotune.tune_eval(ham2, ans, x)
    assert len(rows) == 1 and rows[0]["cached"]
    info = ham2.launch_info(ans, x.shape[0])
    assert {k: info[k] for k in ("grid", "groups", "waves", "cols")} == best["ran"]
    el, _ = ham2.eval(ans, x, want_logpsi=False)
    e = el.cpu().numpy()
    ref = oen.local_energies(p.h1e, p.eri, s.n, s.n_alpha, s.n_beta, s.widths, th, x_np)
    assert np.max(np.abs(e[:, 0] + 1j * e[:, 1] - ref)) <= 1e-5


def test_multi_autotuner_cache(tmp_path, monkeypatch):
    cache = tmp_path / "tune.json"
    monkeypatch.setenv(autotune.CACHE_ENV, str(cache))
    probs = [synth.random_problem(12, 6, 6, (64, 64), seed=31, n_chol=4, decay=5.0, samples=30),
             synth.random_problem(20, 10, 10, (128, 128), seed=32, n_chol=4, decay=5.0, samples=20)]
    hams = [make_ham(q) for q in probs]
    ans = [elocal.Ansatz(q.system.widths, theta_for(q.theta, elocal.BF16)[0], elocal.BF16) for q in probs]
    xs = [words_to_dev(q.x) for q in probs]
    mev = elocal.MultiEval()
    table = autotune.tune_multi(mev, hams, ans, xs, budget_s=5.0)
    assert len(table) > 1
    key = [k for k in json.loads(cache.read_text()) if k.startswith("multi[")]
    assert len(key) == 1
    hams2 = [make_ham(q) for q in probs]
    rows = autotune.tune_multi(mev, hams2, ans, xs)
    assert len(rows) == 1 and rows[0]["cached"]
    outs, _ = mev(hams2, ans, xs)
    for q, o in zip(probs, outs):
        s = q.system
        e = o.cpu().numpy()
        ref = oen.local_energies(q.h1e, q.eri, s.n, s.n_alpha, s.n_beta, s.widths, theta_for(q.theta, elocal.BF16)[1],
                                 q.x)
        assert np.max(np.abs(e[:, 0] + 1j * e[:, 1] - ref)) <= 1e-5
