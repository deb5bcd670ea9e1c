"""Batch autoregressive sampling on the GPU (elocal_sample) against the BAS oracle.

Both sides split every prefix's weight by the same chain of binomials (inversion or BTRD)
from the same Philox4x32-10 stream on FP64 conditionals, so the distinct samples, their
order and their counts must be equal (bit-exact) at moderate N_s. At N_s = 10^12 an ulp of
difference between the two sides' FP64 conditionals can move a binomial variate by one
(its mean n p is then known to 1e-4 only), so there the leaves must be the same and the
counts agree to 1e-6 relative; the counts follow |psi|^2 (chi-square over the full sector)
and the call takes about as long as at N_s = 10^5 (its cost follows the distinct prefixes).
"""
import time

import numpy as np
import pytest
import torch

from oracle import made as omade
from oracle import sampler as osamp
from oracle import slater_condon as osc
from paper_2506_07430_amd import elocal, synth
from tests.gpu_common import make_ham, theta_for, words_from_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    torch.cuda.set_device(0)


@pytest.mark.parametrize("cfg,Ns,seed", [(0, 100000, 11), (0, 777, 0x1234567890AB), (1, 3000, 5)])
def test_sampler_equals_oracle(cfg, Ns, seed):
    p = synth.make_problem(cfg, samples=4)
    s = p.system
    ham = make_ham(p)
    th_dev, th = theta_for(p.theta, elocal.FP64)
    ans = elocal.Ansatz(s.widths, th_dev, elocal.FP64)
    x, c = ham.sample(ans, Ns, seed, max_unique=200000)
    torch.cuda.synchronize()
    occ, cnt = osamp.bas(th, s.n, s.n_alpha, s.n_beta, s.widths, Ns, seed)
    print(f"workload {cfg}: {Ns} draws -> {x.shape[0]} distinct (oracle {occ.shape[0]})")
    assert np.array_equal(words_from_dev(x), osc.pack(occ))
    assert np.array_equal(c.cpu().numpy(), cnt)


def test_sampler_at_1e12_draws():
    from scipy.stats import chi2
    p = synth.make_problem(0)
    s = p.system
    ham = make_ham(p)
    th_dev, th = theta_for(p.theta, elocal.FP64)
    ans = elocal.Ansatz(s.widths, th_dev, elocal.FP64)
    ham.sample(ans, 1000, 1)
    times = {}
    for Ns in (10 ** 5, 10 ** 12):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, c = ham.sample(ans, Ns, 17)
        times[Ns] = time.perf_counter() - t0
    print(f"N_s = 1e5: {times[10 ** 5] * 1e3:.2f} ms, N_s = 1e12: {times[10 ** 12] * 1e3:.2f} ms, "
          f"{x.shape[0]} distinct", flush=True)
    assert int(c.sum().item()) == 10 ** 12
    occ, cnt = osamp.bas(th, s.n, s.n_alpha, s.n_beta, s.widths, 10 ** 12, 17)
    assert np.array_equal(words_from_dev(x), osc.pack(occ))
    cg = c.cpu().numpy()
    assert np.max(np.abs(cg - cnt) / cnt) < 1e-6
    sector = synth.full_sector(s)
    A = omade.forward(th, osc.unpack(sector, s.n), s.n, s.n_alpha, s.n_beta, s.widths)["A"]
    exp = 1e12 * np.exp(2 * A)
    obs = np.zeros(sector.shape[0])
    obs[np.searchsorted(sector[:, 0], words_from_dev(x)[:, 0])] = cg
    stat = np.sum((obs - exp) ** 2 / exp)
    assert chi2.sf(stat, sector.shape[0] - 1) > 1e-6, stat
    assert times[10 ** 12] < 5 * times[10 ** 5] + 0.05


def test_sampler_frequencies_at_scale():
    from scipy.stats import chi2
    p = synth.make_problem(0)
    s = p.system
    ham = make_ham(p)
    th_dev, th = theta_for(p.theta, elocal.FP64)
    ans = elocal.Ansatz(s.widths, th_dev, elocal.FP64)
    Ns = 10_000_000
    ham.sample(ans, 1000, 1)
    t0 = time.perf_counter()
    x, c = ham.sample(ans, Ns, 3)
    dt = time.perf_counter() - t0
    print(f"{Ns} draws -> {x.shape[0]} distinct in {dt * 1e3:.1f} ms ({Ns / dt:.3e} draws/s)")
    assert int(c.sum().item()) == Ns
    sector = synth.full_sector(s)
    A = omade.forward(th, osc.unpack(sector, s.n), s.n, s.n_alpha, s.n_beta, s.widths)["A"]
    exp = Ns * np.exp(2 * A)
    obs = np.zeros(sector.shape[0])
    idx = np.searchsorted(sector[:, 0], words_from_dev(x)[:, 0])
    assert np.array_equal(sector[idx, 0], words_from_dev(x)[:, 0])
    obs[idx] = c.cpu().numpy()
    big = exp >= 5
    stat = np.sum((obs[big] - exp[big]) ** 2 / exp[big])
    assert chi2.sf(stat, int(big.sum()) - 1) > 1e-6, stat


def test_sampler_edge_cases():
    q = synth.random_problem(3, 3, 0, (32,), seed=2, n_chol=1, decay=2.0, samples=1)
    hq = make_ham(q)
    tq, _ = theta_for(q.theta, elocal.FP64)
    x, c = hq.sample(elocal.Ansatz(q.system.widths, tq, elocal.FP64), 4321, 9)
    assert x.shape[0] == 1 and int(c[0].item()) == 4321
    p = synth.make_problem(0)
    ham = make_ham(p)
    th_dev, _ = theta_for(p.theta, elocal.FP64)
    with pytest.raises(elocal.ElocalError):
        ham.sample(elocal.Ansatz(p.system.widths, th_dev, elocal.FP64), 100000, 1, max_unique=50)
    tb, _ = theta_for(p.theta, elocal.BF16)
    with pytest.raises(elocal.ElocalError):
        ham.sample(elocal.Ansatz(p.system.widths, tb, elocal.BF16), 1000, 1)
