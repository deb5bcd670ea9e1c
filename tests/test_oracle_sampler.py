"""Pins of the BAS oracle (oracle/sampler.py).

* Philox4x32-10 reproduces the published known-answer vectors (tests/golden);
* the binomial sampler: degenerate cases; chi-square against the exact binomial pmf in the
  inversion regime, in both BTRD branches (|K - m| <= 15 and the squeeze/final tests) and
  for p > 1/2; at n = 10^12 the standardised variates are N(0, 1) (KS test) with the
  binomial mean and variance;
* the multinomial split: the counts add up to w, unreachable states get none, the
  marginals follow the probabilities;
* BAS invariants: counts sum to N_s, leaves are distinct and in the sector, the same seed
  gives the same tree and another seed another; a one-determinant sector puts all N_s
  draws on it;
* the leaf frequencies follow |psi|^2 over the full 8-orbital sector (chi-square against
  the oracle's normalised ansatz, p > 1e-6), at N_s = 2e5 and at N_s = 10^12 (the cost
  does not depend on N_s).
"""
import os

import numpy as np
import pytest

from oracle import made, sampler
from oracle import slater_condon as osc
from paper_2506_07430_amd import synth

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "philox4x32_kat.txt")


def test_philox_known_answers():
    rows = [l.split() for l in open(GOLD) if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(t, 16) for t in r]
        ctr = np.array(v[0:4], dtype=np.uint32)
        key = np.array(v[4:6], dtype=np.uint32)
        out = sampler.philox4x32_10(ctr[None, :], key[None, :])[0]
        assert [int(t) for t in out] == v[6:10]


def test_uniforms_range_and_independence():
    u = sampler.uniforms(np.arange(100000), 3, 5, seed=123)
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 0.005 and np.unique(u).size == u.size
    assert not np.array_equal(u[:100], sampler.uniforms(np.arange(100), 3, 6, seed=123))


def _pair(seed, i):
    return lambda t: sampler.uniform_pair(t, i, 0, 0, seed)


def _draws(n, p, count, seed):
    return np.array([sampler.binomial(n, p, _pair(seed, i)) for i in range(count)], dtype=np.int64)


def test_binomial_degenerate_cases():
    assert sampler.binomial(0, 0.3, _pair(1, 0)) == 0
    assert sampler.binomial(10 ** 12, 0.0, _pair(1, 0)) == 0
    assert sampler.binomial(10 ** 12, 1.0, _pair(1, 0)) == 10 ** 12
    assert sampler.binomial(1, 0.5, _pair(1, 0)) in (0, 1)


@pytest.mark.parametrize("n,p", [(30, 0.1), (200, 0.3), (3000, 0.45), (100, 0.8)])
def test_binomial_chi_square_against_pmf(n, p):
    """inversion (n p = 3), BTRD near the mode (n p = 60) and far from it (n p = 1350, sd 27:
    |K - m| > 15 reaches the squeeze and the final acceptance), and p > 1/2 by symmetry."""
    from scipy.stats import binom, chi2
    draws = _draws(n, p, 20000, seed=100 + n)
    assert draws.min() >= 0 and draws.max() <= n
    ks = np.arange(n + 1)
    exp = 20000 * binom.pmf(ks, n, p)
    obs = np.bincount(draws, minlength=n + 1).astype(float)
    # pool the tails until every cell expects at least 5
    keep = exp >= 5
    cells_obs = list(obs[keep]) + [obs[~keep].sum()]
    cells_exp = list(exp[keep]) + [exp[~keep].sum()]
    if cells_exp[-1] < 5:
        cells_obs[-2] += cells_obs.pop()
        cells_exp[-2] += cells_exp.pop()
    stat = sum((o - e) ** 2 / e for o, e in zip(cells_obs, cells_exp))
    assert chi2.sf(stat, len(cells_exp) - 1) > 1e-4, stat


def test_binomial_large_n_is_normal_with_binomial_moments():
    from scipy.stats import kstest
    n, p = 10 ** 12, 0.3
    d = _draws(n, p, 4000, seed=77).astype(np.float64)
    z = (d - n * p) / np.sqrt(n * p * (1 - p))
    assert abs(z.mean()) < 5 / np.sqrt(z.size)
    assert abs(z.var() - 1.0) < 5 * np.sqrt(2.0 / z.size)
    assert kstest(z, "norm").pvalue > 1e-4
    # small mean at huge n: inversion, Poisson(1)-like
    d1 = _draws(10 ** 12, 1e-12, 4000, seed=78)
    assert abs(d1.mean() - 1.0) < 5 * np.sqrt(1.0 / d1.size)


def test_multinomial_split():
    w = 10 ** 9
    p = [0.0, 0.25, 0.0, 0.75]
    tot = np.zeros(4)
    for i in range(400):
        c = sampler.multinomial_split(w, p, lambda st, i=i: (lambda t: sampler.uniform_pair(t, i, 3, st, 5)))
        assert sum(c) == w and c[0] == 0 and c[2] == 0
        tot += c
    assert abs(tot[1] / (400 * w) - 0.25) < 5 * np.sqrt(0.25 * 0.75 / (400 * w))
    assert sampler.multinomial_split(17, [0.0, 0.0, 1.0, 0.0], lambda st: _pair(1, 0)) == [0, 0, 17, 0]
    assert sampler.multinomial_split(0, [0.5, 0.5, 0.0, 0.0], lambda st: _pair(1, 0)) == [0, 0, 0, 0]


def _bas(cfg_system, Ns, seed):
    p = synth.make_problem(0) if cfg_system is None else cfg_system
    s = p.system
    return p, sampler.bas(p.theta, s.n, s.n_alpha, s.n_beta, s.widths, Ns, seed)


def test_bas_invariants_and_seed():
    p, (occ, cnt) = _bas(None, 20000, seed=7)
    s = p.system
    assert cnt.sum() == 20000 and np.all(cnt > 0)
    assert np.all(occ[:, 0::2].sum(1) == s.n_alpha) and np.all(occ[:, 1::2].sum(1) == s.n_beta)
    assert np.unique(osc.pack(occ)).size == occ.shape[0]
    _, (occ2, cnt2) = _bas(p, 20000, seed=7)
    assert np.array_equal(occ, occ2) and np.array_equal(cnt, cnt2)
    _, (occ3, cnt3) = _bas(p, 20000, seed=8)
    assert not (np.array_equal(occ, occ3) and np.array_equal(cnt, cnt3))


def test_bas_single_determinant_sector():
    q = synth.random_problem(3, 3, 0, (32,), seed=2, n_chol=1, decay=2.0, samples=1)
    s = q.system
    occ, cnt = sampler.bas(q.theta, s.n, s.n_alpha, s.n_beta, s.widths, 12345, seed=1)
    assert occ.shape[0] == 1 and cnt[0] == 12345


@pytest.mark.parametrize("Ns", [200000, 10 ** 12])
def test_bas_frequencies_follow_psi_squared(Ns):
    from scipy.stats import chi2
    p = synth.make_problem(0)
    s = p.system
    occ, cnt = sampler.bas(p.theta, s.n, s.n_alpha, s.n_beta, s.widths, Ns, seed=11)
    assert cnt.sum() == Ns
    sector = synth.full_sector(s)
    A = made.forward(p.theta, osc.unpack(sector, s.n), s.n, s.n_alpha, s.n_beta, s.widths)["A"]
    prob = np.exp(2 * A)
    assert abs(prob.sum() - 1.0) < 1e-12
    obs = np.zeros(sector.shape[0])
    idx = np.searchsorted(sector[:, 0], osc.pack(occ)[:, 0])
    obs[idx] = cnt
    exp = Ns * prob
    big = exp >= 5
    stat = np.sum((obs[big] - exp[big]) ** 2 / exp[big])
    df = int(big.sum()) - 1
    assert chi2.sf(stat, df) > 1e-6, (stat, df)
