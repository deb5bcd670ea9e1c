"""Pins of the KPM oracle (oracle/kpm.py) against routes that share none of its code paths.

* the sector ranking is a bijection onto [0, dim) with the closed-form extremes;
* the Slater--Condon sparse matrix equals the operator-built dense matrix in that basis;
* recursion + moment doubling equal the spectral formula sum_k |<k|alpha>|^2 T_n(E~_k)
  from a dense eigendecomposition, and the moments formed without doubling;
* the Jackson kernel has g_0 = 1, lies in (0, 1] and decreases; a Jackson-damped single
  line peaks at its position and integrates to its weight;
* the line shape integrates to Omega_0 (Chebyshev orthogonality, Gauss--Chebyshev rule);
* the dipole operator with d = identity is -(N_alpha + N_beta) - mu_c.
"""
from math import comb

import numpy as np
import pytest

from oracle import fock, kpm
from paper_2506_07430_amd import synth


def test_set_rank_bijection_and_extremes():
    import itertools
    for n, k in [(8, 4), (9, 2), (6, 0), (6, 6), (12, 5)]:
        ranks = sorted(kpm.set_rank(s) for s in itertools.combinations(range(n), k))
        assert ranks == list(range(comb(n, k)))
        assert kpm.set_rank(range(k)) == 0
        assert kpm.set_rank(range(n - k, n)) == comb(n, k) - 1
        for r in (0, comb(n, k) // 3, comb(n, k) - 1):
            assert kpm.set_rank(kpm.set_unrank(r, k)) == r


def test_sector_basis_is_the_sector_and_indexes_itself():
    n, na, nb = 6, 3, 2
    occ = kpm.sector_basis(n, na, nb)
    assert occ.shape == (kpm.sector_dim(n, na, nb), 2 * n)
    assert np.all(occ[:, 0::2].sum(1) == na) and np.all(occ[:, 1::2].sum(1) == nb)
    assert all(kpm.sector_index(occ[r], n, nb) == r for r in range(occ.shape[0]))
    assert set(kpm._masks(occ).tolist()) == set(fock.sector_basis(n, na, nb).tolist())


@pytest.mark.parametrize("n,na,nb", [(6, 3, 3), (6, 2, 3), (5, 0, 2)])
def test_sparse_lists_equal_operator_construction(n, na, nb):
    p = synth.random_problem(n, na, nb, (16,), seed=40 + n + na, n_chol=4, decay=3.0, samples=2)
    Hd = kpm.sector_hamiltonian_dense(p.h1e, p.eri, n, na, nb)
    Hs = kpm.sector_hamiltonian_sparse(p.h1e, p.eri, n, na, nb).toarray()
    assert np.max(np.abs(Hd - Hs)) <= 1e-12 * np.max(np.abs(Hd))
    r = 7 % Hd.shape[0]
    v = np.random.default_rng(1).standard_normal(Hd.shape[0])
    assert abs(kpm.row_apply(p.h1e, p.eri, n, na, nb, r, v) - (Hd @ v)[r]) <= 1e-12 * np.abs(Hd).sum()


def _window(Hd):
    e = np.linalg.eigvalsh(Hd)
    a = (e[-1] - e[0]) / (2 - 0.02)
    b = (e[-1] + e[0]) / 2
    return a, b


def test_moments_equal_spectral_formula_and_direct():
    n, na, nb = 6, 3, 3
    p = synth.random_problem(n, na, nb, (16,), seed=3, n_chol=5, decay=3.0, samples=2)
    Hd = kpm.sector_hamiltonian_dense(p.h1e, p.eri, n, na, nb)
    a, b = _window(Hd)
    alpha = np.random.default_rng(7).standard_normal(Hd.shape[0])
    N = 61
    mu = kpm.chebyshev_moments(Hd, alpha, N, a, b)
    e, U = np.linalg.eigh(Hd)
    w = (U.T @ alpha) ** 2
    x = (e - b) / a
    spectral = np.array([np.sum(w * np.cos(k * np.arccos(x))) for k in range(N)])
    assert np.max(np.abs(mu - spectral)) <= 1e-10 * mu[0]
    assert np.max(np.abs(mu - kpm.moments_direct(Hd, alpha, N, a, b))) <= 1e-10 * mu[0]
    assert np.all(np.abs(mu) <= mu[0] * (1 + 1e-12))      # |T_n| <= 1 on the window


def test_jackson_kernel_properties_and_single_line():
    for N in (16, 100, 1000):
        g = kpm.jackson(N)
        assert abs(g[0] - 1.0) <= 1e-14
        assert np.all(g > -1e-15) and np.all(g <= 1 + 1e-15) and np.all(np.diff(g) <= 1e-15)
    N, x0 = 400, 0.3
    mu = np.cos(np.arange(N) * np.arccos(x0))               # moments of delta(x - x0)
    w = np.linspace(-0.99, 0.99, 4001)
    rho = kpm.line_shape(mu, w)
    assert abs(w[np.argmax(rho)] - x0) <= np.pi / N
    M = 2 * N
    nodes = np.cos(np.pi * (np.arange(M) + 0.5) / M)
    # Gauss--Chebyshev: integral of rho = mean over the nodes of rho * pi * sqrt(1 - x^2)
    assert abs(np.mean(kpm.line_shape(mu, nodes) * np.pi * np.sqrt(1 - nodes ** 2)) - 1.0) <= 1e-12


def test_line_shape_integrates_to_omega0():
    rng = np.random.default_rng(0)
    mu = np.cumprod(np.full(50, 0.95)) * rng.uniform(0.5, 1.0, 50)
    mu[0] = 2.5
    M = 200
    nodes = np.cos(np.pi * (np.arange(M) + 0.5) / M)
    # Gauss--Chebyshev: integral of f(x) dx = (pi / M) sum f(x_j) sqrt(1 - x_j^2)
    integral = (np.pi / M) * np.sum(kpm.line_shape(mu, nodes) * np.sqrt(1 - nodes ** 2))
    assert abs(integral - mu[0]) <= 1e-12 * mu[0]


def test_dipole_identity_is_minus_particle_number():
    n, na, nb = 5, 2, 3
    rng = np.random.default_rng(2)
    psi = rng.standard_normal(kpm.sector_dim(n, na, nb))
    out = kpm.dipole_apply(np.eye(n), 0.25, n, na, nb, psi)
    assert np.allclose(out, -(na + nb + 0.25) * psi, rtol=0, atol=1e-13)
