"""Full-sector vectors and the KPM recursion on the GPU, against the FP64 oracle.

Bars: the sector basis is bit-exact; H v within 1e-12 of the largest |(H v)_r| (FP64,
different summation order); moments within 1e-10 Omega_0 after 200 recursion steps;
line shapes within 1e-11 of the largest value; results bitwise repeatable.
"""
from math import comb

import numpy as np
import pytest
import torch

from oracle import kpm as okpm
from oracle import slater_condon as osc
from paper_2506_07430_amd import elocal, synth
from tests.gpu_common import make_ham, words_from_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    torch.cuda.set_device(0)


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64).cuda()


@pytest.mark.parametrize("n,na,nb", [(8, 4, 4), (6, 3, 2), (5, 0, 2), (33, 1, 1), (7, 7, 0)])
def test_sector_basis_bit_exact(n, na, nb):
    p = synth.random_problem(n, na, nb, (32,), seed=60 + n, n_chol=2, decay=3.0, samples=1)
    ham = make_ham(p)
    assert ham.sector_dim == comb(n, na) * comb(n, nb)
    got = words_from_dev(ham.sector_basis())
    want = osc.pack(okpm.sector_basis(n, na, nb))
    assert np.array_equal(got, want)


def test_sector_apply_full_c0_and_dots():
    p = synth.make_problem(0)
    s = p.system
    ham = make_ham(p)
    H = okpm.sector_hamiltonian_sparse(p.h1e, p.eri, s.n, s.n_alpha, s.n_beta)
    rng = np.random.default_rng(5)
    v, z = rng.standard_normal(H.shape[0]), rng.standard_normal(H.shape[0])
    y, d = ham.sector_apply(_dev(v), ch=0.7, cv=-0.3, z=_dev(z), cz=-1.0, dots=True)
    torch.cuda.synchronize()
    ref = 0.7 * (H @ v) - 0.3 * v - z
    got = y.cpu().numpy()
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
    dd = d.cpu().numpy()
    assert abs(dd[0] - ref @ ref) <= 1e-12 * (ref @ ref)
    assert abs(dd[1] - ref @ v) <= 1e-11 * np.abs(ref) @ np.abs(v)
    y2 = ham.sector_apply(_dev(v), ch=0.7, cv=-0.3, z=_dev(z), cz=-1.0)
    torch.cuda.synchronize()
    assert torch.equal(y, y2)


@pytest.mark.parametrize("n,na,nb,rows", [(12, 6, 6, (0, 1, 4321, 853775)), (33, 2, 1, (0, 9000, 17423)),
                                          (16, 3, 4, (0, 777, 1000000 % 1019200))])
def test_sector_apply_rows_of_large_sectors(n, na, nb, rows):
    """Sampled rows of big sectors (12 orbitals: 853,776 determinants; two-word case)."""
    p = synth.random_problem(n, na, nb, (32,), seed=70 + n, n_chol=4, decay=4.0, samples=1)
    ham = make_ham(p)
    dim = ham.sector_dim
    print(f"sector n={n} ({na},{nb}): dim {dim}", flush=True)
    v = np.random.default_rng(n).standard_normal(dim)
    y = ham.sector_apply(_dev(v)).cpu().numpy()
    for r in rows:
        ref = okpm.row_apply(p.h1e, p.eri, n, na, nb, r, v)
        assert abs(y[r] - ref) <= 1e-12 * max(1.0, abs(ref)), f"row {r}"


def _window(Hd):
    e = np.linalg.eigvalsh(Hd)
    return (e[-1] - e[0]) / (2 - 0.02), (e[-1] + e[0]) / 2, e


def test_kpm_moments_and_line_shape_c0_dipole_ground_state():
    p = synth.make_problem(0)
    s = p.system
    n, na, nb = s.n, s.n_alpha, s.n_beta
    Hd = okpm.sector_hamiltonian_dense(p.h1e, p.eri, n, na, nb)
    a, b, e = _window(Hd)
    psi0 = np.linalg.eigh(Hd)[1][:, 0]
    d = synth.make_dipole(n, seed=1)
    mu_core = 0.125
    alpha_ref = okpm.dipole_apply(d, mu_core, n, na, nb, psi0)
    # dipole through a one-body handle (h1e = -d, no two-body part)
    hd = elocal.Hamiltonian(-d, np.zeros((n,) * 4), n, na, nb)
    alpha = hd.sector_apply(_dev(psi0), ch=1.0, cv=-mu_core)
    torch.cuda.synchronize()
    assert np.max(np.abs(alpha.cpu().numpy() - alpha_ref)) <= 1e-12 * np.max(np.abs(alpha_ref))
    ham = make_ham(p)
    N = 200
    mu = ham.kpm_moments(alpha, N, a, b)
    mu2 = ham.kpm_moments(alpha, N, a, b)
    torch.cuda.synchronize()
    assert torch.equal(mu, mu2)
    ref = okpm.chebyshev_moments(Hd, alpha_ref, N, a, b)
    got = mu.cpu().numpy()
    print(f"moments: max |dOmega| / Omega_0 = {np.max(np.abs(got - ref)) / ref[0]:.2e}")
    assert np.max(np.abs(got - ref)) <= 1e-10 * ref[0]
    w = np.linspace(-0.995, 0.995, 501)
    rho = elocal.kpm_line_shape(mu, _dev(w)).cpu().numpy()
    rref = okpm.line_shape(ref, w)
    assert np.max(np.abs(rho - rref)) <= 1e-11 * np.max(np.abs(rref))


@pytest.mark.parametrize("N", [1, 2, 3, 7])
def test_kpm_small_moment_counts(N):
    p = synth.random_problem(6, 3, 3, (32,), seed=5, n_chol=3, decay=3.0, samples=1)
    n = 6
    Hd = okpm.sector_hamiltonian_dense(p.h1e, p.eri, n, 3, 3)
    a, b, _ = _window(Hd)
    alpha = np.random.default_rng(N).standard_normal(Hd.shape[0])
    mu = make_ham(p).kpm_moments(_dev(alpha), N, a, b).cpu().numpy()
    ref = okpm.chebyshev_moments(Hd, alpha, N, a, b)
    assert np.max(np.abs(mu - ref)) <= 1e-12 * ref[0]


def test_sector_errors():
    p = synth.random_problem(40, 20, 20, (32,), seed=1, n_chol=1, decay=2.0, samples=1)
    ham = make_ham(p)
    assert ham.sector_dim == -1          # C(40, 20)^2 > 2^31
    with pytest.raises(elocal.ElocalError):
        ham.sector_basis()
