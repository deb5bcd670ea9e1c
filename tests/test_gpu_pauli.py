"""The paper's Pauli-string local-energy route on the GPU (elocal_eval_pauli).

Checks: the number of strings and of unique flip masks equals the oracle's
Jordan--Wigner Hamiltonian; local energies equal the Slater--Condon route of the same
library (same ansatz values, different grouping of the matrix elements: 1e-9 relative)
and the oracle's own Pauli-route local energy (Algorithm 1 with the Pauli-element
equation) on the same BF16-rounded parameters (1e-5 Ha).
"""
import numpy as np
import pytest
import torch

from oracle import made as omade
from oracle import pauli as opauli
from oracle import slater_condon as osc
from paper_2506_07430_amd import elocal, synth
from tests.gpu_common import ansatz_samples, make_ham, theta_for, words_to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    torch.cuda.set_device(0)


def _c(e):
    e = e.cpu().numpy()
    return e[:, 0] + 1j * e[:, 1]


def test_pauli_route_c0_against_oracle_and_slater_condon():
    p = synth.make_problem(0)
    s = p.system
    ham = make_ham(p)
    n_str, n_flip = ham.pauli_build()
    terms = opauli.qubit_hamiltonian(p.h1e, p.eri)
    cmax = max(abs(v) for v in terms.values())
    kept = {k: v for k, v in terms.items() if abs(v) > 1e-13 * cmax}
    print(f"c0: {n_str} strings, {n_flip} unique flips (oracle {len(kept)} strings)")
    assert n_str == len(kept)
    assert n_flip == len({x for (x, _) in kept}) + (0 if any(x == 0 for (x, _) in kept) else 1)
    x = ansatz_samples(p, 256, seed=2)
    th_dev, th = theta_for(p.theta, elocal.BF16)
    ans = elocal.Ansatz(s.widths, th_dev, elocal.BF16)
    xd = words_to_dev(x)
    e_pauli = _c(ham.eval_pauli(ans, xd))
    e_sc = _c(ham.eval(ans, xd, want_logpsi=False)[0])
    torch.cuda.synchronize()
    rel = np.max(np.abs(e_pauli - e_sc)) / np.max(np.abs(e_sc))
    print(f"c0: Pauli vs Slater-Condon route max rel {rel:.2e}")
    assert rel <= 1e-9
    labels = opauli.pauli_labels(kept, 2 * s.n)

    def psi_of(occ):
        f = omade.forward(th, occ, s.n, s.n_alpha, s.n_beta, s.widths)
        return np.exp(f["A"] + 1j * f["phi"])

    occ = osc.unpack(x[:6], s.n)
    ref = np.array([opauli.local_energy(labels, o, psi_of) for o in occ])
    err = np.max(np.abs(e_pauli[:6] - ref))
    print(f"c0: Pauli route vs oracle max |dE_loc| {err:.2e}")
    assert err <= 1e-5


@pytest.mark.parametrize("precision", [elocal.BF16, elocal.BF16X3])
def test_pauli_route_n24_equals_slater_condon(precision):
    p = synth.make_problem(1, samples=64)
    s = p.system
    ham = make_ham(p)
    n_str, n_flip = ham.pauli_build()
    print(f"n24: {n_str} strings, {n_flip} unique flips vs {ham.C} connected determinants", flush=True)
    th_dev, _ = theta_for(p.theta, precision)
    ans = elocal.Ansatz(s.widths, th_dev, precision)
    xd = words_to_dev(p.x[:32])
    e_pauli = _c(ham.eval_pauli(ans, xd))
    e_sc = _c(ham.eval(ans, xd, want_logpsi=False)[0])
    torch.cuda.synchronize()
    rel = np.max(np.abs(e_pauli - e_sc) / np.abs(e_sc))
    print(f"n24: Pauli vs Slater-Condon route max rel {rel:.2e}")
    assert rel <= 1e-9


def test_pauli_route_needs_build_and_bf16():
    p = synth.make_problem(0)
    ham = make_ham(p)
    th_dev, _ = theta_for(p.theta, elocal.BF16)
    ans = elocal.Ansatz(p.system.widths, th_dev, elocal.BF16)
    with pytest.raises(elocal.ElocalError):
        ham.eval_pauli(ans, words_to_dev(p.x[:4]))
    ham.pauli_build()
    th64, _ = theta_for(p.theta, elocal.FP64)
    with pytest.raises(elocal.ElocalError):
        ham.eval_pauli(elocal.Ansatz(p.system.widths, th64, elocal.FP64), words_to_dev(p.x[:4]))
