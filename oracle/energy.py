"""Local energies, energy statistics and the VMC gradient in FP64.

* Local energy (Results, eq. for l_theta(x); Methods, eq. for l_theta in the VMC
  objective): E_loc(x) = sum_{x'} H_{x x'} Psi(x') / Psi(x), with the sum over the
  canonical list of ``oracle.slater_condon`` (H is real symmetric, H_{x x'} = H_{x' x})
  and Psi(x')/Psi(x) = exp(A(x') - A(x) + i (phi(x') - phi(x))).
* Energy (Methods, batch estimator of <H>): for unique samples with multiplicities
  w_i the estimator is <E> = sum_i w_i E_loc,i / sum_i w_i (complex); the reported
  energy is Re <E>; the weighted variance is sum_i w_i |E_loc,i - <E>|^2 / sum_i w_i.
  The factor 1/2 of the paper's objective is dropped: the energy is <H> itself.
* Gradient (Methods, gradient estimator with baseline b = E[l]): with
  log Psi = A + i phi and real parameters,
      G = 2 Re sum_i wbar_i (E_loc,i - <E>) d log Psi*(x_i)
        = 2 sum_i wbar_i [Re(E_loc,i - <E>) dA_i + Im(E_loc,i - <E>) dphi_i],
  wbar = w / sum w and <E> complex and held fixed. This is twice the paper's
  estimator, i.e. the gradient of <H> rather than of <H>/2.
"""
from __future__ import annotations

import numpy as np

from . import made, slater_condon


def log_psi(theta, x_words, n, n_alpha, n_beta, widths):
    """(A, phi) for packed determinants [B, W]."""
    occ = slater_condon.unpack(x_words, n)
    f = made.forward(theta, occ, n, n_alpha, n_beta, widths)
    return f["A"], f["phi"]


def local_energy_one(occ, n, n_alpha, n_beta, widths, theta, ints):
    states, _, _, H = slater_condon.connected(occ, n, ints)
    f = made.forward(theta, states, n, n_alpha, n_beta, widths)
    f0 = made.forward(theta, occ[None, :], n, n_alpha, n_beta, widths)
    ratio = np.exp(f["A"] - f0["A"][0] + 1j * (f["phi"] - f0["phi"][0]))
    return np.sum(H * ratio)


def local_energies(h1e, eri, n, n_alpha, n_beta, widths, theta, x_words):
    """E_loc for each packed determinant (complex128 [B])."""
    occ = slater_condon.unpack(x_words, n)
    ints = slater_condon.SpinIntegrals(h1e, eri)
    return np.array([local_energy_one(o, n, n_alpha, n_beta, widths, theta, ints) for o in occ])


def local_energies_given_psi(h1e, eri, n, x_words, psi_of):
    """E_loc with an arbitrary amplitude function psi_of(states [M, 2n]) -> complex [M]."""
    occ = slater_condon.unpack(x_words, n)
    ints = slater_condon.SpinIntegrals(h1e, eri)
    out = []
    for o in occ:
        states, _, _, H = slater_condon.connected(o, n, ints)
        out.append(np.sum(H * psi_of(states)) / psi_of(o[None, :])[0])
    return np.array(out)


def energy_stats(eloc, w):
    """(Re<E>, Im<E>, weighted variance, sum of weights)."""
    eloc = np.asarray(eloc, dtype=np.complex128)
    w = np.asarray(w, dtype=np.float64)
    sw = w.sum()
    e = np.sum(w * eloc) / sw
    var = np.sum(w * np.abs(eloc - e) ** 2) / sw
    return e.real, e.imag, var, sw


def vmc_gradient(theta, x_words, w, eloc, n, n_alpha, n_beta, widths):
    """Flat gradient 2 Re <(E_loc - <E>) d log Psi*> (masked entries exactly 0)."""
    eloc = np.asarray(eloc, dtype=np.complex128)
    w = np.asarray(w, dtype=np.float64)
    wbar = w / w.sum()
    e = np.sum(wbar * eloc)
    d = eloc - e
    gA = 2.0 * wbar * d.real
    gphi = 2.0 * wbar * d.imag
    occ = slater_condon.unpack(x_words, n)
    return made.backward(theta, occ, n, n_alpha, n_beta, widths, gA, gphi)
