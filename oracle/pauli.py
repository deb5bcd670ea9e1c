"""The paper's own local-energy route: Jordan--Wigner Pauli strings (small systems only).

Methods ("Mapping fermionic Hamiltonians to the qubits"): a+_j -> (prod_{i<j} Z_i)
sigma+_j, giving H_Q = sum_p h_p P_p with real h_p. Results (local-energy equation,
Algorithm 1, Pauli-element equation): each Pauli string P_p couples x to exactly one
x^p = x XOR (positions of X and Y in P_p), with
    <x|P_p|x^p> = (-i)^r prod_{k: P_k in {Y, Z}} (-1)^{x_k},   r = number of Y's,
and l(x) = sum_p h_p <x|P_p|x^p> Psi(x^p)/Psi(x).

Reading of sigma+ (the paper writes sigma^x +- i sigma^y without the 1/2 and does not
fix which of |0>, |1> is occupied): occupied = |1> with Z|n> = (-1)^n |n>, so
a+_j = (prod_{i<j} Z_i) (X_j - i Y_j)/2, which is the reading consistent with the
Pauli-element equation above.

Strings are held as (xbits, zbits) with value i^ph X^xbits Z^zbits (X before Z on
each qubit; Y = i X Z). Used only as an independent cross-check on tiny systems.
"""
from __future__ import annotations

from collections import defaultdict

import numpy as np


def _mul(a, b):
    """(c1, x1, z1) * (c2, x2, z2) for strings c X^x Z^z."""
    c1, x1, z1 = a
    c2, x2, z2 = b
    sign = -1 if bin(z1 & x2).count("1") % 2 else 1
    return (c1 * c2 * sign, x1 ^ x2, z1 ^ z2)


def _ladder(j: int, dagger: bool):
    """a_j or a+_j as a list of (coef, xbits, zbits)."""
    zs = (1 << j) - 1
    e = 1 << j
    # X_j -/+ i Y_j = X_j -/+ i (i X_j Z_j) = X_j +/- X_j Z_j  (a+ uses -iY)
    s = 1.0 if dagger else -1.0
    return [(0.5, e, zs), (0.5 * s, e, zs | e)]


def _product(ops):
    terms = [(1.0 + 0j, 0, 0)]
    for op in ops:
        terms = [_mul(t, o) for t in terms for o in op]
    return terms


def qubit_hamiltonian(h1e, eri):
    """{(xbits, zbits): coefficient of X^x Z^z} for the Hamiltonian of ``oracle.fock``."""
    n = h1e.shape[0]
    acc = defaultdict(complex)
    for s in (0, 1):
        for p in range(n):
            for q in range(n):
                if h1e[p, q] != 0.0:
                    for c, x, z in _product([_ladder(2 * p + s, True), _ladder(2 * q + s, False)]):
                        acc[(x, z)] += h1e[p, q] * c
    for s in (0, 1):
        for t in (0, 1):
            for p in range(n):
                for q in range(n):
                    for r in range(n):
                        for ss in range(n):
                            v = 0.5 * eri[p, q, r, ss]
                            if v == 0.0 or (2 * p + s == 2 * r + t) or (2 * q + s == 2 * ss + t):
                                continue
                            ops = [_ladder(2 * p + s, True), _ladder(2 * r + t, True),
                                   _ladder(2 * ss + t, False), _ladder(2 * q + s, False)]
                            for c, x, z in _product(ops):
                                acc[(x, z)] += v * c
    return {k: v for k, v in acc.items() if abs(v) > 1e-14}


def pauli_labels(terms, n_qubits):
    """Convert c X^x Z^z to h_p P_p with Pauli labels: returns [(h_p, label string)].

    On a qubit with both bits set, X Z = -i Y, so c X^x Z^z = c (-i)^r P_label.
    """
    out = []
    for (x, z), c in terms.items():
        lab = []
        r = 0
        for k in range(n_qubits):
            xb, zb = (x >> k) & 1, (z >> k) & 1
            if xb and zb:
                lab.append("y")
                r += 1
            elif xb:
                lab.append("x")
            elif zb:
                lab.append("z")
            else:
                lab.append("i")
        h = c * (-1j) ** r
        out.append((h, "".join(lab)))
    return out


def pauli_element(label: str, x_bits) -> complex:
    """<x|P|x^p> = (-i)^r prod_{k: P_k in {y,z}} (-1)^{x_k}."""
    r = label.count("y")
    sgn = 1
    for k, c in enumerate(label):
        if c in "yz" and x_bits[k]:
            sgn = -sgn
    return ((-1j) ** r) * sgn


def local_energy(strings, x_bits, psi_of) -> complex:
    """l(x) = sum_p h_p <x|P_p|x^p> Psi(x^p)/Psi(x) (Algorithm 1, one sample)."""
    x_bits = np.asarray(x_bits, dtype=np.uint8)
    flips = np.array([[1 if c in "xy" else 0 for c in lab] for _, lab in strings], dtype=np.uint8)
    xp = x_bits[None, :] ^ flips
    amp = psi_of(xp)
    amp0 = psi_of(x_bits[None, :])[0]
    tot = 0j
    for (h, lab), a in zip(strings, amp):
        if a != 0:
            tot += h * pauli_element(lab, x_bits) * a
    return tot / amp0
