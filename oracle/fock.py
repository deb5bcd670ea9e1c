"""Hamiltonian matrix built by applying creation/annihilation operators (oracle A).

Follows the Methods section ("Mapping fermionic Hamiltonians to the qubits"): the
second-quantised electronic Hamiltonian with one- and two-body integrals, and the
Jordan--Wigner map in which the occupation of mode j sits on qubit j and the
fermionic sign is the parity of the occupied modes before j.

Readings fixed here (the paper leaves them open):

* spin-orbital index k = 2p + s for spatial orbital p and spin s (0 = alpha/up,
  1 = beta/down): the paper puts spatial orbital i on qubits 2i-1 (up) and 2i
  (down), 1-based; this is the same order 0-based;
* |x> = a+_{k1} a+_{k2} ... a+_{km} |vac> with k1 < k2 < ... < km, so
  a_k |x> = (-1)^{#occupied l < k} |x - e_k> and likewise for a+_k (the string of
  Z's of the Jordan--Wigner map runs over the modes before k);
* the integrals are spatial and in chemists' order, h1e[p, q] and
  eri[p, q, r, s] = (pq|rs); the Hamiltonian is

      H = sum_{pq,s} h_pq a+_{ps} a_{qs}
          + 1/2 sum_{pqrs, s t} (pq|rs) a+_{ps} a+_{rt} a_{st} a_{qs}

  (the paper's ``h_pqrs a+_p a+_q a_r a_s`` read with h_pqrs = <pq|sr> = (ps|qr)).

Determinants are int64 bit masks (2n <= 62), bit k = spin-orbital k. This module
is independent of the Slater--Condon enumerator: it never uses excitation rules,
only operator algebra applied determinant by determinant (vectorised with NumPy).
"""
from __future__ import annotations

import itertools

import numpy as np


def _parity_below(states: np.ndarray, k: int) -> np.ndarray:
    """Number of occupied modes l < k, modulo 2 (the Jordan--Wigner string)."""
    below = np.int64((1 << k) - 1)
    return np.bitwise_count(states & below).astype(np.int64) & 1


def annihilate(states: np.ndarray, signs: np.ndarray, k: int):
    """Apply a_k to the determinants (with accumulated signs); drop those killed."""
    bit = np.int64(1 << k)
    alive = (states & bit) != 0
    st = states[alive]
    sg = signs[alive] * (1 - 2 * _parity_below(st, k))
    return st ^ bit, sg, alive


def create(states: np.ndarray, signs: np.ndarray, k: int):
    """Apply a+_k to the determinants (with accumulated signs); drop those killed."""
    bit = np.int64(1 << k)
    alive = (states & bit) == 0
    st = states[alive]
    sg = signs[alive] * (1 - 2 * _parity_below(st, k))
    return st | bit, sg, alive


def sector_basis(n: int, n_alpha: int, n_beta: int) -> np.ndarray:
    """Sorted int64 masks of every determinant with n_alpha up and n_beta down electrons."""
    out = []
    for a in itertools.combinations(range(n), n_alpha):
        for b in itertools.combinations(range(n), n_beta):
            m = 0
            for p in a:
                m |= 1 << (2 * p)
            for p in b:
                m |= 1 << (2 * p + 1)
            out.append(m)
    return np.array(sorted(out), dtype=np.int64)


def fock_basis(n: int) -> np.ndarray:
    """All 2^(2n) determinants (every particle number)."""
    return np.arange(1 << (2 * n), dtype=np.int64)


def hamiltonian_matrix(h1e: np.ndarray, eri: np.ndarray, basis: np.ndarray) -> np.ndarray:
    """Dense <x'|H|x> over `basis` (sorted int64 masks), by explicit operator application.

    Every term of H is applied right-to-left to every basis determinant; the
    resulting determinant must lie in `basis` (true for a full sector or the whole
    Fock space, since H conserves both electron numbers).
    """
    n = h1e.shape[0]
    D = basis.size
    H = np.zeros((D, D))
    col0 = np.arange(D)
    ones = np.ones(D, dtype=np.int64)

    def scatter(states, signs, cols, coef):
        rows = np.searchsorted(basis, states)
        if np.any(rows >= D) or np.any(basis[np.minimum(rows, D - 1)] != states):
            raise ValueError("basis is not closed under H")
        np.add.at(H, (rows, cols), coef * signs)

    # one-body part: h_pq a+_{p s} a_{q s}
    for s in (0, 1):
        for q in range(n):
            st1, sg1, m1 = annihilate(basis, ones, 2 * q + s)
            c1 = col0[m1]
            for p in range(n):
                if h1e[p, q] == 0.0:
                    continue
                st2, sg2, m2 = create(st1, sg1, 2 * p + s)
                scatter(st2, sg2, c1[m2], h1e[p, q])

    # two-body part: 1/2 (pq|rs) a+_{p s} a+_{r t} a_{s t} a_{q s}
    for s in (0, 1):
        for q in range(n):
            st1, sg1, m1 = annihilate(basis, ones, 2 * q + s)
            c1 = col0[m1]
            for t in (0, 1):
                for ss in range(n):
                    st2, sg2, m2 = annihilate(st1, sg1, 2 * ss + t)
                    c2 = c1[m2]
                    if st2.size == 0:
                        continue
                    for r in range(n):
                        st3, sg3, m3 = create(st2, sg2, 2 * r + t)
                        c3 = c2[m3]
                        if st3.size == 0:
                            continue
                        for p in range(n):
                            coef = 0.5 * eri[p, q, r, ss]
                            if coef == 0.0:
                                continue
                            st4, sg4, m4 = create(st3, sg3, 2 * p + s)
                            if st4.size:
                                scatter(st4, sg4, c3[m4], coef)
    return H


def number_operators(basis: np.ndarray, n: int):
    """Diagonals of N_alpha and N_beta over `basis`."""
    a_mask = np.int64(sum(1 << (2 * p) for p in range(n)))
    b_mask = np.int64(sum(1 << (2 * p + 1) for p in range(n)))
    return (np.bitwise_count(basis & a_mask).astype(np.int64),
            np.bitwise_count(basis & b_mask).astype(np.int64))
