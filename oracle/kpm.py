"""Kernel polynomial method for the dipole spectrum, in FP64 (test infrastructure).

Follows the Methods section ("KPM for absorption spectra") and the KPM expansion of the
Results section:

* full-sector vectors: every determinant of the (n_alpha, n_beta) sector gets the index
  r = rank(alpha set) * C(n, n_beta) + rank(beta set), where a set of occupied spatial
  orbitals o_1 < o_2 < ... < o_k (0-based) has the combinatorial-number-system rank
  sum_i C(o_i, i) (i = 1..k); this is a reading (the paper stores no full-space vectors);
* the dipole operator mu = -sum_pq d_pq (a+_{p up} a_{q up} + a+_{p down} a_{q down}) - mu_c,
  a one-body operator, so |alpha> = mu |0> is the one-body "Hamiltonian" with h = -d and no
  two-body part applied to |0>, minus mu_c |0>;
* rescaling H~ = (H - b) / a (a > 0 the half-width, b the centre of the spectrum window);
* the recursion alpha_0 = alpha, alpha_1 = H~ alpha_0, alpha_{n+1} = 2 H~ alpha_n - alpha_{n-1};
* moment doubling Omega_{2n} = 2 <alpha_n|alpha_n> - Omega_0,
  Omega_{2n+1} = 2 <alpha_{n+1}|alpha_n> - Omega_1;
* the Jackson kernel in its standard form g_n = [(N - n + 1) cos(pi n / (N + 1))
  + sin(pi n / (N + 1)) cot(pi / (N + 1))] / (N + 1) (the printed formula has N - n - 1,
  read as a typo: with it g_0 != 1);
* the line shape rho(w~) = [g_0 Omega_0 + 2 sum_n g_n Omega_n T_n(w~)] / (pi sqrt(1 - w~^2)),
  which approximates sum_k |<k|alpha>|^2 delta(w~ - E~_k) (the printed expansion lacks the
  1/pi and places the delta at -E_k; Im C = -pi rho is the paper's quantity).

Nothing here is shared with the HIP library.
"""
from __future__ import annotations

from math import comb

import numpy as np

from . import fock, slater_condon


# ----------------------------------------------------------------------------- sector indexing
def set_rank(orbitals) -> int:
    """Combinatorial-number-system rank of a set of 0-based orbitals."""
    return sum(comb(int(o), i + 1) for i, o in enumerate(sorted(int(o) for o in orbitals)))


def set_unrank(r: int, k: int) -> list:
    """Inverse of set_rank for sets of size k (greedy from the largest element)."""
    out = []
    for i in range(k, 0, -1):
        o = i - 1
        while comb(o + 1, i) <= r:
            o += 1
        out.append(o)
        r -= comb(o, i)
    return sorted(out)


def sector_dim(n: int, n_alpha: int, n_beta: int) -> int:
    return comb(n, n_alpha) * comb(n, n_beta)


def sector_index(occ: np.ndarray, n: int, n_beta: int) -> int:
    """Index of one determinant (uint8[2n]) in the full-sector vector."""
    a = [p for p in range(n) if occ[2 * p]]
    b = [p for p in range(n) if occ[2 * p + 1]]
    return set_rank(a) * comb(n, n_beta) + set_rank(b)


def sector_basis(n: int, n_alpha: int, n_beta: int) -> np.ndarray:
    """All determinants of the sector as occupations [dim, 2n] (uint8), row r = index r."""
    nb_dim = comb(n, n_beta)
    dim = comb(n, n_alpha) * nb_dim
    occ = np.zeros((dim, 2 * n), dtype=np.uint8)
    for ra in range(comb(n, n_alpha)):
        a = set_unrank(ra, n_alpha)
        for rb in range(nb_dim):
            r = ra * nb_dim + rb
            occ[r, [2 * p for p in a]] = 1
            occ[r, [2 * p + 1 for p in set_unrank(rb, n_beta)]] = 1
    return occ


def _masks(occ: np.ndarray) -> np.ndarray:
    w = np.zeros(occ.shape[0], dtype=np.int64)
    for k in range(occ.shape[1]):
        w |= occ[:, k].astype(np.int64) << k
    return w


# ----------------------------------------------------------------------------- operators
def sector_hamiltonian_dense(h1e, eri, n: int, n_alpha: int, n_beta: int) -> np.ndarray:
    """Dense H in the sector basis, by operator construction (small sectors only)."""
    masks = _masks(sector_basis(n, n_alpha, n_beta))
    order = np.argsort(masks)                 # operator construction wants sorted masks
    Hs = fock.hamiltonian_matrix(np.asarray(h1e, float), np.asarray(eri, float), masks[order])
    pos = np.empty_like(order)
    pos[order] = np.arange(order.size)        # ranked index -> position among sorted masks
    return Hs[np.ix_(pos, pos)]


def sector_hamiltonian_sparse(h1e, eri, n: int, n_alpha: int, n_beta: int):
    """H as a scipy CSR matrix, rows from the Slater--Condon lists of every basis state."""
    import scipy.sparse as sp
    occ = sector_basis(n, n_alpha, n_beta)
    ints = slater_condon.SpinIntegrals(h1e, eri)
    rows, cols, vals = [], [], []
    for r in range(occ.shape[0]):
        states, _, _, H = slater_condon.connected(occ[r], n, ints)
        rows.append(np.full(states.shape[0], r))
        cols.append(np.array([sector_index(s, n, n_beta) for s in states]))
        vals.append(H)
    dim = occ.shape[0]
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(dim, dim))


def row_apply(h1e, eri, n: int, n_alpha: int, n_beta: int, r: int, v: np.ndarray) -> float:
    """(H v)[r] from row r's Slater--Condon list alone (for spot checks of big sectors)."""
    occ = np.zeros(2 * n, dtype=np.uint8)
    nb_dim = comb(n, n_beta)
    occ[[2 * p for p in set_unrank(r // nb_dim, n_alpha)]] = 1
    occ[[2 * p + 1 for p in set_unrank(r % nb_dim, n_beta)]] = 1
    states, _, _, H = slater_condon.connected(occ, n, slater_condon.SpinIntegrals(h1e, eri))
    idx = np.array([sector_index(s, n, n_beta) for s in states])
    return float(np.sum(H * v[idx]))


def dipole_apply(d, mu_core: float, n: int, n_alpha: int, n_beta: int, psi: np.ndarray, H_of=None) -> np.ndarray:
    """|alpha> = mu |psi> with mu = -sum_pq d_pq (spin-summed hopping) - mu_core."""
    n_ = n
    D = (H_of or sector_hamiltonian_sparse)(-np.asarray(d, float), np.zeros((n_,) * 4), n, n_alpha, n_beta)
    return D @ psi - mu_core * psi


# ----------------------------------------------------------------------------- KPM
def chebyshev_moments(Hmat, alpha: np.ndarray, n_moments: int, a: float, b: float) -> np.ndarray:
    """Omega_0 .. Omega_{n_moments-1} by the recursion and moment doubling (Methods)."""
    def Ht(v):
        return (Hmat @ v - b * v) / a
    mu = np.zeros(n_moments)
    a0 = np.asarray(alpha, float)
    a1 = Ht(a0)
    mu[0] = a0 @ a0
    if n_moments > 1:
        mu[1] = a1 @ a0
    prev, cur = a0, a1
    n = 1
    while 2 * n < n_moments:
        # cur = alpha_n, prev = alpha_{n-1}
        mu[2 * n] = 2.0 * (cur @ cur) - mu[0]
        nxt = 2.0 * Ht(cur) - prev
        if 2 * n + 1 < n_moments:
            mu[2 * n + 1] = 2.0 * (nxt @ cur) - mu[1]
        prev, cur = cur, nxt
        n += 1
    return mu


def moments_direct(Hmat, alpha: np.ndarray, n_moments: int, a: float, b: float) -> np.ndarray:
    """Omega_n = <alpha| T_n(H~) |alpha> without doubling (every alpha_n formed)."""
    a0 = np.asarray(alpha, float)
    out = np.zeros(n_moments)
    prev, cur = None, a0
    for k in range(n_moments):
        out[k] = a0 @ cur
        nxt = (Hmat @ cur - b * cur) / a if k == 0 else 2.0 * (Hmat @ cur - b * cur) / a - prev
        prev, cur = cur, nxt
    return out


def jackson(n_moments: int) -> np.ndarray:
    N = n_moments
    n = np.arange(N)
    q = np.pi / (N + 1)
    return ((N - n + 1) * np.cos(q * n) + np.sin(q * n) / np.tan(q)) / (N + 1)


def line_shape(moments: np.ndarray, w: np.ndarray, kernel: np.ndarray = None) -> np.ndarray:
    """rho(w~) from the moments (Jackson-damped unless a kernel is given)."""
    mu = np.asarray(moments, float)
    g = jackson(mu.size) if kernel is None else kernel
    w = np.asarray(w, float)
    T = np.cos(np.outer(np.arange(mu.size), np.arccos(w)))        # [N, points]
    s = g[0] * mu[0] + 2.0 * (g[1:, None] * mu[1:, None] * T[1:]).sum(axis=0)
    return s / (np.pi * np.sqrt(1.0 - w * w))
