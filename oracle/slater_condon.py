"""Connected determinants and Hamiltonian matrix elements (oracle B).

The local energy (Results, "GPU-supported local energy calculation", eq. for
l_theta(x) and Algorithm 1) sums H_{x x'} psi(x')/psi(x) over every x' coupled to x.
In the occupation basis the Hamiltonian of the Methods section couples x only to x
itself and to its single and double excitations; this module lists them in one
fixed (canonical) order and evaluates the matrix elements with the Slater--Condon
rules of the textbook the paper cites for the basics (Szabo & Ostlund), written
with spin-orbital integrals:

    diagonal        sum_k h_kk + 1/2 sum_{k,l} [(kk|ll) - (kl|lk)]        k,l occupied
    single i -> a   h_ai + sum_k [(ai|kk) - (ak|ki)]                         k occupied
    double ij -> ab (ai|bj) - (aj|bi)

where a spin-orbital integral vanishes unless the spins pair up as in (same|same).
Signs are *not* taken from a formula: each entry's determinant is produced by
applying the operators a_i, a_j, a+_b, a+_a (right to left) one at a time, with the
Jordan--Wigner sign (-1)^{#occupied below} at each step (same conventions as
``oracle.fock``), so  H_{x' x} = <x'| a+_a a+_b a_j a_i |x> * value.

Canonical order (this order is part of the contract with the HIP library):
  0. the diagonal entry;
  1. alpha singles: i over occupied alpha (ascending, outer), a over virtual alpha;
  2. beta singles, same order;
  3. alpha-alpha doubles: occupied pairs i<j (lexicographic, outer) x virtual pairs a<b;
  4. beta-beta doubles, same order;
  5. alpha-beta doubles: (i,a) in alpha-single order (outer) x (j,b) in beta-single order.
Indices in the excitation code are spin-orbitals k = 2p + s; unused slots are 0xFF.
"""
from __future__ import annotations

import itertools
import math

import numpy as np


# ----------------------------------------------------------------------------- bit layout
def unpack(x_words: np.ndarray, n: int) -> np.ndarray:
    """[B, W] uint64 words -> [B, 2n] uint8; spin-orbital k is bit k%64 of word k//64."""
    x = np.asarray(x_words, dtype=np.uint64).reshape(-1, (2 * n + 63) // 64)
    occ = np.zeros((x.shape[0], 2 * n), dtype=np.uint8)
    for k in range(2 * n):
        occ[:, k] = (x[:, k // 64] >> np.uint64(k % 64)) & np.uint64(1)
    return occ


def pack(occ: np.ndarray) -> np.ndarray:
    occ = np.asarray(occ, dtype=np.uint64)
    lead = occ.shape[:-1]
    N = occ.shape[-1]
    W = (N + 63) // 64
    out = np.zeros(lead + (W,), dtype=np.uint64)
    for k in range(N):
        out[..., k // 64] |= occ[..., k] << np.uint64(k % 64)
    return out


def num_connected(n: int, n_alpha: int, n_beta: int) -> int:
    """Closed-form size of the canonical list (diagonal + singles + doubles)."""
    va, vb = n - n_alpha, n - n_beta
    return (1 + n_alpha * va + n_beta * vb
            + math.comb(n_alpha, 2) * math.comb(va, 2)
            + math.comb(n_beta, 2) * math.comb(vb, 2)
            + n_alpha * va * n_beta * vb)


# ----------------------------------------------------------------------------- excitations
def excitation_list(occ: np.ndarray, n: int) -> np.ndarray:
    """Canonical [C, 4] int array of (i, j, a, b) spin-orbitals; -1 marks an unused slot."""
    occ_s = [np.array([p for p in range(n) if occ[2 * p + s]], dtype=np.int64) for s in (0, 1)]
    vir_s = [np.array([p for p in range(n) if not occ[2 * p + s]], dtype=np.int64) for s in (0, 1)]
    blocks = [np.array([[-1, -1, -1, -1]], dtype=np.int64)]
    singles = []
    for s in (0, 1):
        I, A = np.meshgrid(occ_s[s], vir_s[s], indexing="ij")
        i, a = 2 * I.ravel() + s, 2 * A.ravel() + s
        singles.append((i, a))
        neg = -np.ones_like(i)
        blocks.append(np.stack([i, neg, a, neg], axis=1))
    for s in (0, 1):
        po = np.array(list(itertools.combinations(occ_s[s].tolist(), 2)), dtype=np.int64).reshape(-1, 2)
        pv = np.array(list(itertools.combinations(vir_s[s].tolist(), 2)), dtype=np.int64).reshape(-1, 2)
        O = np.repeat(po, pv.shape[0], axis=0)
        V = np.tile(pv, (po.shape[0], 1))
        blocks.append(np.stack([2 * O[:, 0] + s, 2 * O[:, 1] + s, 2 * V[:, 0] + s, 2 * V[:, 1] + s], axis=1))
    (ia, aa), (ib, ab) = singles
    i = np.repeat(ia, ib.size)
    a = np.repeat(aa, ib.size)
    j = np.tile(ib, ia.size)
    b = np.tile(ab, ia.size)
    blocks.append(np.stack([i, j, a, b], axis=1))
    return np.concatenate(blocks, axis=0)


def _apply(states: np.ndarray, signs: np.ndarray, k: np.ndarray, creation: bool) -> None:
    """Apply a+_k (creation) or a_k to each row in place, with the Jordan--Wigner sign."""
    rows = np.nonzero(k >= 0)[0]
    if rows.size == 0:
        return
    kk = k[rows]
    before = states[rows, kk]
    expect = 0 if creation else 1
    if np.any(before != expect):
        raise AssertionError("operator annihilates the determinant")
    below = (np.cumsum(states[rows], axis=1, dtype=np.int64) - states[rows])[np.arange(rows.size), kk]
    signs[rows] *= 1 - 2 * (below & 1)
    states[rows, kk] ^= 1


def apply_excitations(occ: np.ndarray, exc: np.ndarray):
    """States a+_a a+_b a_j a_i |x> for each excitation row, and their signs."""
    C = exc.shape[0]
    states = np.repeat(occ[None, :].astype(np.uint8), C, axis=0)
    signs = np.ones(C, dtype=np.int64)
    _apply(states, signs, exc[:, 0], creation=False)   # a_i
    _apply(states, signs, exc[:, 1], creation=False)   # a_j
    _apply(states, signs, exc[:, 3], creation=True)    # a+_b
    _apply(states, signs, exc[:, 2], creation=True)    # a+_a
    return states, signs


# ----------------------------------------------------------------------------- values
class SpinIntegrals:
    """Spin-orbital integrals from spatial ones: zero unless the spins pair up."""

    def __init__(self, h1e: np.ndarray, eri: np.ndarray):
        self.h1e = np.asarray(h1e, dtype=np.float64)
        self.eri = np.asarray(eri, dtype=np.float64)

    def h(self, k, l):
        k, l = np.asarray(k), np.asarray(l)
        return self.h1e[k // 2, l // 2] * ((k % 2) == (l % 2))

    def g(self, k, l, m, o):
        """(kl|mo) for spin-orbitals."""
        k, l, m, o = (np.asarray(v) for v in (k, l, m, o))
        same = ((k % 2) == (l % 2)) & ((m % 2) == (o % 2))
        return self.eri[k // 2, l // 2, m // 2, o // 2] * same


def matrix_elements(occ: np.ndarray, exc: np.ndarray, ints: SpinIntegrals) -> np.ndarray:
    """Slater--Condon value of each entry, before the operator sign."""
    K = np.nonzero(occ)[0]
    i, j, a, b = exc.T
    diag = (i < 0)
    single = (i >= 0) & (j < 0)
    double = (j >= 0)
    val = np.zeros(exc.shape[0])
    kk, ll = np.meshgrid(K, K, indexing="ij")
    e_diag = ints.h(K, K).sum() + 0.5 * (ints.g(kk, kk, ll, ll) - ints.g(kk, ll, ll, kk)).sum()
    val[diag] = e_diag
    if np.any(single):
        si, sa = i[single][:, None], a[single][:, None]
        Kb = K[None, :]
        val[single] = ints.h(sa[:, 0], si[:, 0]) + (ints.g(sa, si, Kb, Kb) - ints.g(sa, Kb, Kb, si)).sum(axis=1)
    if np.any(double):
        di, dj, da, db = i[double], j[double], a[double], b[double]
        val[double] = ints.g(da, di, db, dj) - ints.g(da, dj, db, di)
    return val


def connected(occ: np.ndarray, n: int, ints: SpinIntegrals):
    """For one determinant (uint8[2n]): (states [C,2n], signs [C], exc [C,4], H [C])."""
    exc = excitation_list(occ, n)
    states, signs = apply_excitations(occ, exc)
    H = signs * matrix_elements(occ, exc, ints)
    return states, signs, exc, H


def encode_exc(exc: np.ndarray) -> np.ndarray:
    """(i, j, a, b) with -1 unused -> uint32 i | j<<8 | a<<16 | b<<24, unused = 0xFF."""
    e = np.where(exc < 0, 0xFF, exc).astype(np.uint64)
    return (e[:, 0] | (e[:, 1] << np.uint64(8)) | (e[:, 2] << np.uint64(16)) | (e[:, 3] << np.uint64(24))).astype(np.uint32)


def connect(x_words: np.ndarray, n: int, n_alpha: int, n_beta: int, h1e, eri):
    """Materialised lists for a batch: xp [B,C,W] uint64, H [B,C], sign [B,C] int8, exc [B,C] uint32."""
    occ_all = unpack(x_words, n)
    ints = SpinIntegrals(h1e, eri)
    C = num_connected(n, n_alpha, n_beta)
    B = occ_all.shape[0]
    W = (2 * n + 63) // 64
    xp = np.zeros((B, C, W), dtype=np.uint64)
    hv = np.zeros((B, C))
    sg = np.zeros((B, C), dtype=np.int8)
    ex = np.zeros((B, C), dtype=np.uint32)
    for bi in range(B):
        states, signs, exc, H = connected(occ_all[bi], n, ints)
        if states.shape[0] != C:
            raise AssertionError("sample is not in the (n_alpha, n_beta) sector")
        xp[bi] = pack(states)
        hv[bi] = H
        sg[bi] = signs
        ex[bi] = encode_exc(exc)
    return xp, hv, sg, ex
