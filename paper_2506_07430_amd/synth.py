"""Seeded synthetic inputs for the local-energy path.

This module only *draws* inputs; it holds none of the method's arithmetic. The
same arrays go, unchanged, to the HIP library and to the CPU checker, which each
apply the ansatz masks, the Slater--Condon rules and the energy formulas on their
own.

What is drawn (the paper's molecules, integrals and trained weights are not
available, so these stand in for them):

* one-body integrals ``h1e[n, n]``: symmetric, diagonal ~ N(-2, 0.5), off-diagonal
  ~ N(0, 0.1), optionally damped by ``exp(-|p-q| / decay)`` to imitate the
  distance-decaying couplings of a chain;
* two-electron integrals ``eri[n, n, n, n]`` in chemists' order ``(pq|rs)``, built
  as ``sum_k L_k[p,q] L_k[r,s]`` from random symmetric matrices
  ``L_k = 0.1 (G + G^T) / 2`` (damped like ``h1e``), so the tensor is positive
  semidefinite, low rank and exactly 8-fold symmetric (each entry is summed in
  the same order);
* a flat vector of ansatz parameters, every entry ~ N(0, 0.1), *without* the
  autoregressive mask applied (the consumer applies the mask);
* unique occupation bitstrings with fixed alpha/beta electron counts, packed as
  ``W = ceil(2n / 64)`` little-endian uint64 words with spin-orbital ``k = 2p + s``
  (s = 0 alpha, 1 beta) at bit ``k % 64`` of word ``k // 64``, sorted ascending as
  multi-word integers;
* integer sample multiplicities (all ones, or Zipf(1.5)).

Seeds: ``numpy.random.default_rng([250607430, cfg, stream, system])``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

SEED_ROOT = 250607430
STREAM_H1E, STREAM_ERI, STREAM_PARAMS, STREAM_SAMPLES, STREAM_MULT, STREAM_FD, STREAM_DIPOLE = range(7)


def rng(cfg: int, stream: int, system: int = 0) -> np.random.Generator:
    return np.random.default_rng([SEED_ROOT, cfg, stream, system])


@dataclasses.dataclass(frozen=True)
class System:
    """One molecule-like problem: orbitals, electrons, ansatz widths, integral recipe."""
    n: int                      # spatial orbitals
    n_alpha: int
    n_beta: int
    widths: tuple               # hidden-layer widths of the autoregressive ansatz
    n_chol: int = 16            # number of random symmetric factors in eri
    decay: Optional[float] = None  # damping length of off-diagonal couplings

    @property
    def words(self) -> int:
        return (2 * self.n + 63) // 64


@dataclasses.dataclass(frozen=True)
class Workload:
    cfg: int
    name: str
    systems: tuple
    samples: tuple              # unique samples per system
    multiplicity: str           # "ones" or "zipf1.5"
    precision: str              # "fp64" or "bf16"
    grad: bool


WORKLOADS = {
    0: Workload(0, "n8_a4b4_h32", (System(8, 4, 4, (32,), 16, None),), (1024,), "ones", "fp64", True),
    1: Workload(1, "n24_a12b12_h128x2_zipf", (System(24, 12, 12, (128, 128), 16, 6.0),), (16384,),
                "zipf1.5", "bf16", True),
    2: None,  # filled below (sample counts are seeded)
    3: Workload(3, "n40_a14b14_h256x3", (System(40, 14, 14, (256, 256, 256), 16, 6.0),), (8192,),
                "ones", "bf16", True),
    4: Workload(4, "n60_a26b26_h256x3", (System(60, 26, 26, (256, 256, 256), 60, 8.0),), (1024,),
                "ones", "bf16", True),
}


def _multi_system_workload() -> Workload:
    g = rng(2, STREAM_MULT)
    counts = tuple(int(c) for c in g.integers(2048, 8193, size=8))
    systems = tuple(System(n, n // 2, n // 2, (128, 128), 16, 6.0) for n in range(12, 41, 4))
    return Workload(2, "8sys_n12-40_half_h128x2", systems, counts, "ones", "bf16", False)


WORKLOADS[2] = _multi_system_workload()


# ----------------------------------------------------------------------------- integrals
def make_h1e(sys: System, cfg: int, system_index: int = 0) -> np.ndarray:
    n = sys.n
    g = rng(cfg, STREAM_H1E, system_index)
    h = np.zeros((n, n))
    h[np.diag_indices(n)] = g.normal(-2.0, 0.5, n)
    iu = np.triu_indices(n, 1)
    off = g.normal(0.0, 0.1, iu[0].size)
    if sys.decay is not None:
        off = off * np.exp(-np.abs(iu[0] - iu[1]) / sys.decay)
    h[iu] = off
    h[(iu[1], iu[0])] = off
    return h


def make_eri(sys: System, cfg: int, system_index: int = 0) -> np.ndarray:
    n = sys.n
    g = rng(cfg, STREAM_ERI, system_index)
    damp = None
    if sys.decay is not None:
        idx = np.arange(n)
        damp = np.exp(-np.abs(idx[:, None] - idx[None, :]) / sys.decay)
    eri = np.zeros((n, n, n, n))
    for _ in range(sys.n_chol):
        G = g.standard_normal((n, n))
        L = 0.1 * (G + G.T) / 2.0
        if damp is not None:
            L = L * damp
        eri += np.multiply.outer(L, L)
    return eri


# ----------------------------------------------------------------------------- parameters
def make_dipole(n: int, seed: int) -> np.ndarray:
    """Synthetic dipole integrals d_pq (one Cartesian component), symmetric: a chain-like
    position on the diagonal, (p - (n - 1) / 2) / 2, plus N(0, 0.05) couplings damped by
    exp(-|p - q|) (molecular dipole integrals are not available)."""
    g = rng(seed, STREAM_DIPOLE)
    d = np.diag((np.arange(n) - (n - 1) / 2.0) / 2.0)
    iu = np.triu_indices(n, 1)
    off = g.normal(0.0, 0.05, iu[0].size) * np.exp(-np.abs(iu[0] - iu[1]))
    d[iu] = off
    d[(iu[1], iu[0])] = off
    return d


def num_params(n: int, widths: Sequence[int]) -> int:
    """Length of the flat parameter vector (layout documented in include/elocal.h)."""
    dims = [2 * n] + list(widths) + [4 * n]
    p = sum(dims[l + 1] * dims[l] + dims[l + 1] for l in range(len(dims) - 1))
    return p + widths[-1] + 1


def make_params(sys: System, cfg: int, system_index: int = 0) -> np.ndarray:
    g = rng(cfg, STREAM_PARAMS, system_index)
    return g.normal(0.0, 0.1, num_params(sys.n, sys.widths))


# ----------------------------------------------------------------------------- bitstrings
def pack_occupations(occ: np.ndarray) -> np.ndarray:
    """occ: [B, 2n] 0/1 array in spin-orbital order -> [B, W] uint64 words."""
    occ = np.asarray(occ, dtype=np.uint64)
    B, N = occ.shape
    W = (N + 63) // 64
    out = np.zeros((B, W), dtype=np.uint64)
    for k in range(N):
        out[:, k // 64] |= occ[:, k] << np.uint64(k % 64)
    return out


def unpack_words(x: np.ndarray, n_spin_orbitals: int) -> np.ndarray:
    """[B, W] uint64 -> [B, 2n] uint8 occupations."""
    x = np.asarray(x, dtype=np.uint64)
    out = np.zeros((x.shape[0], n_spin_orbitals), dtype=np.uint8)
    for k in range(n_spin_orbitals):
        out[:, k] = ((x[:, k // 64] >> np.uint64(k % 64)) & np.uint64(1)).astype(np.uint8)
    return out


def sort_unique_words(x: np.ndarray) -> np.ndarray:
    """Unique rows of a [B, W] word array, ascending as multi-word integers."""
    x = np.ascontiguousarray(x, dtype=np.uint64)
    key = x[:, ::-1]                      # most significant word first
    u = np.unique(key, axis=0)
    return u[:, ::-1].copy()


def uniform_determinants(sys: System, count: int, g: np.random.Generator) -> np.ndarray:
    """`count` distinct determinants drawn uniformly from the (n_alpha, n_beta) sector."""
    n = sys.n
    total = math.comb(n, sys.n_alpha) * math.comb(n, sys.n_beta)
    if count > total:
        raise ValueError(f"asked for {count} unique determinants, sector has {total}")
    have = np.zeros((0, sys.words), dtype=np.uint64)
    while have.shape[0] < count:
        m = max(2 * (count - have.shape[0]), 64)
        occ = np.zeros((m, 2 * n), dtype=np.uint8)
        for spin, ne in ((0, sys.n_alpha), (1, sys.n_beta)):
            keys = g.random((m, n))
            chosen = np.argsort(keys, axis=1)[:, :ne]
            rows = np.repeat(np.arange(m), ne)
            occ[rows, 2 * chosen.ravel() + spin] = 1
        have = sort_unique_words(np.concatenate([have, pack_occupations(occ)]))
    # keep a seeded random subset of the right size, then sort
    pick = g.choice(have.shape[0], size=count, replace=False)
    return sort_unique_words(have[pick])


def multiplicities(kind: str, count: int, g: np.random.Generator) -> np.ndarray:
    if kind == "ones":
        return np.ones(count)
    if kind == "zipf1.5":
        return g.zipf(1.5, count).astype(np.int64).astype(np.float64)
    raise ValueError(kind)


@dataclasses.dataclass
class Problem:
    system: System
    h1e: np.ndarray
    eri: np.ndarray
    theta: np.ndarray
    x: np.ndarray        # [B, W] uint64
    w: np.ndarray        # [B] float64


def make_problem(cfg: int, system_index: int = 0, samples: Optional[int] = None,
                 x: Optional[np.ndarray] = None) -> Problem:
    """Integrals, raw parameters, uniformly drawn determinants and multiplicities.

    ``samples`` overrides the workload's count; ``x`` replaces the drawn
    determinants (e.g. by determinants drawn from the ansatz in the tests).
    """
    wl = WORKLOADS[cfg]
    sys = wl.systems[system_index]
    h1e = make_h1e(sys, cfg, system_index)
    eri = make_eri(sys, cfg, system_index)
    theta = make_params(sys, cfg, system_index)
    count = wl.samples[system_index] if samples is None else samples
    if x is None:
        x = uniform_determinants(sys, count, rng(cfg, STREAM_SAMPLES, system_index))
    w = multiplicities(wl.multiplicity, x.shape[0], rng(cfg, STREAM_MULT, 100 + system_index))
    return Problem(sys, h1e, eri, theta, x, w)


def random_problem(n: int, n_alpha: int, n_beta: int, widths: Sequence[int], seed: int,
                   n_chol: int = 8, decay: Optional[float] = None, samples: int = 64,
                   multiplicity: str = "ones") -> Problem:
    """Small ad-hoc problem for edge-case tests (seeded by `seed`)."""
    sys = System(n, n_alpha, n_beta, tuple(widths), n_chol, decay)
    cfg = 1000 + seed
    h1e = make_h1e(sys, cfg)
    eri = make_eri(sys, cfg)
    theta = make_params(sys, cfg)
    total = math.comb(n, n_alpha) * math.comb(n, n_beta)
    x = uniform_determinants(sys, min(samples, total), rng(cfg, STREAM_SAMPLES))
    w = multiplicities(multiplicity, x.shape[0], rng(cfg, STREAM_MULT))
    return Problem(sys, h1e, eri, theta, x, w)


def full_sector(sys: System) -> np.ndarray:
    """Every determinant of the (n_alpha, n_beta) sector, packed and sorted."""
    import itertools
    n = sys.n
    rows: List[np.ndarray] = []
    for a in itertools.combinations(range(n), sys.n_alpha):
        for b in itertools.combinations(range(n), sys.n_beta):
            occ = np.zeros(2 * n, dtype=np.uint8)
            occ[[2 * p for p in a]] = 1
            occ[[2 * p + 1 for p in b]] = 1
            rows.append(occ)
    if not rows:
        return np.zeros((0, sys.words), dtype=np.uint64)
    return sort_unique_words(pack_occupations(np.stack(rows)))
