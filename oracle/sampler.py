"""Batch autoregressive sampling (BAS) of the ansatz, in FP64 (test infrastructure).

Follows the Methods/Results description of BAS: the N_s samples are carried as a tree of
unique prefixes with multiplicities; at orbital k every unique prefix x_<k with weight w
draws its w children from the (number-conserving, renormalised) conditional of orbital
k, children with no draws are pruned, and after the last orbital the leaves are the
unique samples with their counts.

Readings fixed here (the paper leaves them open):

* the w draws of a prefix are w independent categorical draws (an exact multinomial
  split), each from one uniform u in [0, 1): the category is the first feasible state s
  (in the order 0 = empty, 1 = alpha, 2 = beta, 3 = both) whose running sum of
  probabilities exceeds u, else the last feasible state;
* the uniform of draw j of prefix i at orbital k is the first 53 bits of the first two
  words of Philox4x32-10 (Salmon et al., "Parallel random numbers: as easy as 1, 2, 3",
  SC 2011) at counter (j, i, k, 0) and key (seed low word, seed high word):
  u = ((w0 << 32 | w1) >> 11) 2^-53;
* prefixes are kept in the order (parent index, state), so the tree's indices, and
  with them the random stream, are fixed by the seed.

Nothing here is shared with the HIP library.
"""
from __future__ import annotations

import numpy as np

from . import made

_M0, _M1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
_W0, _W1 = np.uint32(0x9E3779B9), np.uint32(0xBB67AE85)
_MASK32 = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr, key):
    """Philox4x32 with 10 rounds. ctr: uint32 [..., 4], key: uint32 [..., 2] -> uint32 [..., 4]."""
    c = [np.asarray(ctr[..., i], dtype=np.uint32) for i in range(4)]
    k0 = np.asarray(key[..., 0], dtype=np.uint32)
    k1 = np.asarray(key[..., 1], dtype=np.uint32)
    for r in range(10):
        p0 = c[0].astype(np.uint64) * _M0
        p1 = c[2].astype(np.uint64) * _M1
        hi0, lo0 = (p0 >> np.uint64(32)).astype(np.uint32), (p0 & _MASK32).astype(np.uint32)
        hi1, lo1 = (p1 >> np.uint64(32)).astype(np.uint32), (p1 & _MASK32).astype(np.uint32)
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
        if r < 9:
            k0 = (k0 + _W0).astype(np.uint32)
            k1 = (k1 + _W1).astype(np.uint32)
    return np.stack(c, axis=-1)


def uniforms(j, i, k, seed: int) -> np.ndarray:
    """u in [0, 1) for draws j (array) of prefix i at orbital k."""
    j = np.asarray(j, dtype=np.uint32)
    ctr = np.zeros(j.shape + (4,), dtype=np.uint32)
    ctr[..., 0] = j
    ctr[..., 1] = np.uint32(i)
    ctr[..., 2] = np.uint32(k)
    key = np.zeros(j.shape + (2,), dtype=np.uint32)
    key[..., 0] = np.uint32(seed & 0xFFFFFFFF)
    key[..., 1] = np.uint32((seed >> 32) & 0xFFFFFFFF)
    w = philox4x32_10(ctr, key).astype(np.uint64)
    bits = ((w[..., 0] << np.uint64(32)) | w[..., 1]) >> np.uint64(11)
    return bits.astype(np.float64) * (2.0 ** -53)


def categories(u: np.ndarray, p: np.ndarray) -> np.ndarray:
    """First feasible state whose running probability sum exceeds u, else the last feasible."""
    run = 0.0
    out = np.full(u.shape, -1, dtype=np.int64)
    last = -1
    for s in range(4):
        if p[s] > 0.0:
            run = run + p[s]
            out[(out < 0) & (u < run)] = s
            last = s
    out[out < 0] = last
    return out


def bas(theta, n: int, n_alpha: int, n_beta: int, widths, n_samples: int, seed: int):
    """(unique samples as occupations [U, 2n] uint8, counts [U] int64) in tree order."""
    prefixes = np.zeros((1, 2 * n), dtype=np.uint8)
    weights = np.array([n_samples], dtype=np.int64)
    for k in range(n):
        f = made.forward(theta, prefixes, n, n_alpha, n_beta, widths, keep=True)
        probs = np.where(f["ok"][:, k, :], np.exp(f["logp"][:, k, :]), 0.0)   # [U, 4]
        children, counts = [], []
        for i in range(prefixes.shape[0]):
            u = uniforms(np.arange(weights[i]), i, k, seed)
            cat = categories(u, probs[i])
            c = np.bincount(cat, minlength=4)
            for s in range(4):
                if c[s] > 0:
                    ch = prefixes[i].copy()
                    ch[2 * k] = s & 1
                    ch[2 * k + 1] = s >> 1
                    children.append(ch)
                    counts.append(c[s])
        prefixes = np.array(children, dtype=np.uint8)
        weights = np.array(counts, dtype=np.int64)
    return prefixes, weights
