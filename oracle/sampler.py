"""Batch autoregressive sampling (BAS) of the ansatz, in FP64 (test infrastructure).

Follows the Results description of BAS: the N_s samples are carried as a tree of unique
prefixes with multiplicities; at orbital k every unique prefix x_<k with weight w splits
w among its children by one multinomial draw from the (number-conserving, renormalised)
conditional of orbital k, children with no draws are pruned, and after the last orbital
the leaves are the unique samples with their counts. The cost of a step depends on the
number of unique prefixes, not on N_s.

Readings fixed here (the paper leaves them open):

* the multinomial split of w over the feasible states s_1 < s_2 < ... (0 = empty,
  1 = alpha, 2 = beta, 3 = both; feasible: probability > 0) is a chain of binomials: state
  s_j gets c_j ~ Binomial(w - c_1 - ... - c_{j-1}, p_{s_j} / (p_{s_j} + p_{s_{j+1}} + ...)),
  the sums taken in ascending state order, and the last feasible state gets the rest;
* a binomial variate Binomial(n, p) uses p' = min(p, 1 - p) and returns n - K when p > 1/2;
  with n p' < 10 it is drawn by inversion (sequential search from K = 0 with the pmf
  recursion f(K) = f(K - 1) ((n + 1) s / K - s), s = p' / (1 - p'), f(0) = exp(n log1p(-p'))),
  otherwise by the transformed rejection with decomposition BTRD (W. Hormann, "The
  generation of binomial random variates", J. Stat. Comput. Simul. 46, 1993) with its
  constants and its Stirling correction f_c;
* the uniforms of attempt t of the binomial of state s of prefix i at orbital k are the
  two 53-bit halves of one Philox4x32-10 output (Salmon et al., "Parallel random numbers:
  as easy as 1, 2, 3", SC 2011) at counter (t, i, k, s) and key (seed low word, seed high
  word): u_1 = ((w0 << 32 | w1) >> 11) 2^-53, u_2 = ((w2 << 32 | w3) >> 11) 2^-53; an
  inversion that runs past the last representable pmf term restarts at the next attempt;
* prefixes are kept in the order (parent index, state), so the tree's indices, and with
  them the random stream, are fixed by the seed.

Nothing here is shared with the HIP library.
"""
from __future__ import annotations

import math

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


def uniform_pair(t: int, i: int, k: int, st: int, seed: int):
    """(u_1, u_2) of attempt t, prefix i, orbital k, state st."""
    ctr = np.array([[t, i, k, st]], dtype=np.uint32)
    key = np.array([[seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF]], dtype=np.uint32)
    w = [int(v) for v in philox4x32_10(ctr, key)[0]]
    u1 = (((w[0] << 32) | w[1]) >> 11) * 2.0 ** -53
    u2 = (((w[2] << 32) | w[3]) >> 11) * 2.0 ** -53
    return u1, u2


def stirling_fc(k: int) -> float:
    """f_c(k) = ln k! - (k + 1/2) ln(k + 1) + (k + 1) - ln(2 pi) / 2, the Stirling-series
    correction of BTRD: from the definition (lgamma) for k < 10, from the series
    1/12 - 1/360 (k+1)^-2 + 1/1260 (k+1)^-4 over (k + 1) above."""
    if k < 10:
        return math.lgamma(k + 1.0) - (k + 0.5) * math.log(k + 1.0) + (k + 1.0) - 0.5 * math.log(2.0 * math.pi)
    kk = 1.0 / ((k + 1.0) * (k + 1.0))
    return (1.0 / 12.0 - (1.0 / 360.0 - 1.0 / 1260.0 * kk) * kk) / (k + 1.0)


def binomial(n: int, p: float, pair) -> int:
    """One Binomial(n, p) variate; pair(t) gives the two uniforms of attempt t."""
    if n <= 0 or p <= 0.0:
        return 0
    if p >= 1.0:
        return n
    flip = p > 0.5
    pp = 1.0 - p if flip else p
    k = _binomial_small_p(n, pp, pair)
    return n - k if flip else k


def _binomial_small_p(n: int, p: float, pair) -> int:
    nf = float(n)
    if nf * p < 10.0:
        # inversion: walk the pmf from K = 0
        s = p / (1.0 - p)
        a = (nf + 1.0) * s
        f0 = math.exp(nf * math.log1p(-p))
        t = 0
        while True:
            u, _ = pair(t)
            t += 1
            f = f0
            kk = 0
            while u > f:
                u -= f
                kk += 1
                f *= a / kk - s
                if f <= 0.0 or kk > n:
                    break
            if u <= f and kk <= n:
                return kk
    # BTRD
    m = math.floor((nf + 1.0) * p)
    r = p / (1.0 - p)
    nr = (nf + 1.0) * r
    npq = nf * p * (1.0 - p)
    spq = math.sqrt(npq)
    b = 1.15 + 2.53 * spq
    a = -0.0873 + 0.0248 * b + 0.01 * p
    c = nf * p + 0.5
    alpha = (2.83 + 5.1 / b) * spq
    vr = 0.92 - 4.2 / b
    urvr = 0.86 * vr
    t = 0
    while True:
        v, u2 = pair(t)
        t += 1
        if v <= urvr:
            u = v / vr - 0.43
            kf = math.floor((2.0 * a / (0.5 - abs(u)) + b) * u + c)
            if 0.0 <= kf <= nf:
                return int(kf)
            continue
        if v >= vr:
            u = u2 - 0.5
        else:
            u = v / vr - 0.93
            u = (0.5 if u > 0.0 else -0.5) - u
            v = u2 * vr
        us = 0.5 - abs(u)
        kf = math.floor((2.0 * a / us + b) * u + c)
        if kf < 0.0 or kf > nf:
            continue
        k = int(kf)
        v = v * alpha / (a / (us * us) + b)
        km = abs(k - m)
        if km <= 15:
            f = 1.0
            if m < k:
                for i in range(int(m) + 1, k + 1):
                    f *= nr / i - r
            elif m > k:
                for i in range(k + 1, int(m) + 1):
                    v *= nr / i - r
            if v <= f:
                return k
            continue
        v = math.log(v)
        rho = (km / npq) * (((km / 3.0 + 0.625) * km + 1.0 / 6.0) / npq + 0.5)
        tt = -km * km / (2.0 * npq)
        if v < tt - rho:
            return k
        if v > tt + rho:
            continue
        nm = nf - m + 1.0
        h = (m + 0.5) * math.log((m + 1.0) / (r * nm)) + stirling_fc(int(m)) + stirling_fc(int(n - m))
        nk = nf - k + 1.0
        if v <= h + (nf + 1.0) * math.log(nm / nk) + (k + 0.5) * math.log(nk * r / (k + 1.0)) \
                - stirling_fc(k) - stirling_fc(n - k):
            return k


def multinomial_split(w: int, p, pair_of_state):
    """Counts [4] of w over the states with probabilities p [4] (a chain of binomials over
    the feasible states in ascending order; the last feasible state takes the rest)."""
    feas = [s for s in range(4) if p[s] > 0.0]
    out = [0, 0, 0, 0]
    if not feas:
        return out
    left = int(w)
    for j, s in enumerate(feas[:-1]):
        rem = 0.0
        for q in feas[j:]:
            rem = rem + p[q]
        c = binomial(left, min(1.0, p[s] / rem), pair_of_state(s))
        out[s] = c
        left -= c
    out[feas[-1]] = left
    return out


def bas(theta, n: int, n_alpha: int, n_beta: int, widths, n_samples: int, seed: int):
    """(unique samples as occupations [U, 2n] uint8, counts [U] int64) in tree order."""
    prefixes = np.zeros((1, 2 * n), dtype=np.uint8)
    weights = [int(n_samples)]
    for k in range(n):
        f = made.forward(theta, prefixes, n, n_alpha, n_beta, widths, keep=True)
        probs = np.where(f["ok"][:, k, :], np.exp(f["logp"][:, k, :]), 0.0)   # [U, 4]
        children, counts = [], []
        for i in range(prefixes.shape[0]):
            split = multinomial_split(weights[i], [float(v) for v in probs[i]],
                                      lambda st, i=i: (lambda t: uniform_pair(t, i, k, st, seed)))
            for s in range(4):
                if split[s] > 0:
                    ch = prefixes[i].copy()
                    ch[2 * k] = s & 1
                    ch[2 * k + 1] = s >> 1
                    children.append(ch)
                    counts.append(split[s])
        prefixes = np.array(children, dtype=np.uint8)
        weights = counts
    return prefixes, np.array(weights, dtype=np.int64)
