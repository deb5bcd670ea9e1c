"""Autoregressive amplitude/phase ansatz in FP64 (Results: "Neural-network wavefunction
ansatz", Fig. 1b; "Parallel sampling" for the number-conserving conditionals).

Psi(x) = pi(x) e^{i phi(x)}: a masked dense network (MADE) gives, for each spatial
orbital p in order, a distribution over its four occupations s_p = x_{2p} + 2 x_{2p+1}
(empty, up, down, both) conditioned on the orbitals before it; a sigmoid head on the
same trunk gives the phase in [0, 2 pi).

Readings fixed here (the paper does not spell them out):

* the pi_k of the paper are conditional probabilities, so |Psi(x)|^2 = prod_p p_p(s_p)
  and A(x) = log|Psi(x)| = 1/2 sum_p log p_p(s_p) (Psi is then normalised);
* degrees: input bit k has degree k//2 + 1 (its orbital, 1-based); hidden unit j of
  every hidden layer has degree (j mod (n-1)) + 1; input->hidden allowed iff
  m_hidden >= d_input, hidden->hidden iff m_out >= m_in, hidden->output of orbital p
  (0-based) iff m_hidden < p + 1; the phase head sees the whole last hidden layer;
* ReLU after every hidden layer; raw parameters outside the mask are ignored
  (treated as zero);
* the number constraint removes an occupation s of orbital p unless, for both spins,
  the count so far plus s_sigma stays <= N_sigma *and* can still reach N_sigma with the
  n - p - 1 orbitals left; the remaining logits are renormalised by a softmax;
* phi = 2 pi sigmoid(w_phi . h_last + b_phi).

Flat parameter layout: for each layer l = 0..L (L hidden layers, then the output
layer of 4n logits ordered [orbital][state]) the weight W_l[out][in] row-major then
the bias b_l[out]; then w_phi[h_L] and b_phi[1].
"""
from __future__ import annotations

import numpy as np


def layer_dims(n: int, widths) -> list:
    return [2 * n] + list(widths) + [4 * n]


def num_params(n: int, widths) -> int:
    d = layer_dims(n, widths)
    return sum(d[l + 1] * d[l] + d[l + 1] for l in range(len(d) - 1)) + widths[-1] + 1


def degrees(n: int, widths):
    """(input degrees, [hidden degrees per layer], output degrees)."""
    d_in = np.arange(2 * n) // 2 + 1
    d_hid = [np.arange(w) % (n - 1) + 1 for w in widths]
    d_out = np.arange(4 * n) // 4 + 1
    return d_in, d_hid, d_out


def masks(n: int, widths) -> list:
    """Boolean [out, in] connectivity of every layer (hidden layers, then output)."""
    d_in, d_hid, d_out = degrees(n, widths)
    m = [d_hid[0][:, None] >= d_in[None, :]]
    for l in range(1, len(widths)):
        m.append(d_hid[l][:, None] >= d_hid[l - 1][None, :])
    m.append(d_out[:, None] > d_hid[-1][None, :])
    return m


def unpack_params(theta: np.ndarray, n: int, widths, apply_mask: bool = True):
    """Flat vector -> ([(W_l, b_l)], w_phi, b_phi), with the mask applied."""
    theta = np.asarray(theta, dtype=np.float64)
    d = layer_dims(n, widths)
    mk = masks(n, widths)
    layers, off = [], 0
    for l in range(len(d) - 1):
        W = theta[off:off + d[l + 1] * d[l]].reshape(d[l + 1], d[l]).copy()
        off += d[l + 1] * d[l]
        b = theta[off:off + d[l + 1]].copy()
        off += d[l + 1]
        if apply_mask:
            W = W * mk[l]
        layers.append((W, b))
    w_phi = theta[off:off + widths[-1]].copy()
    off += widths[-1]
    b_phi = float(theta[off])
    off += 1
    if off != theta.size:
        raise ValueError(f"parameter vector has {theta.size} entries, layout needs {off}")
    return layers, w_phi, b_phi


def feasible(occ: np.ndarray, n: int, n_alpha: int, n_beta: int) -> np.ndarray:
    """[M, n, 4] bool: which occupations of orbital p keep the electron counts reachable."""
    occ = np.asarray(occ, dtype=np.int64)
    up, dn = occ[:, 0::2], occ[:, 1::2]
    c_up = np.cumsum(up, axis=1) - up            # electrons before orbital p
    c_dn = np.cumsum(dn, axis=1) - dn
    left = n - np.arange(n) - 1                  # orbitals after p
    s = np.arange(4)
    s_up, s_dn = s & 1, s >> 1
    cu = c_up[:, :, None] + s_up[None, None, :]
    cd = c_dn[:, :, None] + s_dn[None, None, :]
    r = left[None, :, None]
    return (cu <= n_alpha) & (cd <= n_beta) & (cu + r >= n_alpha) & (cd + r >= n_beta)


def forward(theta, occ, n, n_alpha, n_beta, widths, keep=False):
    """A = log|Psi|, phi for each row of occ [M, 2n] (0/1). Returns a dict."""
    layers, w_phi, b_phi = unpack_params(theta, n, widths)
    h = np.asarray(occ, dtype=np.float64)
    hs, zs = [h], []
    for W, b in layers[:-1]:
        z = h @ W.T + b
        h = np.maximum(z, 0.0)
        zs.append(z)
        hs.append(h)
    Wo, bo = layers[-1]
    logits = (h @ Wo.T + bo).reshape(-1, n, 4)
    ok = feasible(occ, n, n_alpha, n_beta)
    masked = np.where(ok, logits, -np.inf)
    any_ok = ok.any(axis=2, keepdims=True)                 # False only past an impossible prefix
    mx = np.where(any_ok, masked.max(axis=2, keepdims=True), 0.0)
    with np.errstate(divide="ignore"):
        lse = mx + np.log(np.exp(masked - mx).sum(axis=2, keepdims=True))
    logp = np.where(ok, logits - lse, -np.inf)             # log-softmax over allowed states
    state = np.asarray(occ, dtype=np.int64)[:, 0::2] + 2 * np.asarray(occ, dtype=np.int64)[:, 1::2]
    logp_x = np.take_along_axis(logp, state[:, :, None], axis=2)[:, :, 0]   # [M, n]
    A = 0.5 * logp_x.sum(axis=1)
    zphi = h @ w_phi + b_phi
    sig = 1.0 / (1.0 + np.exp(-zphi))
    phi = 2.0 * np.pi * sig
    out = dict(A=A, phi=phi, logp_x=logp_x)
    if keep:
        out.update(hs=hs, zs=zs, logp=logp, ok=ok, state=state, sig=sig, layers=layers, w_phi=w_phi)
    return out


def backward(theta, occ, n, n_alpha, n_beta, widths, gA, gphi) -> np.ndarray:
    """d/dtheta of sum_m gA[m] A[m] + gphi[m] phi[m], as a flat vector (mask -> exact 0).

    Hand-derived: d logp_p(s_p)/d z_{p,s} = [s == s_p] - softmax_{p,s} (allowed s only),
    d phi/d z_phi = 2 pi sig (1 - sig), ReLU passes the gradient where z > 0.
    """
    f = forward(theta, occ, n, n_alpha, n_beta, widths, keep=True)
    gA = np.asarray(gA, dtype=np.float64)
    gphi = np.asarray(gphi, dtype=np.float64)
    M = gA.size
    prob = np.where(f["ok"], np.exp(f["logp"]), 0.0)
    onehot = np.zeros_like(prob)
    np.put_along_axis(onehot, f["state"][:, :, None], 1.0, axis=2)
    dlogits = (0.5 * gA[:, None, None]) * (onehot - prob) * f["ok"]
    dlogits = dlogits.reshape(M, 4 * n)
    dz_phi = gphi * 2.0 * np.pi * f["sig"] * (1.0 - f["sig"])
    layers = f["layers"]
    mk = masks(n, widths)
    grads = [None] * len(layers)
    hL = f["hs"][-1]
    Wo, _ = layers[-1]
    grads[-1] = ((dlogits.T @ hL) * mk[-1], dlogits.sum(axis=0))
    g_wphi = dz_phi @ hL
    g_bphi = dz_phi.sum()
    dh = dlogits @ Wo + dz_phi[:, None] * f["w_phi"][None, :]
    for l in range(len(layers) - 2, -1, -1):
        dz = dh * (f["zs"][l] > 0.0)
        W, _ = layers[l]
        grads[l] = ((dz.T @ f["hs"][l]) * mk[l], dz.sum(axis=0))
        dh = dz @ W
    flat = []
    for gW, gb in grads:
        flat.append(gW.ravel())
        flat.append(gb)
    flat.append(g_wphi)
    flat.append(np.array([g_bphi]))
    return np.concatenate(flat)


def draw(theta, n, n_alpha, n_beta, widths, m, g: np.random.Generator) -> np.ndarray:
    """`m` independent ancestral draws from |Psi|^2 (with repetition), [m, 2n] uint8.

    Orbital by orbital: the conditionals of orbital p depend only on orbitals < p,
    so the network is run on the partial determinant (later orbitals still empty)
    and s_p is drawn from the renormalised, number-conserving distribution.
    """
    layers, _, _ = unpack_params(theta, n, widths)
    occ = np.zeros((m, 2 * n), dtype=np.uint8)
    for p in range(n):
        h = occ.astype(np.float64)
        for W, b in layers[:-1]:
            h = np.maximum(h @ W.T + b, 0.0)
        Wo, bo = layers[-1]
        z = h @ Wo[4 * p:4 * p + 4].T + bo[4 * p:4 * p + 4]
        ok = feasible(occ, n, n_alpha, n_beta)[:, p, :]
        z = np.where(ok, z, -np.inf)
        z = z - z.max(axis=1, keepdims=True)
        pr = np.exp(z)
        pr /= pr.sum(axis=1, keepdims=True)
        u = g.random(m)
        s = np.minimum((u[:, None] > np.cumsum(pr, axis=1)).sum(axis=1), 3)
        bad = ~ok[np.arange(m), s]          # cumulative sum rounded below u at the top end
        if np.any(bad):
            s[bad] = np.argmax(np.where(ok[bad], pr[bad], -1.0), axis=1)
        occ[:, 2 * p] = s & 1
        occ[:, 2 * p + 1] = s >> 1
    return occ


def sample(theta, n, n_alpha, n_beta, widths, count, g: np.random.Generator, batch: int = 4096):
    """The first `count` distinct determinants (in draw order) of repeated ancestral draws."""
    seen = {}
    while len(seen) < count:
        for row in draw(theta, n, n_alpha, n_beta, widths, batch, g):
            key = row.tobytes()
            if key not in seen:
                seen[key] = row.copy()
                if len(seen) == count:
                    break
    return np.stack(list(seen.values())[:count])
