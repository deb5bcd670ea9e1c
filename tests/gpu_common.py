"""Shared helpers of the GPU parity tests (inputs from the seeded generators, expected
values from the oracle)."""
import numpy as np
import torch

from oracle import bf16 as obf16
from oracle import made as omade
from oracle import slater_condon as osc
from paper_2506_07430_amd import elocal, synth


def words_to_dev(x: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.array(x, dtype=np.uint64, order="C", copy=True).view(np.int64)).cuda()


def words_from_dev(t: torch.Tensor) -> np.ndarray:
    return t.cpu().numpy().view(np.uint64)


def theta_for(theta: np.ndarray, precision: int):
    """(device tensor for the library, FP64 values the oracle must use)."""
    if precision == elocal.FP64:
        return torch.tensor(theta, dtype=torch.float64).cuda(), np.asarray(theta, dtype=np.float64)
    # ELOCAL_BF16 and ELOCAL_BF16X3 take the same bf16 parameters
    dev = torch.tensor(theta, dtype=torch.float64).to(torch.float32).to(torch.bfloat16).cuda()
    return dev, obf16.round_to_bf16(theta)


def ansatz_samples(p: synth.Problem, count: int, seed: int, theta=None) -> np.ndarray:
    """`count` distinct determinants drawn from the ansatz by the oracle's sampler, sorted."""
    s = p.system
    th = p.theta if theta is None else theta
    occ = omade.sample(th, s.n, s.n_alpha, s.n_beta, s.widths, count, np.random.default_rng(seed),
                       batch=max(256, 2 * count))
    return synth.sort_unique_words(osc.pack(occ))


def make_ham(p: synth.Problem) -> elocal.Hamiltonian:
    s = p.system
    return elocal.Hamiltonian(p.h1e, p.eri, s.n, s.n_alpha, s.n_beta)
