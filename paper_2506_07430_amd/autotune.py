"""Launch-shape autotuner of the fused local-energy kernel.

The kernel's arithmetic tile is fixed (16x16x32 BF16 or 16x16x4 FP64 matrix-core
tiles, 32 or 16 rows per network pass); what depends on the workload is how its work
is cut and spread: how many list-entry groups form one work item (longer items amortise
the per-sample set-up, shorter ones balance the tail better) and how many blocks the
persistent grid has. ``tune_eval`` times candidate shapes on the caller's own batch with
the library's HIP-event timer of the fused kernel, keeps the fastest on the handle
(``elocal_tune``) and returns the table. Only the launch shape changes: every shape
computes the same per-entry terms, summed per work item in a fixed order, so the
results differ between shapes by rounding alone.
"""
from __future__ import annotations

from typing import Dict, List, Optional, Sequence

import torch

from . import elocal


def _cu_count() -> int:
    return torch.cuda.get_device_properties(torch.cuda.current_device()).multi_processor_count


def candidates(precision: int, hidden_max: int, cu: Optional[int] = None):
    """(grid, groups) pairs to try; grid 0 and groups 0 mean the library's own choice."""
    cu = cu or _cu_count()
    bf16 = precision != elocal.FP64
    nterms = 3 if precision == elocal.BF16X3 else 2
    waves = 8 if (bf16 and hidden_max * nterms <= 256) else 4
    grids = [0] + [cu * m // waves for m in (8, 16, 64)]
    groups = [0, 2, 4, 16, 32] if bf16 else [0, 4, 8, 32, 64]
    return [(g, k) for g in grids for k in groups]


def time_eval(ham: elocal.Hamiltonian, ansatz: elocal.Ansatz, x: torch.Tensor, reps: int = 2,
              out: Optional[torch.Tensor] = None) -> float:
    """Mean milliseconds of the fused kernel over `reps` evaluations (after one warm-up)."""
    if out is None:
        out = torch.empty((x.shape[0], 2), dtype=torch.float64, device=x.device)
    ham.eval(ansatz, x, out=out, want_logpsi=False)
    torch.cuda.synchronize()
    ham.timing(True)
    ham.kernel_time(reset=True)
    for _ in range(reps):
        ham.eval(ansatz, x, out=out, want_logpsi=False)
    ms, n = ham.kernel_time(reset=True)
    ham.timing(False)
    return ms / max(n, 1)


def tune_eval(ham: elocal.Hamiltonian, ansatz: elocal.Ansatz, x: torch.Tensor,
              shapes: Optional[Sequence] = None, reps: int = 2, budget_s: float = 60.0) -> List[Dict]:
    """Try launch shapes on this batch, keep the fastest on `ham`; returns the timings.

    Stops early once `budget_s` seconds of kernel time have been spent (the built-in
    shape is always tried first, so the result is never worse than it).
    """
    shapes = list(shapes) if shapes is not None else candidates(ansatz.precision, max(ansatz.widths))
    out = torch.empty((x.shape[0], 2), dtype=torch.float64, device=x.device)
    table, spent = [], 0.0
    for grid, groups in shapes:
        ham.tune(grid, groups)
        ms = time_eval(ham, ansatz, x, reps, out)
        table.append({"grid": grid, "groups": groups, "ms": ms})
        spent += ms * (reps + 1) / 1e3
        if spent > budget_s:
            break
    best = min(table, key=lambda r: r["ms"])
    ham.tune(best["grid"], best["groups"])
    return table


def tune_multi(mev: elocal.MultiEval, hams: Sequence[elocal.Hamiltonian], ansatze: Sequence[elocal.Ansatz],
               xs: Sequence[torch.Tensor], shapes: Optional[Sequence] = None, reps: int = 1,
               budget_s: float = 30.0) -> List[Dict]:
    """The same search for the several-system launch (elocal_eval_multi): the grid comes
    from the first handle, the groups per work item from each system's handle, so every
    candidate is set on all of them. Keeps the fastest; returns the timings."""
    shapes = list(shapes) if shapes is not None else candidates(ansatze[0].precision,
                                                                max(max(a.widths) for a in ansatze))
    table, spent = [], 0.0
    for grid, groups in shapes:
        for h in hams:
            h.tune(grid, groups)
        mev(hams, ansatze, xs)
        torch.cuda.synchronize()
        hams[0].timing(True)
        hams[0].kernel_time(reset=True)
        for _ in range(reps):
            mev(hams, ansatze, xs)
        ms, n = hams[0].kernel_time(reset=True)
        hams[0].timing(False)
        ms /= max(n, 1)
        table.append({"grid": grid, "groups": groups, "ms": ms})
        spent += ms * (reps + 1) / 1e3
        if spent > budget_s:
            break
    best = min(table, key=lambda r: r["ms"])
    for h in hams:
        h.tune(best["grid"], best["groups"])
    return table
