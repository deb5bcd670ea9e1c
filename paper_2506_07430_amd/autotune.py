"""Launch-shape autotuner of the fused local-energy kernel.

The arithmetic tile is fixed (16x16x32 16-bit or 16x16x4 FP64 matrix-core tiles); what
depends on the workload is how the work is cut and spread:

* ``cols``   -- 16-row tiles per network pass (BF16: 1 or 2; two tiles let each weight
  fragment feed twice the rows but need twice the registers, so the kernel variant has half
  the waves per block);
* ``waves``  -- waves per block (at most what the variant is built for);
* ``groups`` -- list-entry groups per work item (longer items amortise the per-sample
  set-up, shorter ones balance the tail);
* ``grid``   -- blocks of the persistent grid.

``tune_eval`` times candidate shapes on the caller's own batch with the library's
HIP-event timer of the fused kernel and keeps the fastest on the handle; ``tune_multi``
does the same for the several-system launch. Every candidate is read back from the library
(``launch_info``), so shapes the kernels do not provide are recorded as what actually ran.
Only the launch shape changes: every shape computes the same per-entry terms, summed per
work item in a fixed order, so results differ between shapes by rounding alone.

Choices persist in a JSON file named by the environment variable ``ELOCAL_AUTOTUNE_CACHE``
(no file when it is unset), keyed by device, orbitals, electrons, hidden widths,
precision and batch size (for the several-system launch: the tuple of every system's key).
A cached shape is applied without timing anything.
"""
from __future__ import annotations

import json
import os
from typing import Dict, List, Optional, Sequence

import torch

from . import elocal

CACHE_ENV = "ELOCAL_AUTOTUNE_CACHE"


def _cu_count() -> int:
    return torch.cuda.get_device_properties(torch.cuda.current_device()).multi_processor_count


def _device_name() -> str:
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return f"{getattr(p, 'gcnArchName', p.name)}:{p.multi_processor_count}cu"


def problem_key(ham: elocal.Hamiltonian, ansatz: elocal.Ansatz, B: int) -> str:
    """Cache key of one evaluation: device, n, electrons, widths, precision, batch size."""
    return (f"{_device_name()}|n{ham.n}|a{ham.na}b{ham.nb}|w{'x'.join(map(str, ansatz.widths))}"
            f"|p{ansatz.precision}|B{int(B)}")


def load_cache(path: Optional[str] = None) -> Dict[str, dict]:
    path = path or os.environ.get(CACHE_ENV)
    if not path or not os.path.exists(path):
        return {}
    with open(path) as f:
        data = json.load(f)
    return data if isinstance(data, dict) else {}


def store_cache(key: str, entry: dict, path: Optional[str] = None) -> None:
    """Adds one entry (read-modify-write of the whole file, written atomically)."""
    path = path or os.environ.get(CACHE_ENV)
    if not path:
        return
    data = load_cache(path)
    data[key] = entry
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = f"{path}.tmp{os.getpid()}"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def dimensions(ham: elocal.Hamiltonian, ansatz: elocal.Ansatz, B: int, cu: Optional[int] = None) -> Dict[str, list]:
    """Values to try per launch-shape dimension, the built-in choice (0) first. Waves per
    block come from the library (the maximum of the tiles-per-pass variant and half of it),
    grids are multiples of the CU count."""
    cu = cu or _cu_count()
    if ansatz.precision == elocal.FP64:
        return {"groups": [0, 4, 8, 32, 64], "grid": [0, cu * 2, cu * 4, cu * 16]}
    ham.tune()
    default = ham.launch_info(ansatz, B)
    cols = [0]
    for c in (1, 2):
        ham.tune(0, 0, 0, c)
        if c != default["cols"] and ham.launch_info(ansatz, B)["cols"] == c:
            cols.append(c)
    ham.tune()
    wmax = default["max_waves"]
    return {"cols": cols, "waves": [0, max(1, wmax // 2)], "groups": [0, 2, 4, 16, 32],
            "grid": [0] + [cu * m // max(wmax, 1) for m in (8, 16, 64)]}


def _search(dims: Dict[str, list], timed, budget_s: float) -> List[Dict]:
    """Coordinate search from the built-in shape: each dimension in turn over its values,
    the others held at the best so far. timed(shape) -> milliseconds."""
    best = {k: 0 for k in ("grid", "groups", "waves", "cols")}
    table, spent = [], 0.0
    seen = {}

    def run(shape):
        nonlocal spent
        key = tuple(sorted(shape.items()))
        if key in seen:
            return seen[key]
        ms = timed(shape)
        seen[key] = ms
        table.append({"shape": dict(shape), "ms": ms})
        spent += ms / 1e3
        return ms

    best_ms = run(best)
    for dim, values in dims.items():
        for v in values:
            if spent > budget_s:
                return table
            cand = dict(best, **{dim: v})
            ms = run(cand)
            if ms < best_ms:
                best, best_ms = cand, ms
    return table


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


def _apply(ham: elocal.Hamiltonian, shape: dict) -> None:
    ham.tune(shape.get("grid", 0), shape.get("groups", 0), shape.get("waves", 0), shape.get("cols", 0))


def tune_eval(ham: elocal.Hamiltonian, ansatz: elocal.Ansatz, x: torch.Tensor,
              shapes: Optional[Sequence[dict]] = None, reps: int = 2, budget_s: float = 60.0,
              use_cache: bool = True) -> List[Dict]:
    """Try launch shapes on this batch, keep the fastest on `ham`; returns the timings
    (each row: the requested shape, the shape the library ran, and its milliseconds).

    A shape cached for this problem is applied without timing (one row, "cached": True).
    Stops early once `budget_s` seconds of kernel time have been spent (the built-in shape
    is always tried first, so the result is never worse than it)."""
    B = int(x.shape[0])
    key = problem_key(ham, ansatz, B)
    if use_cache:
        hit = load_cache().get(key)
        if hit is not None:
            _apply(ham, hit["shape"])
            return [dict(hit, cached=True)]
    out = torch.empty((B, 2), dtype=torch.float64, device=x.device)

    def timed(shape):
        _apply(ham, shape)
        return time_eval(ham, ansatz, x, reps, out)

    if shapes is None:
        table = _search(dimensions(ham, ansatz, B), timed, budget_s / (reps + 1))
    else:
        table = [{"shape": dict(sh), "ms": timed(sh)} for sh in shapes]
    for row in table:
        _apply(ham, row["shape"])
        ran = ham.launch_info(ansatz, B)
        row["ran"] = {k: ran[k] for k in ("grid", "groups", "waves", "cols")}
    best = min(table, key=lambda r: r["ms"])
    _apply(ham, best["shape"])
    if use_cache:
        store_cache(key, {"shape": best["shape"], "ran": best["ran"], "ms": best["ms"], "tried": len(table)})
    return table


def tune_multi(mev: elocal.MultiEval, hams: Sequence[elocal.Hamiltonian], ansatze: Sequence[elocal.Ansatz],
               xs: Sequence[torch.Tensor], shapes: Optional[Sequence[dict]] = None, reps: int = 1,
               budget_s: float = 30.0, use_cache: bool = True) -> List[Dict]:
    """The same search for the several-system launch (elocal_eval_multi): grid, waves and
    tiles per pass come from the first handle, the groups per work item from each system's
    handle, so every candidate is set on all of them. Keeps the fastest; returns the timings."""
    key = "multi[" + ";".join(problem_key(h, a, x.shape[0]) for h, a, x in zip(hams, ansatze, xs)) + "]"
    if use_cache:
        hit = load_cache().get(key)
        if hit is not None:
            for h in hams:
                _apply(h, hit["shape"])
            return [dict(hit, cached=True)]
    widest = max(range(len(hams)), key=lambda i: max(ansatze[i].widths))

    def timed(shape):
        for h in hams:
            _apply(h, shape)
        mev(hams, ansatze, xs)
        torch.cuda.synchronize()
        hams[0].timing(True)
        hams[0].kernel_time(reset=True)
        for _ in range(reps):
            mev(hams, ansatze, xs)
        ms, n = hams[0].kernel_time(reset=True)
        hams[0].timing(False)
        return ms / max(n, 1)

    if shapes is None:
        table = _search(dimensions(hams[widest], ansatze[widest], xs[widest].shape[0]), timed, budget_s / (reps + 1))
    else:
        table = [{"shape": dict(sh), "ms": timed(sh)} for sh in shapes]
    best = min(table, key=lambda r: r["ms"])
    for h in hams:
        _apply(h, best["shape"])
    if use_cache:
        store_cache(key, {"shape": best["shape"], "ms": best["ms"], "tried": len(table)})
    return table
