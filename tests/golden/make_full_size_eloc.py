"""Writes full_size_eloc.json: oracle local energies of sampled determinants of the
full-size workloads, for the GPU parity tests that run those workloads whole.

Inputs come from the seeded generators (paper_2506_07430_amd.synth); values from the
FP64 oracle only: "bf16" entries use the parameters rounded to bfloat16 (what the
BF16 mode evaluates), "fp64" entries the raw parameters. The determinant words are
stored with each value, so a test can confirm it regenerated the same input.

Run from the repository root:  python tests/golden/make_full_size_eloc.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import bf16 as obf16  # noqa: E402
from oracle import energy as oen  # noqa: E402
from paper_2506_07430_amd import synth  # noqa: E402

# (workload, system index, sample indices (negative: from the end), precisions)
CASES = [(1, 0, (0, 8191, -1), ("bf16",)), (1, 0, (0,), ("fp64",))] + \
    [(2, s, (0, -1), ("bf16",)) for s in range(8)] + [
    (3, 0, (0, 4095, -1), ("bf16",)),
    (3, 0, (0,), ("fp64",)),
    (4, 0, (0, 100, 200, 300, 400, 500, 600, 700, 800, -1), ("bf16",)),
    (4, 0, (0,), ("fp64",)),
]


def main():
    out = []
    for cfg, si, picks, precs in CASES:
        p = synth.make_problem(cfg, si)
        s = p.system
        B = p.x.shape[0]
        for prec in precs:
            th = obf16.round_to_bf16(p.theta) if prec == "bf16" else p.theta
            for k in picks:
                i = k % B
                t0 = time.perf_counter()
                e = oen.local_energies(p.h1e, p.eri, s.n, s.n_alpha, s.n_beta, s.widths, th, p.x[i:i + 1])[0]
                out.append({"workload": cfg, "system": si, "n": s.n, "samples": B, "index": i,
                            "x": [f"{int(v):016x}" for v in p.x[i]], "precision": prec,
                            "re": float(e.real), "im": float(e.imag)})
                print(f"workload {cfg} system {si} sample {i} {prec}: {e:.12f} ({time.perf_counter() - t0:.1f} s)",
                      flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "full_size_eloc.json")
    with open(path, "w") as f:
        json.dump({"generator": "tests/golden/make_full_size_eloc.py", "entries": out}, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
