#!/usr/bin/env python3
"""Throughput of the local-energy hot path on one MI355X.

One step = the whole path on one batch: local energies of every sample (generator,
Slater--Condon elements, ansatz on every connected determinant, FP64 ratio sums),
the weighted energy statistics and the VMC gradient (forward recomputation and
backward at the samples). Inputs are resident in device memory before timing.

Workload (default): 24 spatial orbitals, 12 alpha + 12 beta electrons, integrals
with couplings damped by exp(-|p-q|/6), 16384 unique samples with Zipf(1.5)
multiplicities, ansatz 48 -> 128 -> 128 -> 96 (+ phase) in BF16 on matrix cores with
FP32 accumulation and FP64 assembly. The all-FP64 path is timed beside it.

Prints one JSON line (see the fields at the bottom).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "local energies/s + H_xx' elems/s at 1 GPU, BF16+FP64 vs all-FP64, |dE|<=1e-5 Ha"
PEAK_BF16_TFLOPS = 2500.0     # MI355X dense BF16 matrix peak
PEAK_F64_TFLOPS = 78.6        # MI355X FP64 matrix/vector peak
COUNTERS = os.path.join(ROOT, "profiles", "eval_bf16_n24_counters.json")
KERNEL_SRC = os.path.join(ROOT, "paper_2506_07430_amd", "csrc", "made_bf16.hip")
CONNECT_COUNTERS = os.path.join(ROOT, "profiles", "connect_n24_counters.json")
CONNECT_SRC = os.path.join(ROOT, "paper_2506_07430_amd", "csrc", "hamiltonian.hip")
PEAK_HBM_GBS = 8000.0         # MI355X HBM3E


def unmasked_weights(n: int, widths) -> int:
    """Weights the autoregressive mask keeps (degree rule of include/elocal.h) that E_loc needs,
    phase head included. The last orbital's logits are left out: its conditional is 1 whatever
    they are (one occupation keeps both electron counts reachable)."""
    deg_in = np.arange(2 * n) // 2 + 1
    hid = [np.arange(w) % (n - 1) + 1 for w in widths]
    total = int(np.sum(hid[0][:, None] >= deg_in[None, :]))
    for l in range(1, len(widths)):
        total += int(np.sum(hid[l][:, None] >= hid[l - 1][None, :]))
    deg_out = np.arange(4 * (n - 1)) // 4 + 1
    total += int(np.sum(deg_out[:, None] > hid[-1][None, :]))
    return total + widths[-1]


def dense_weights(n: int, widths) -> int:
    """Weights of the same network without the mask (last orbital's logits left out)."""
    dims = [2 * n] + list(widths) + [4 * (n - 1)]
    return sum(dims[i] * dims[i + 1] for i in range(len(dims) - 1)) + widths[-1]


def file_hash(path: str) -> str:
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--fp64-steps", type=int, default=2)
    ap.add_argument("--cpu-samples", type=int, default=128)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-fp64", action="store_true", help="skip the all-FP64 comparison")
    ap.add_argument("--no-graph", action="store_true",
                    help="time eager launches instead of replays of the captured step")
    ap.add_argument("--no-autotune", action="store_true", help="keep the built-in launch shape")
    ap.add_argument("--sampler-draws", type=int, default=1_000_000,
                    help="draws of the batch autoregressive sampler leg (FP64 ansatz of the workload); 0 skips")
    ap.add_argument("--pauli-samples", type=int, default=1024,
                    help="samples of the Pauli-string route leg (Algorithm 1 over unique flips); 0 skips")
    ap.add_argument("--dedup-reps", type=int, default=5,
                    help="timed runs of the deduplicated evaluation on the 8-orbital workload; 0 skips")
    ap.add_argument("--kpm-moments", type=int, default=64,
                    help="Chebyshev moments of the KPM leg (12 orbitals, 6a+6b, 853,776 determinants); 0 skips")
    ap.add_argument("--connect-reps", type=int, default=3,
                    help="timed runs of the materialising generator (elocal_connect) on the whole batch; 0 skips")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run one plain device copy of this many MiB (a known-size reference "
                         "for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}): the local-energy path would shard "
              "over samples, but only the one-GPU path is implemented and timed.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2506_07430_amd import autotune, elocal, synth

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    cfg = 1
    wl = synth.WORKLOADS[cfg]
    p = synth.make_problem(cfg)
    s = p.system
    B = p.x.shape[0]
    ham = elocal.Hamiltonian(p.h1e, p.eri, s.n, s.n_alpha, s.n_beta)
    C = ham.C
    x = torch.from_numpy(p.x.view(np.int64).copy()).to(dev)
    w = torch.tensor(p.w, dtype=torch.float64, device=dev)
    th64 = torch.tensor(p.theta, dtype=torch.float64, device=dev)
    th16 = th64.to(torch.float32).to(torch.bfloat16).contiguous()
    ans16 = elocal.Ansatz(s.widths, th16, elocal.BF16)
    ans64 = elocal.Ansatz(s.widths, th64, elocal.FP64)
    eloc = torch.empty((B, 2), dtype=torch.float64, device=dev)
    stats = torch.empty(4, dtype=torch.float64, device=dev)
    dth = torch.empty(th64.numel(), dtype=torch.float64, device=dev)

    if args.copy_calibration > 0:
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def step(ans):
        ham.eval(ans, x, out=eloc, want_logpsi=False)
        ham.grad(ans, x, w, eloc, stats=stats, dtheta=dth)

    def timed(ans, steps, warmup):
        """Eager launches; also the fused kernel's time from the library's HIP events."""
        for _ in range(warmup):
            step(ans)
        torch.cuda.synchronize()
        ham.timing(True)
        ham.kernel_time(reset=True)
        t0 = time.perf_counter()
        for _ in range(steps):
            step(ans)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        kms, nl = ham.kernel_time(reset=True)
        ham.timing(False)
        return (t1 - t0) / steps, kms / max(nl, 1), nl

    def timed_graph(ans, steps):
        """The whole step captured once as a HIP graph, then replayed `steps` times."""
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            step(ans)                       # workspaces exist before capture
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        with torch.cuda.graph(g):
            step(ans)
        g.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            g.replay()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    tune_table = None
    if not args.no_autotune:
        tune_table = autotune.tune_eval(ham, ans16, x)
    sec16_eager, kern16_ms, nl16 = timed(ans16, args.steps, args.warmup)
    sec16 = sec16_eager if args.no_graph else timed_graph(ans16, args.steps)
    eloc16 = eloc.cpu().numpy().copy()
    stats16 = stats.cpu().numpy().copy()
    out = {}
    if not args.no_fp64:
        sec64, kern64_ms, nl64 = timed(ans64, args.fp64_steps, 1)
        eloc64 = eloc.cpu().numpy().copy()
        out["fp64"] = {
            "ms_per_step": sec64 * 1e3,
            "local_energies_per_s": B / sec64,
            "h_elems_per_s": B * C / sec64,
            "eval_kernel_ms": kern64_ms,
            "eval_kernel_tflops_alg": B * (C - 1) * 2 * unmasked_weights(s.n, s.widths) / (kern64_ms * 1e-3) / 1e12,
            "peak_tflops": PEAK_F64_TFLOPS,
            "steps": args.fp64_steps,
        }

    # --- roofline of the dominant kernel (fused BF16 local-energy kernel)
    uw = unmasked_weights(s.n, s.widths)
    dw = dense_weights(s.n, s.widths)
    flops_alg = B * (C - 1) * 2.0 * uw
    achieved = flops_alg / (kern16_ms * 1e-3) / 1e12
    traffic = None
    if os.path.exists(COUNTERS):
        with open(COUNTERS) as f:
            cnt = json.load(f)
        if cnt.get("kernel_src_sha256_16") == file_hash(KERNEL_SRC) and cnt.get("samples") == B:
            traffic = cnt.get("hbm_bytes_per_launch")
    roof = {"bound": "mfma", "achieved": achieved, "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / PEAK_BF16_TFLOPS, "traffic": traffic,
            "kernel": "k_eval_bf16", "kernel_ms": kern16_ms, "launches_timed": nl16,
            "alg_flops_per_row": 2 * uw, "dense_flops_per_row": 2 * dw,
            "dense_frac": B * (C - 1) * 2.0 * dw / (kern16_ms * 1e-3) / 1e12 / PEAK_BF16_TFLOPS}

    # --- the materialising generator + matrix elements (elocal_connect), HBM-write-bound:
    # algorithmic bytes per listed pair = x' (8W) + H (8) + sign (1) + exc (4)
    if args.connect_reps > 0:
        W = ham.W
        outs = (torch.empty((B, C, W), dtype=torch.int64, device=dev),
                torch.empty((B, C), dtype=torch.float64, device=dev),
                torch.empty((B, C), dtype=torch.int8, device=dev),
                torch.empty((B, C), dtype=torch.int32, device=dev))
        ham.connect(x, out=outs)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(args.connect_reps):
            ham.connect(x, out=outs)
        ev1.record()
        torch.cuda.synchronize()
        cms = ev0.elapsed_time(ev1) / args.connect_reps
        per_pair = 8 * W + 8 + 1 + 4
        alg = B * C * per_pair
        ctraffic = None
        if os.path.exists(CONNECT_COUNTERS):
            with open(CONNECT_COUNTERS) as f:
                cc = json.load(f)
            if cc.get("kernel_src_sha256_16") == file_hash(CONNECT_SRC) and cc.get("samples") == B:
                ctraffic = cc.get("hbm_bytes_per_launch")
        out["connect"] = {"bound": "hbm", "ms": cms, "pairs_per_s": B * C / (cms * 1e-3),
                          "bytes_per_pair": per_pair, "achieved": alg / (cms * 1e-3) / 1e9, "peak": PEAK_HBM_GBS,
                          "unit": "GB/s", "frac": alg / (cms * 1e-3) / 1e9 / PEAK_HBM_GBS, "traffic": ctraffic,
                          "note": "prep + generator launches on the caller's stream, HIP events around them"}
        del outs
        torch.cuda.empty_cache()

    # --- batch autoregressive sampling from the same ansatz (FP64 conditionals)
    if args.sampler_draws > 0:
        ham.sample(ans64, 1000, 1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xs_, cs_ = ham.sample(ans64, args.sampler_draws, 2026)
        t_s = time.perf_counter() - t0
        out["sampler"] = {"draws": args.sampler_draws, "distinct": int(xs_.shape[0]), "seconds": t_s,
                          "draws_per_s": args.sampler_draws / t_s, "orbital_steps": s.n,
                          "note": "synchronous call (the tree size is read back per orbital)"}
        del xs_, cs_

    # --- the paper's Pauli-string route on the same ansatz and samples: every unique flip
    # of the Jordan--Wigner strings goes through the ansatz (vs the C connected ones)
    if args.pauli_samples > 0:
        Bp = min(args.pauli_samples, B)
        xp = x[:Bp].contiguous()
        t0 = time.perf_counter()
        n_str, n_flip = ham.pauli_build()
        t_build = time.perf_counter() - t0
        ep = torch.empty((Bp, 2), dtype=torch.float64, device=dev)
        es = torch.empty((Bp, 2), dtype=torch.float64, device=dev)
        ham.eval_pauli(ans16, xp, out=ep)
        ham.eval(ans16, xp, out=es, want_logpsi=False)
        torch.cuda.synchronize()
        ham.timing(True)
        ham.kernel_time(reset=True)
        ham.eval_pauli(ans16, xp, out=ep)
        pms, _ = ham.kernel_time(reset=True)
        ham.eval(ans16, xp, out=es, want_logpsi=False)
        sms, _ = ham.kernel_time(reset=True)
        ham.timing(False)
        diff = float(((ep - es).norm(dim=1) / es.norm(dim=1)).max().item())
        out["pauli_route"] = {"samples": Bp, "strings": n_str, "unique_flips": n_flip, "connected": C,
                              "build_s": t_build, "kernel_ms": pms, "slater_condon_kernel_ms": sms,
                              "ansatz_rows_ratio": (n_flip - 1) / (C - 1), "time_ratio": pms / sms,
                              "max_rel_diff_vs_slater_condon": diff}

    # --- deduplicated evaluation (each distinct x' of the batch once) against the fused kernel,
    # on the 8-orbital workload (1024 samples x 361 listed pairs); whole calls between events
    if args.dedup_reps > 0:
        dp = synth.make_problem(0)
        dsys = dp.system
        dham = elocal.Hamiltonian(dp.h1e, dp.eri, dsys.n, dsys.n_alpha, dsys.n_beta)
        dth = torch.tensor(dp.theta).to(dev).float().to(torch.bfloat16).contiguous()
        dans = elocal.Ansatz(dsys.widths, dth, elocal.BF16)
        dx = torch.from_numpy(dp.x.view(np.int64).copy()).to(dev)
        ed = torch.empty((dx.shape[0], 2), dtype=torch.float64, device=dev)
        ef = torch.empty((dx.shape[0], 2), dtype=torch.float64, device=dev)
        _, _, cnt = dham.eval_dedup(dans, dx, out=ed)
        dham.eval(dans, dx, out=ef, want_logpsi=False)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.dedup_reps):
            dham.eval_dedup(dans, dx, out=ed)
        e1.record()
        torch.cuda.synchronize()
        dms = e0.elapsed_time(e1) / args.dedup_reps
        e0.record()
        for _ in range(args.dedup_reps):
            dham.eval(dans, dx, out=ef, want_logpsi=False)
        e1.record()
        torch.cuda.synchronize()
        fms = e0.elapsed_time(e1) / args.dedup_reps
        out["dedup"] = {"workload": "8 orbitals, 4a+4b, 1024 samples, 361 listed per sample",
                        "listed": int(dx.shape[0]) * dham.C, "distinct": int(cnt.item()),
                        "ms": dms, "fused_ms": fms,
                        "max_abs_diff_vs_fused": float((ed - ef).abs().max().item()),
                        "note": "whole calls on the caller's stream, HIP events around them"}
        del dham, dans

    # --- KPM: Chebyshev moments on a full-sector vector (12 orbitals, 6a+6b); each step is
    # one sector-wide H v (row-by-row generator + Slater--Condon + ranked gathers)
    if args.kpm_moments > 0:
        kp = synth.random_problem(12, 6, 6, (32,), seed=12, n_chol=16, decay=6.0, samples=1)
        kham = elocal.Hamiltonian(kp.h1e, kp.eri, 12, 6, 6)
        kdim = kham.sector_dim
        g = torch.Generator(device="cpu").manual_seed(12)
        alpha = torch.randn(kdim, generator=g, dtype=torch.float64).to(dev)
        alpha /= alpha.norm()
        scale = 4.0 * float(np.abs(kp.h1e).sum() + 0.5 * np.abs(kp.eri).sum())   # loose spectral bound
        kham.kpm_moments(alpha, 4, scale, 0.0)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        mu = kham.kpm_moments(alpha, args.kpm_moments, scale, 0.0)
        e1.record()
        torch.cuda.synchronize()
        kms = e0.elapsed_time(e1)
        steps = (args.kpm_moments) // 2
        out["kpm"] = {"sector": "12 orbitals, 6a+6b", "dim": kdim, "connected_per_row": kham.C,
                      "n_moments": args.kpm_moments, "ms": kms, "hv_ms": kms / max(steps, 1),
                      "moments_per_s": args.kpm_moments / (kms * 1e-3),
                      "h_elems_per_s": kdim * kham.C * steps / (kms * 1e-3),
                      "omega_0": float(mu[0].item()), "max_abs_omega": float(mu.abs().max().item())}
        del kham, alpha

    # --- CPU oracle on a bounded sample (host cores), and the error of both GPU modes on it
    if not args.no_cpu:
        from threadpoolctl import threadpool_info
        from oracle import bf16 as obf16
        from oracle import energy as oen
        S = min(args.cpu_samples, B)
        th_or = obf16.round_to_bf16(p.theta)
        t0 = time.perf_counter()
        ref = oen.local_energies(p.h1e, p.eri, s.n, s.n_alpha, s.n_beta, s.widths, th_or, p.x[:S])
        t1 = time.perf_counter()
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
        out["cpu_baseline"] = {"value": S / (t1 - t0), "unit": "local energies/s", "cores": threads,
                               "kind": "oracle",
                               "sample": f"first {S} of the {B} samples, BF16-rounded parameters, FP64 NumPy; "
                                         f"{len(os.sched_getaffinity(0))} host cores visible",
                               "seconds": t1 - t0}
        g16 = eloc16[:S, 0] + 1j * eloc16[:S, 1]
        err = {"samples": S, "bf16_max_abs_dEloc": float(np.max(np.abs(g16 - ref))),
               "bf16_abs_dE_weighted": float(abs(np.sum(p.w[:S] * g16) / p.w[:S].sum()
                                                 - np.sum(p.w[:S] * ref) / p.w[:S].sum()))}
        if not args.no_fp64:
            S64 = min(8, S)
            ref64 = oen.local_energies(p.h1e, p.eri, s.n, s.n_alpha, s.n_beta, s.widths, p.theta, p.x[:S64])
            g64 = eloc64[:S64, 0] + 1j * eloc64[:S64, 1]
            err["fp64_max_rel_dEloc"] = float(np.max(np.abs(g64 - ref64) / np.abs(ref64)))
            err["fp64_samples"] = S64
        out["error_vs_oracle"] = err

    line = {
        "metric": METRIC,
        "value": B / sec16,
        "unit": "local energies/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec16 * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16+f64",
        "data": "synthetic",
        "config": {"workload": f"{wl.name}: n=24 orbitals, 12a+12b, {B} unique samples (Zipf 1.5 weights), "
                               f"{C} connected determinants each, ansatz 48-128-128-96(+phase)",
                   "orbitals": s.n, "alpha": s.n_alpha, "beta": s.n_beta, "hidden": list(s.widths),
                   "samples": B, "connected_per_sample": C, "step": "eval + stats + grad"},
        "h_elems_per_s": B * C / sec16,
        "energy": {"re": float(stats16[0]), "im": float(stats16[1]), "var": float(stats16[2])},
        "roofline": roof,
        "timing": {"mode": "eager" if args.no_graph else "hip graph replay", "eager_ms_per_step": sec16_eager * 1e3,
                   "launch_shape": ({"autotuned": True, "chosen": min(tune_table, key=lambda r: r["ms"]),
                                     "tried": len(tune_table)} if tune_table else {"autotuned": False})},
    }
    line.update(out)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
