#!/usr/bin/env python3
"""Throughput of the local-energy hot path on one MI355X.

One step = the whole path on one batch: local energies of every sample (generator,
Slater--Condon elements, ansatz on every connected determinant, FP64 ratio sums),
the weighted energy statistics and the VMC gradient (forward recomputation and
backward at the samples). Inputs are resident in device memory before timing.

Headline workload (default): the largest single-GPU case, 60 spatial orbitals,
26 alpha + 26 beta electrons, integrals with couplings damped by exp(-|p-q|/8) and 60
Cholesky vectors, 1024 unique samples, 1,147,875 connected determinants each, ansatz
120 -> 256 -> 256 -> 256 -> 240 (+ phase) with bfloat16 parameters on the 16-bit matrix
cores (FP32 accumulation) and FP64 matrix elements, ratios and sums.

Further legs: the 24-orbital workload (16384 samples, Zipf(1.5) weights), the eight
systems of 12..40 orbitals in one persistent launch, the 40-orbital forward+gradient
workload, the all-FP64 path, the materialising generator, the sampler, the Pauli-string
route, the deduplicated evaluation, the KPM moments, and the CPU oracle on a bounded
sample. Prints one JSON line.
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
PEAK_16BIT_TFLOPS = 2500.0    # MI355X dense bf16/fp16 matrix peak
PEAK_F64_TFLOPS = 78.6        # MI355X FP64 matrix/vector peak
PEAK_HBM_GBS = 8000.0         # MI355X HBM3E
KERNEL_SRC = os.path.join(ROOT, "paper_2506_07430_amd", "csrc", "made_bf16.hip")
CONNECT_SRC = os.path.join(ROOT, "paper_2506_07430_amd", "csrc", "hamiltonian.hip")
GOLDEN = os.path.join(ROOT, "tests", "golden", "full_size_eloc.json")
# HBM bytes per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE runs, kept with the source
# hash they were taken on (a changed kernel makes them stale: traffic is then null)
COUNTERS = {1: os.path.join(ROOT, "profiles", "eval_bf16_n24_counters.json"),
            4: os.path.join(ROOT, "profiles", "eval_bf16_n60_counters.json")}
CONNECT_COUNTERS = os.path.join(ROOT, "profiles", "connect_n24_counters.json")


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


def stored_traffic(path: str, src: str, samples: int):
    if not os.path.exists(path):
        return None
    with open(path) as f:
        cnt = json.load(f)
    if cnt.get("kernel_src_sha256_16") == file_hash(src) and cnt.get("samples") == samples:
        return cnt.get("hbm_bytes_per_launch")
    return None


def describe(wl, p, C):
    s = p.system
    dims = [2 * s.n] + list(s.widths) + [4 * s.n]
    return (f"{wl.name}: n={s.n} orbitals, {s.n_alpha}a+{s.n_beta}b, {p.x.shape[0]} unique samples "
            f"({'Zipf 1.5' if wl.multiplicity != 'ones' else 'unit'} weights), {C} connected determinants each, "
            f"ansatz {'-'.join(map(str, dims))}(+phase)")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", type=int, default=4, choices=(1, 3, 4),
                    help="headline workload (4: 60 orbitals, the largest; 3: 40 orbitals; 1: 24 orbitals)")
    ap.add_argument("--legs", default="c1,c2,c3,fp64,connect,sampler,pauli,dedup,kpm,cpu",
                    help="comma-separated extra legs to run (empty: headline only)")
    ap.add_argument("--cpu-samples", type=int, default=1,
                    help="samples of the headline workload the CPU oracle evaluates")
    ap.add_argument("--fp64-samples", type=int, default=64,
                    help="samples of the headline workload timed in all-FP64 mode")
    ap.add_argument("--no-graph", action="store_true",
                    help="time eager launches instead of replays of the captured step")
    ap.add_argument("--no-autotune", action="store_true", help="keep the built-in launch shape")
    ap.add_argument("--sampler-draws", type=int, default=1_000_000)
    ap.add_argument("--pauli-samples", type=int, default=1024)
    ap.add_argument("--dedup-reps", type=int, default=5)
    ap.add_argument("--kpm-moments", type=int, default=64)
    ap.add_argument("--connect-reps", type=int, default=10)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run one plain device copy of this many MiB (a known-size reference "
                         "for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}): the local-energy path would shard "
              "over samples, but only the one-GPU path is implemented and timed.", file=sys.stderr)
        sys.exit(2)
    legs = set(l for l in args.legs.split(",") if l)

    import torch
    from paper_2506_07430_amd import autotune, elocal, synth

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")

    if args.copy_calibration > 0:
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def setup(cfg, samples=None):
        wl = synth.WORKLOADS[cfg]
        p = synth.make_problem(cfg, samples=samples)
        s = p.system
        ham = elocal.Hamiltonian(p.h1e, p.eri, s.n, s.n_alpha, s.n_beta)
        x = torch.from_numpy(p.x.view(np.int64).copy()).to(dev)
        w = torch.tensor(p.w, dtype=torch.float64, device=dev)
        th64 = torch.tensor(p.theta, dtype=torch.float64, device=dev)
        th16 = th64.to(torch.float32).to(torch.bfloat16).contiguous()
        return wl, p, ham, x, w, elocal.Ansatz(s.widths, th16, elocal.BF16), elocal.Ansatz(s.widths, th64, elocal.FP64)

    class Step:
        """eval + stats + grad on one batch, with preallocated outputs."""

        def __init__(self, ham, ans, x, w):
            B = x.shape[0]
            self.ham, self.ans, self.x, self.w = ham, ans, x, w
            self.eloc = torch.empty((B, 2), dtype=torch.float64, device=dev)
            self.stats = torch.empty(4, dtype=torch.float64, device=dev)
            self.dth = torch.empty(ans.theta.numel(), dtype=torch.float64, device=dev)

        def __call__(self):
            self.ham.eval(self.ans, self.x, out=self.eloc, want_logpsi=False)
            self.ham.grad(self.ans, self.x, self.w, self.eloc, stats=self.stats, dtheta=self.dth)

        def eager(self, steps, warmup):
            """Seconds per step of eager launches and the fused kernel's milliseconds (library
            HIP events on the launch stream)."""
            for _ in range(warmup):
                self()
            torch.cuda.synchronize()
            self.ham.timing(True)
            self.ham.kernel_time(reset=True)
            t0 = time.perf_counter()
            for _ in range(steps):
                self()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            kms, nl = self.ham.kernel_time(reset=True)
            self.ham.timing(False)
            return (t1 - t0) / steps, kms / max(nl, 1), nl

        def graph(self, steps):
            """The whole step captured once as a HIP graph, then replayed `steps` times."""
            g = torch.cuda.CUDAGraph()
            side = torch.cuda.Stream()
            side.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(side):
                self()                      # workspaces exist before capture
            torch.cuda.current_stream().wait_stream(side)
            torch.cuda.synchronize()
            with torch.cuda.graph(g):
                self()
            g.replay()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                g.replay()
            torch.cuda.synchronize()
            return (time.perf_counter() - t0) / steps

        def grad_ms(self, reps=3):
            """Milliseconds of elocal_grad alone (HIP events on the launch stream)."""
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            self.ham.grad(self.ans, self.x, self.w, self.eloc, stats=self.stats, dtheta=self.dth)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(reps):
                self.ham.grad(self.ans, self.x, self.w, self.eloc, stats=self.stats, dtheta=self.dth)
            e1.record()
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / reps

    def roofline(cfg, p, C, kernel_ms, launches, samples):
        s = p.system
        uw, dw = unmasked_weights(s.n, s.widths), dense_weights(s.n, s.widths)
        rows = samples * (C - 1)
        achieved = rows * 2.0 * uw / (kernel_ms * 1e-3) / 1e12
        traffic = stored_traffic(COUNTERS[cfg], KERNEL_SRC, samples) if cfg in COUNTERS else None
        return {"bound": "mfma", "achieved": achieved, "peak": PEAK_16BIT_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_16BIT_TFLOPS, "traffic": traffic,
                "kernel": "k_eval_bf16", "kernel_ms": kernel_ms, "launches_timed": launches,
                "alg_flops_per_row": 2 * uw, "rows_per_launch": rows, "dense_flops_per_row": 2 * dw,
                "dense_frac": rows * 2.0 * dw / (kernel_ms * 1e-3) / 1e12 / PEAK_16BIT_TFLOPS}

    def golden_errors(cfg, p, eloc_np, tag="bf16", system=0):
        """|dE_loc| at the samples whose oracle values tests/golden/full_size_eloc.json holds."""
        if not os.path.exists(GOLDEN):
            return None
        with open(GOLDEN) as f:
            ents = [e for e in json.load(f)["entries"]
                    if e["workload"] == cfg and e["system"] == system and e["precision"] == tag]
        out = []
        for e in ents:
            if [f"{int(v):016x}" for v in p.x[e["index"]]] != e["x"]:
                continue
            got = eloc_np[e["index"], 0] + 1j * eloc_np[e["index"], 1]
            out.append({"index": e["index"], "abs_dEloc": float(abs(got - (e["re"] + 1j * e["im"])))})
        return out

    out = {}

    # ------------------------------------------------------------------ headline
    cfg = args.workload
    wl, p, ham, x, w, ans16, ans64 = setup(cfg)
    s = p.system
    B, C = p.x.shape[0], ham.C
    tune_table = None if args.no_autotune else autotune.tune_eval(ham, ans16, x, reps=1, budget_s=30.0)
    st = Step(ham, ans16, x, w)
    sec_eager, kern_ms, nl = st.eager(args.steps, args.warmup)
    sec = sec_eager if args.no_graph else st.graph(args.steps)
    grad_ms = st.grad_ms()
    eloc16 = st.eloc.cpu().numpy().copy()
    stats16 = st.stats.cpu().numpy().copy()
    roof = roofline(cfg, p, C, kern_ms, nl, B)

    if "fp64" in legs and args.fp64_samples > 0:
        # all-FP64 mode on the first samples of the same batch (a whole batch takes seconds)
        S64 = min(args.fp64_samples, B)
        st64 = Step(ham, ans64, x[:S64].contiguous(), w[:S64].contiguous())
        # the launch shape tuned for the BF16 kernel is a property of the handle: the FP64
        # kernel runs its built-in shape, and the tuned one is put back afterwards
        tuned_shape = min(tune_table, key=lambda r: r["ms"])["shape"] if tune_table else None
        ham.tune()
        sec64, kern64_ms, _ = st64.eager(1, 1)
        if tuned_shape:
            ham.tune(tuned_shape.get("grid", 0), tuned_shape.get("groups", 0), tuned_shape.get("waves", 0),
                     tuned_shape.get("cols", 0))
        uw = unmasked_weights(s.n, s.widths)
        out["fp64"] = {"samples": S64, "ms_per_step": sec64 * 1e3, "local_energies_per_s": S64 / sec64,
                       "h_elems_per_s": S64 * C / sec64, "eval_kernel_ms": kern64_ms,
                       "eval_kernel_tflops_alg": S64 * (C - 1) * 2 * uw / (kern64_ms * 1e-3) / 1e12,
                       "peak_tflops": PEAK_F64_TFLOPS,
                       "frac": S64 * (C - 1) * 2 * uw / (kern64_ms * 1e-3) / 1e12 / PEAK_F64_TFLOPS,
                       "bf16_over_fp64_speed": (B / sec) / (S64 / sec64),
                       "note": "first samples of the headline batch, eval + stats + grad, eager"}
        eloc64 = st64.eloc.cpu().numpy().copy()
        del st64

    if "cpu" in legs and args.cpu_samples > 0:
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
                               "sample": f"first {S} of the {B} samples of the headline workload (each "
                                         f"{C} connected determinants through the FP64 NumPy ansatz), "
                                         f"BF16-rounded parameters; {len(os.sched_getaffinity(0))} host cores "
                                         f"visible", "seconds": t1 - t0}
        g16 = eloc16[:S, 0] + 1j * eloc16[:S, 1]
        err = {"samples": S, "bf16_max_abs_dEloc": float(np.max(np.abs(g16 - ref))),
               "bf16_abs_dE_weighted": float(abs(np.sum(p.w[:S] * g16) / p.w[:S].sum()
                                                 - np.sum(p.w[:S] * ref) / p.w[:S].sum())),
               "golden_bf16": golden_errors(cfg, p, eloc16)}
        if "fp64" in out:
            err["golden_fp64"] = golden_errors(cfg, p, eloc64, "fp64")
        out["error_vs_oracle"] = err

    # ------------------------------------------------------------------ other workloads
    for leg_cfg in (1, 3):
        key = f"c{leg_cfg}"
        if key not in legs or leg_cfg == cfg:
            continue
        lwl, lp, lham, lx, lw, la16, _ = setup(leg_cfg)
        lt = autotune.tune_eval(lham, la16, lx, reps=1, budget_s=10.0) if not args.no_autotune else None
        lst = Step(lham, la16, lx, lw)
        steps = 10 if leg_cfg == 1 else 2
        lsec_e, lkms, lnl = lst.eager(steps, 1)
        lsec = lsec_e if args.no_graph else lst.graph(steps)
        lB = lp.x.shape[0]
        le = lst.eloc.cpu().numpy()
        out[key] = {"workload": describe(lwl, lp, lham.C), "ms_per_step": lsec * 1e3,
                    "local_energies_per_s": lB / lsec, "h_elems_per_s": lB * lham.C / lsec,
                    "grad_ms": lst.grad_ms(), "roofline": roofline(leg_cfg, lp, lham.C, lkms, lnl, lB),
                    "launch_shape": (min(lt, key=lambda r: r["ms"]) if lt else None),
                    "golden_bf16": golden_errors(leg_cfg, lp, le)}
        del lst, lham

    if "c2" in legs:
        mwl = synth.WORKLOADS[2]
        probs = [synth.make_problem(2, si) for si in range(len(mwl.systems))]
        hams = [elocal.Hamiltonian(q.h1e, q.eri, q.system.n, q.system.n_alpha, q.system.n_beta) for q in probs]
        mans = [elocal.Ansatz(q.system.widths, torch.tensor(q.theta, device=dev).float().to(torch.bfloat16)
                              .contiguous(), elocal.BF16) for q in probs]
        mxs = [torch.from_numpy(q.x.view(np.int64).copy()).to(dev) for q in probs]
        mev = elocal.MultiEval()
        mt = None if args.no_autotune else autotune.tune_multi(mev, hams, mans, mxs, budget_s=10.0)
        outs, _ = mev(hams, mans, mxs)
        torch.cuda.synchronize()
        hams[0].timing(True)
        hams[0].kernel_time(reset=True)
        t0 = time.perf_counter()
        reps = 3
        for _ in range(reps):
            mev(hams, mans, mxs, outs=outs)
        torch.cuda.synchronize()
        msec = (time.perf_counter() - t0) / reps
        mkms, mnl = hams[0].kernel_time(reset=True)
        hams[0].timing(False)
        mkms /= max(mnl, 1)
        rows = sum(q.x.shape[0] * (h.C - 1) for q, h in zip(probs, hams))
        flops = sum(q.x.shape[0] * (h.C - 1) * 2.0 * unmasked_weights(q.system.n, q.system.widths)
                    for q, h in zip(probs, hams))
        pairs = sum(q.x.shape[0] * h.C for q, h in zip(probs, hams))
        nsamp = sum(q.x.shape[0] for q in probs)
        out["c2"] = {"workload": "eight systems n=12..40 step 4, half filling, 128x2, one persistent launch",
                     "samples": [q.x.shape[0] for q in probs], "connected": [h.C for h in hams],
                     "ms_per_call": msec * 1e3, "local_energies_per_s": nsamp / msec, "h_elems_per_s": pairs / msec,
                     "roofline": {"bound": "mfma", "achieved": flops / (mkms * 1e-3) / 1e12,
                                  "peak": PEAK_16BIT_TFLOPS, "unit": "TFLOP/s",
                                  "frac": flops / (mkms * 1e-3) / 1e12 / PEAK_16BIT_TFLOPS, "traffic": None,
                                  "kernel": "k_eval_multi_bf16", "kernel_ms": mkms, "rows_per_launch": rows},
                     "launch_shape": (min(mt, key=lambda r: r["ms"]) if mt else None),
                     "golden_bf16": [golden_errors(2, q, o.cpu().numpy(), system=si)
                                     for si, (q, o) in enumerate(zip(probs, outs))]}
        del hams, mans, mxs, outs

    # --- the materialising generator + matrix elements (elocal_connect) on the 24-orbital
    # batch, HBM-write-bound: algorithmic bytes per listed pair = x' (8W) + H (8) + sign (1) + exc (4)
    if "connect" in legs and args.connect_reps > 0:
        _, cp, cham, cx, _, ca16, ca64 = setup(1)
        cB, cC, W = cp.x.shape[0], cham.C, cham.W
        outs = (torch.empty((cB, cC, W), dtype=torch.int64, device=dev),
                torch.empty((cB, cC), dtype=torch.float64, device=dev),
                torch.empty((cB, cC), dtype=torch.int8, device=dev),
                torch.empty((cB, cC), dtype=torch.int32, device=dev))
        cham.connect(cx, out=outs)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        cham.timing(True)
        cham.kernel_time(reset=True)
        ev0.record()
        for _ in range(args.connect_reps):
            cham.connect(cx, out=outs)
        ev1.record()
        torch.cuda.synchronize()
        gms, gn = cham.kernel_time(reset=True)
        cham.timing(False)
        cms = ev0.elapsed_time(ev1) / args.connect_reps   # prep + generator
        gms = gms / max(gn, 1)                              # generator kernel alone
        per_pair = 8 * W + 8 + 1 + 4
        alg = cB * cC * per_pair
        out["connect"] = {"workload": "24 orbitals, 12a+12b, 16384 samples x 29737", "bound": "hbm",
                          "kernel": "k_connect_flat", "kernel_ms": gms, "call_ms": cms,
                          "pairs_per_s": cB * cC / (gms * 1e-3), "bytes_per_pair": per_pair,
                          "achieved": alg / (gms * 1e-3) / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                          "frac": alg / (gms * 1e-3) / 1e9 / PEAK_HBM_GBS,
                          "traffic": stored_traffic(CONNECT_COUNTERS, CONNECT_SRC, cB),
                          "note": "kernel_ms: library HIP events around the generator kernel; call_ms: the "
                                  "whole call (per-sample preparation + generator)"}
        del outs
        torch.cuda.empty_cache()

        # --- batch autoregressive sampling from the same 24-orbital ansatz (FP64 conditionals)
        if "sampler" in legs and args.sampler_draws > 0:
            cham.sample(ca64, 1000, 1)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            xs_, cs_ = cham.sample(ca64, args.sampler_draws, 2026)
            t_s = time.perf_counter() - t0
            # the same call at 10^12 draws on the 8-orbital ansatz: the cost follows the distinct
            # prefixes (4,900 leaves), not the draws
            sp = synth.make_problem(0)
            sham = elocal.Hamiltonian(sp.h1e, sp.eri, sp.system.n, sp.system.n_alpha, sp.system.n_beta)
            sans = elocal.Ansatz(sp.system.widths, torch.tensor(sp.theta, dtype=torch.float64, device=dev), elocal.FP64)
            sham.sample(sans, 1000, 1)
            big = {}
            for nd in (10 ** 5, 10 ** 12):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                xb, _ = sham.sample(sans, nd, 2026)
                big[nd] = (time.perf_counter() - t0, int(xb.shape[0]))
            out["sampler"] = {"workload": "24 orbitals, 12a+12b, FP64 ansatz 128x2", "draws": args.sampler_draws,
                              "distinct": int(xs_.shape[0]), "seconds": t_s,
                              "draws_per_s": args.sampler_draws / t_s, "orbital_steps": cp.system.n,
                              "n8_1e5_draws_s": big[10 ** 5][0], "n8_1e12_draws_s": big[10 ** 12][0],
                              "n8_distinct": big[10 ** 12][1],
                              "note": "multinomial split per prefix (binomial chain); one host sync per call"}
            del xs_, cs_, sham

        # --- the paper's Pauli-string route on the same ansatz and samples: every unique flip
        # of the Jordan--Wigner strings goes through the ansatz (vs the C connected ones)
        if "pauli" in legs and args.pauli_samples > 0:
            Bp = min(args.pauli_samples, cB)
            xp = cx[:Bp].contiguous()
            t0 = time.perf_counter()
            n_str, n_flip = cham.pauli_build()
            t_build = time.perf_counter() - t0
            ep = torch.empty((Bp, 2), dtype=torch.float64, device=dev)
            es = torch.empty((Bp, 2), dtype=torch.float64, device=dev)
            cham.eval_pauli(ca16, xp, out=ep)
            cham.eval(ca16, xp, out=es, want_logpsi=False)
            torch.cuda.synchronize()
            cham.timing(True)
            cham.kernel_time(reset=True)
            cham.eval_pauli(ca16, xp, out=ep)
            pms, _ = cham.kernel_time(reset=True)
            cham.eval(ca16, xp, out=es, want_logpsi=False)
            sms, _ = cham.kernel_time(reset=True)
            cham.timing(False)
            diff = float(((ep - es).norm(dim=1) / es.norm(dim=1)).max().item())
            out["pauli_route"] = {"samples": Bp, "strings": n_str, "unique_flips": n_flip, "connected": cC,
                                  "build_s": t_build, "kernel_ms": pms, "slater_condon_kernel_ms": sms,
                                  "ansatz_rows_ratio": (n_flip - 1) / (cC - 1), "time_ratio": pms / sms,
                                  "max_rel_diff_vs_slater_condon": diff}
        del cham

    # --- deduplicated evaluation (each distinct x' of the batch once) against the fused kernel,
    # on the 8-orbital workload (1024 samples x 361 listed pairs); whole calls between events
    if "dedup" in legs and args.dedup_reps > 0:
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
    if "kpm" in legs and args.kpm_moments > 0:
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

    line = {
        "metric": METRIC,
        "value": B / sec,
        "unit": "local energies/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16 params, f16x2 MFMA/f32 acc, f64 sums",
        "data": "synthetic",
        "config": {"workload": describe(wl, p, C), "orbitals": s.n, "alpha": s.n_alpha, "beta": s.n_beta,
                   "hidden": list(s.widths), "samples": B, "connected_per_sample": C,
                   "step": "eval + stats + grad"},
        "h_elems_per_s": B * C / sec,
        "grad_ms": grad_ms,
        "energy": {"re": float(stats16[0]), "im": float(stats16[1]), "var": float(stats16[2])},
        "roofline": roof,
        "timing": {"mode": "eager" if args.no_graph else "hip graph replay", "eager_ms_per_step": sec_eager * 1e3,
                   "launch_shape": ({"autotuned": True, "chosen": min(tune_table, key=lambda r: r["ms"]),
                                     "tried": len(tune_table)} if tune_table else {"autotuned": False})},
    }
    line.update(out)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
