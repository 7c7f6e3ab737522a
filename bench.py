#!/usr/bin/env python3
"""Throughput of the direct-sum force path on one MI355X, with accuracy and roofline.

Workload (default): N = 131072 equal-mass Plummer sphere (scale 1, total mass 1,
truncated at 20 scale radii, distribution-function velocities), eps = 0.4 / N^{1/3},
FP32 structure-of-arrays positions and masses, seed 2.

A step is one force + potential evaluation of all N particles (N^2 pair
interactions) with compensated FP32 accumulation and FP64 reduction.  The same
number of steps is timed with plain FP32 accumulation.  ``value`` is pair
interactions per second of the compensated path with inputs resident in HBM.

Accuracy: the CPU-baseline leg runs the FP64 oracle on the same particles (all N
i-particles, i.e. one full evaluation); its result gives the relative RMS and
maximum (eq. (3)) errors of every mode, and its wall time gives the CPU rate.

Prints one JSON line.  ``--gpus`` above 1 is refused: the path runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "pair interactions/s at N=131072, compensated vs plain FP32, error vs FP64"

# MI355X issue model: 256 CUs x 4 SIMDs, each issuing FP32 VALU work for 32 lanes per
# clock (a wave64 FP32 add/mul/FMA every 2 clocks, which is the 157.3 TFLOP/s FP32
# figure with FMA = 2 flops) at 2.4 GHz: 7.86e13 lane-operations per second.  A
# transcendental (v_rsq_f32) issues at a quarter of that rate, so it takes 4 slots.
# A pair term needs 13 FP32 VALU operations plus one v_rsq_f32: 17 slots.
CUS, SIMDS, LANES, CLOCK_HZ = 256, 4, 32, 2.4e9
LANE_ISSUE = CUS * SIMDS * LANES * CLOCK_HZ
VALU_PER_PAIR = 13
RSQ_SLOTS = 4.0
FLOPS_PER_PAIR = 20  # the paper's operation count per pair (Sec. 1.1)


def peak_pairs_per_s() -> float:
    return LANE_ISSUE / (VALU_PER_PAIR + RSQ_SLOTS)


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="plummer_131072")
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the FP64 oracle leg (no errors, no CPU rate)")
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="i-particles the oracle evaluates (0 = all N)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this path runs on one GPU; --gpus %d is not supported "
              "(the multi-GPU sharding is described, not built)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_astro_ph_0703100_amd import _lib, api, ics, metrics

    w = ics.WORKLOADS[args.workload]
    n = w.n
    pos, _vel, mass = ics.plummer(n, seed=w.seed)
    p32 = np.ascontiguousarray(pos.T.astype(np.float32))
    m32 = mass.astype(np.float32)
    eps = float(np.float32(w.eps))
    dev = torch.device("cuda:0")
    p = torch.from_numpy(p32).to(dev)
    m = torch.from_numpy(m32).to(dev)
    acc = torch.empty((3, n), dtype=torch.float64, device=dev)
    pot = torch.empty(n, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    sp = stream.cuda_stream
    pairs = float(n) * float(n)

    def run_mode(precision: str, steps: int, warmup: int):
        opts = api.make_opts(precision=precision)
        for _ in range(warmup):
            _lib.nbody_force_ex(n, p.data_ptr(), m.data_ptr(), eps, acc.data_ptr(), pot.data_ptr(),
                                opts, sp)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            ev[k][0].record(stream)
            _lib.nbody_force_ex(n, p.data_ptr(), m.data_ptr(), eps, acc.data_ptr(), pot.data_ptr(),
                                opts, sp)
            ev[k][1].record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        kms = [a.elapsed_time(b) for a, b in ev]
        return wall, kms, acc.cpu().numpy().T.copy(), pot.cpu().numpy().copy()

    res = {}
    for precision in ("comp", "plain", "fp64red"):
        steps = args.steps if precision != "fp64red" else max(1, min(args.steps, 2))
        wall, kms, a_np, p_np = run_mode(precision, steps, args.warmup)
        res[precision] = {"wall": wall, "steps": steps, "kernel_ms": float(np.mean(kms)),
                          "kernel_ms_min": float(np.min(kms)), "acc": a_np, "pot": p_np}
        print("bench: %-8s %d steps  %.3f ms/step  kernel %.3f ms" %
              (precision, steps, wall / steps * 1e3, np.mean(kms)), file=sys.stderr, flush=True)

    comp = res["comp"]
    value = pairs * comp["steps"] / comp["wall"]
    k_ms = comp["kernel_ms"]
    achieved_tf = pairs * FLOPS_PER_PAIR / (k_ms * 1e-3) / 1e12
    peak_tf = peak_pairs_per_s() * FLOPS_PER_PAIR / 1e12

    cpu = None
    errors = {}
    if not args.no_cpu_baseline:
        import oracle
        k = n if args.cpu_sample <= 0 else min(n, args.cpu_sample)
        idx = np.arange(n) if k == n else ics.sample_indices(n, k, seed=w.seed + 1000)
        x64 = p32.T.astype(np.float64)
        t0 = time.perf_counter()
        ra, rp = oracle.force_sampled(x64, m32.astype(np.float64), eps, idx)
        ct = time.perf_counter() - t0
        cpu = {"value": k * float(n) / ct, "unit": "pair-interactions/s",
               "cores": oracle.threads(), "kind": "oracle",
               "sample": "%d i-particles x %d j-particles of the same sphere, FP64, one "
                         "force+potential evaluation (%.1f s)" % (k, n, ct)}
        for precision, r in res.items():
            ea = metrics.rel_errors(r["acc"][idx], ra)
            ep = metrics.rel_errors(r["pot"][idx], rp)
            errors[precision] = {"acc_rel_rms": ea["rel_rms"], "acc_e_max": ea["e_max"],
                                 "acc_normwise": ea["normwise"], "pot_rel_rms": ep["rel_rms"],
                                 "pot_e_max": ep["e_max"], "sample": int(idx.size)}

    plain = res["plain"]
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "pair-interactions/s",
        "n_gpus": 1,
        "steps": comp["steps"],
        "warmup": args.warmup,
        "ms_per_step": comp["wall"] / comp["steps"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "n": n, "eps": eps, "seed": w.seed,
                   "precision": "comp", "step": "one force+potential evaluation (N^2 pairs)",
                   "description": w.description},
        "roofline": {"bound": "alu", "achieved": achieved_tf, "peak": peak_tf, "unit": "TFLOP/s",
                     "frac": achieved_tf / peak_tf, "traffic": None,
                     "kernel": "pair_kernel + finalize", "kernel_ms": k_ms,
                     "flops_per_pair": FLOPS_PER_PAIR,
                     "issue_slots_per_pair": VALU_PER_PAIR + RSQ_SLOTS},
        "cpu_baseline": cpu,
        "plain": {"value": pairs * plain["steps"] / plain["wall"],
                  "ms_per_step": plain["wall"] / plain["steps"] * 1e3,
                  "kernel_ms": plain["kernel_ms"]},
        "fp64red": {"kernel_ms": res["fp64red"]["kernel_ms"]},
        "errors": errors,
        "gflops_38": metrics.gflops(pairs, k_ms * 1e-3, 38),
        "gflops_20": metrics.gflops(pairs, k_ms * 1e-3, 20),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
