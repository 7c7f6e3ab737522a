#!/usr/bin/env python3
"""Throughput of the direct-sum gravity path on one MI355X, with accuracy and roofline.

Workload (default ``plummer_131072``): N = 131072 equal-mass Plummer sphere (scale 1,
total mass 1, truncated at 20 scale radii, distribution-function velocities), seed 2,
eps = 0.4 / N^{1/3}, FP32 masses, FP64 positions and velocities.

A step is one kick-drift-kick leapfrog step (dt = 1/256) replayed from a HIP graph:
first kick + drift (FP64), FP64 centre, FP32 conversion, pair kernel (N^2 pair
interactions: accelerations and potentials, compensated FP32 accumulation), FP64
reduction fused with the second kick.  ``value`` is N^2 * steps / wall time (pair interactions per second, inputs
resident in HBM).  The same is timed with plain FP32 accumulation.

Roofline: the pair kernel (plus its FP64 finalize) is timed with HIP events around
standalone force evaluations on the same stream, and compared with the issue limit
of 17 VALU slots per pair.

Accuracy: the CPU-baseline leg runs the FP64 oracle on the initial positions (all N
i-particles by default); its result gives the relative RMS and maximum (eq. (3))
errors of each mode's force evaluation, and its wall time the CPU rate.

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
    ap.add_argument("--modes", default="comp,plain,fp64red")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="run one device-to-device copy of this many MiB first (a plain copy "
                         "kernel of known size, to calibrate hardware byte counters)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this path runs on one GPU; --gpus %d is not supported "
              "(the multi-GPU sharding is described in DESIGN.md, not built)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_astro_ph_0703100_amd import _lib, api, ics, metrics

    w = ics.WORKLOADS[args.workload]
    n = w.n
    dt = w.dt or 1.0 / 256
    pos, vel, mass = ics.plummer(n, seed=w.seed)
    m32 = mass.astype(np.float32)
    eps = float(np.float32(w.eps))
    dev = torch.device("cuda:0")
    x0 = torch.from_numpy(np.ascontiguousarray(pos.T)).to(dev)
    v0 = torch.from_numpy(np.ascontiguousarray(vel.T)).to(dev)
    m = torch.from_numpy(m32).to(dev)
    p32 = torch.from_numpy(np.ascontiguousarray(pos.T.astype(np.float32))).to(dev)
    stream = torch.cuda.current_stream()
    sp = stream.cuda_stream
    pairs = float(n) * float(n)
    modes = [s for s in args.modes.split(",") if s]

    def timed_steps(precision: str):
        """K graph-replayed KDK steps from the initial state; wall time and per-step ms."""
        x, v = x0.clone(), v0.clone()
        acc, _, _ = api.leapfrog(x, v, m, eps, dt, 0, precision=precision)
        pot = torch.empty(n, dtype=torch.float64, device=dev)
        g = api.LeapfrogGraph(x, v, m, eps, dt, 1, acc, pot=pot, precision=precision)
        for _ in range(args.warmup):
            g.launch()
        torch.cuda.synchronize()
        x.copy_(x0)
        v.copy_(v0)
        api.leapfrog(x, v, m, eps, dt, 0, acc=acc, precision=precision)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            ev[k][0].record(stream)
            g.launch()
            ev[k][1].record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        g.close()
        return wall, [a.elapsed_time(b) for a, b in ev]

    def timed_force(precision: str, reps: int):
        """Events around standalone force evaluations (pair kernel + FP64 finalize)."""
        acc = torch.empty((3, n), dtype=torch.float64, device=dev)
        pot = torch.empty(n, dtype=torch.float64, device=dev)
        opts = api.make_opts(precision=precision)
        call = lambda: _lib.nbody_force_ex(n, p32.data_ptr(), m.data_ptr(), eps, acc.data_ptr(),
                                           pot.data_ptr(), opts, sp)
        call()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(reps)]
        torch.cuda.synchronize()
        for k in range(reps):
            ev[k][0].record(stream)
            call()
            ev[k][1].record(stream)
        torch.cuda.synchronize()
        return [a.elapsed_time(b) for a, b in ev]

    def force_f64(precision: str):
        acc, pot = api.force_f64(x0, m, eps, precision=precision)
        torch.cuda.synchronize()
        return acc.cpu().numpy().T.copy(), pot.cpu().numpy().copy()

    if args.calib_copy_mb > 0:
        nb = args.calib_copy_mb * (1 << 20) // 4
        src = torch.ones(nb, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    res = {}
    for precision in modes:
        wall, step_ms = timed_steps(precision)
        kms = timed_force(precision, max(args.steps, 3))
        a_np, p_np = force_f64(precision)
        res[precision] = {"wall": wall, "step_ms": step_ms, "kernel_ms": float(np.mean(kms)),
                          "acc": a_np, "pot": p_np}
        print("bench: %-8s %d steps  %.3f ms/step (wall)  force kernel %.3f ms" %
              (precision, args.steps, wall / args.steps * 1e3, np.mean(kms)),
              file=sys.stderr, flush=True)

    cpu = None
    errors = {}
    if not args.no_cpu_baseline:
        import oracle
        k = n if args.cpu_sample <= 0 else min(n, args.cpu_sample)
        idx = np.arange(n) if k == n else ics.sample_indices(n, k, seed=w.seed + 1000)
        t0 = time.perf_counter()
        ra, rp = oracle.force_sampled(pos, m32.astype(np.float64), eps, idx)
        ct = time.perf_counter() - t0
        cpu = {"value": k * float(n) / ct, "unit": "pair-interactions/s",
               "cores": oracle.threads(), "kind": "oracle",
               "sample": "force+potential of %d i-particles from all %d particles of the same "
                         "sphere at the initial positions, FP64 (%.1f s)" % (k, n, ct)}
        for precision, r in res.items():
            ea = metrics.rel_errors(r["acc"][idx], ra)
            ep = metrics.rel_errors(r["pot"][idx], rp)
            errors[precision] = {"acc_rel_rms": ea["rel_rms"], "acc_e_max": ea["e_max"],
                                 "acc_normwise": ea["normwise"], "pot_rel_rms": ep["rel_rms"],
                                 "pot_e_max": ep["e_max"], "sample": int(idx.size)}

    head = modes[0]
    r0 = res[head]
    k_ms = r0["kernel_ms"]
    achieved_tf = pairs * FLOPS_PER_PAIR / (k_ms * 1e-3) / 1e12
    peak_tf = peak_pairs_per_s() * FLOPS_PER_PAIR / 1e12
    line = {
        "metric": METRIC,
        "value": pairs * args.steps / r0["wall"],
        "unit": "pair-interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r0["wall"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "n": n, "eps": eps, "seed": w.seed, "dt": dt,
                   "precision": head,
                   "step": "one graph-replayed KDK leapfrog step: FP64 state, FP32 pair "
                           "arithmetic relative to the system centre, one N^2 force+potential "
                           "evaluation",
                   "description": w.description},
        "roofline": {"bound": "alu", "achieved": achieved_tf, "peak": peak_tf, "unit": "TFLOP/s",
                     "frac": achieved_tf / peak_tf, "traffic": None,
                     "kernel": "pair_kernel (+ finalize_kernel, <0.3%)", "kernel_ms": k_ms,
                     "flops_per_pair": FLOPS_PER_PAIR,
                     "issue_slots_per_pair": VALU_PER_PAIR + RSQ_SLOTS,
                     "peak_pairs_per_s": peak_pairs_per_s()},
        "cpu_baseline": cpu,
        "modes": {p: {"value": pairs * args.steps / r["wall"],
                      "ms_per_step": r["wall"] / args.steps * 1e3,
                      "step_ms_events": float(np.mean(r["step_ms"])),
                      "force_kernel_ms": r["kernel_ms"],
                      "roofline_frac": pairs / (r["kernel_ms"] * 1e-3) / peak_pairs_per_s(),
                      "errors": errors.get(p)} for p, r in res.items()},
        "gflops_38": metrics.gflops(pairs, k_ms * 1e-3, 38),
        "gflops_20": metrics.gflops(pairs, k_ms * 1e-3, 20),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
