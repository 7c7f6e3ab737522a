#!/usr/bin/env python3
"""Throughput of the direct-sum gravity path on one MI355X, with accuracy and roofline.

Default workload ``plummer_131072``: N = 131072 equal-mass Plummer sphere (scale 1,
total mass 1, truncated at 20 scale radii, distribution-function velocities), seed 2,
eps = 0.4 / N^{1/3}, FP32 masses, FP64 positions and velocities.  A step is one
kick-drift-kick leapfrog step (dt = 1/256) replayed from a HIP graph: first kick +
drift (FP64), FP64 centre, FP32 conversion, pair kernel (N^2 pair interactions:
accelerations and potentials, compensated FP32 accumulation), FP64 reduction fused
with the second kick.  ``value`` is N^2 * steps / wall time (pair interactions per
second, inputs resident in HBM).  The same is timed with plain FP32 accumulation and
with FP64-reduced accumulation ("modes").

The default run also measures the other configurations of the workload set and puts
one compact entry per configuration into ``configs`` (same units; each with its own
accuracy against the FP64 oracle on the configuration's stated sample):
  plummer_2048   N = 2048 sphere, v = 0, eps = 1/64: one force+potential evaluation,
                 every mode, oracle on all N^2 pairs.
  stress_1m      2^20-particle precision-stress system at (1000,0,0), Morton-ordered:
                 one evaluation from FP64 positions, modes x reference centres (none,
                 system, tile), oracle on 4096 stratified particles, and the same
                 oracle on the FP32-rounded inputs the kernel saw (representation
                 error apart from arithmetic error).
  clusters_2048  2048 ragged Plummer clusters: one graph-replayed batched KDK step
                 (persistent work-queue kernel); pairs = sum N_k^2; 16 systems checked
                 (acceleration and potential) at step 0 and after the timed steps.
  adjoint_16384  N = 16384, 32 KDK steps dt = 1/256 and the reverse pass: one loss +
                 gradient (33 force and 33 adjoint evaluations of N^2 pairs).
``--no-configs`` leaves them out; ``--workload`` runs one of them (or the secondary
workloads shard8_131072, active8_131072, jerk_131072) as the whole line.

Roofline: the dominant kernel's duration is taken from HIP events on the launch
stream (standalone calls) and its algorithmic work (20 flop per gravity pair, the
paper's count; 60 per force-jerk-potential pair; 45 per adjoint pair) is compared
with the published FP32 vector peak of the MI355X, 157.3 TFLOP/s (``frac``).  Beside
it, ``issue_model`` compares the pair rate with the VALU issue limit of the pair body:
13 FP32 VALU instructions at 32 lanes per clock and one quarter-rate v_rsq_f32 (17
issue slots per gravity pair; 31 per force-jerk-potential pair, 35 per adjoint pair)
at 256 CUs x 4 SIMDs x 2.4 GHz.  ``traffic`` comes from the committed rocprofv3
counter summary of the same kernel and is null when its sources changed since.

Accuracy: the CPU-baseline leg runs the FP64 oracle on a bounded sample of the same
workload; its result gives the relative RMS and maximum (eq. (3)) errors of each
mode, and its wall time the CPU rate.

Warm-up: unless ``--warmup`` is given, each timed loop is preceded by enough untimed
steps to keep the GPU busy for about a quarter of a second (``warmup`` in the line is
the count of the headline mode), so the timed steps run at the steady rate.

Prints one JSON line.  ``--gpus`` above 1 is refused: the path runs on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "pair interactions/s at N=131072, compensated vs plain FP32, error vs FP64"

# Published FP32 vector peak of the MI355X (FMA = 2 flops), the roofline's peak.
FP32_VECTOR_PEAK_TFLOPS = 157.3
# Issue model of the pair bodies: 256 CUs x 4 SIMDs, FP32 VALU work for 32 lanes per
# clock (a wave64 instruction every 2 clocks; 157.3 TFLOP/s is that rate with FMA = 2
# flops) at 2.4 GHz; a transcendental (v_rsq_f32) issues at a quarter of that rate and
# takes 4 slots.  The pair kernel's own counters bear the model out (its committed
# summary: 0.35 VALU wave-instructions per SIMD per cycle, above the 0.25 a 4-clock
# wave64 issue allows).
CUS, SIMDS, LANES, CLOCK_HZ = 256, 4, 32, 2.4e9
LANE_ISSUE = CUS * SIMDS * LANES * CLOCK_HZ
RSQ_SLOTS = 4
SLOTS = {"gravity": 13 + RSQ_SLOTS, "jerk": 27 + RSQ_SLOTS, "adjoint": 31 + RSQ_SLOTS}
# Flops per pair: the paper's count for gravity (Sec. 1.1); 60 for force, jerk and
# potential, the count customary for fourth-order Hermite codes; 45 for the adjoint.
FLOPS = {"gravity": 20, "jerk": 60, "adjoint": 45}

# The files that define the pair kernel tile_kernel<Gravity> (force.hip only instantiates
# it; its own kernels are the finalize and centre passes), and the tuning file whose
# force-kernel entries for N = 131072 (size bucket 17) pick the launch shape; the
# committed counter record is dropped when either changes.
KERNEL_SOURCES = ["paper_astro_ph_0703100_amd/csrc/nbody_internal.h",
                  "paper_astro_ph_0703100_amd/csrc/tile_engine.h",
                  "paper_astro_ph_0703100_amd/csrc/gravity.h"]
TUNING_FILE = "paper_astro_ph_0703100_amd/tuning_gfx950.json"
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "pair_kernel_plummer_131072.md")
CONFIG_WORKLOADS = ("plummer_2048", "stress_1m", "clusters_2048", "adjoint_16384")


def peak_pairs(kind: str) -> float:
    """Pair rate of the issue model for a pipeline (pairs/s at the 2.4 GHz spec clock)."""
    return LANE_ISSUE / SLOTS[kind]


_TOKEN = re.compile(r'"(?:\\.|[^"\\\n])*"|\'(?:\\.|[^\'\\\n])*\'|//[^\n]*|/\*.*?\*/', re.S)


def code_text(src: str) -> str:
    """C++ source with its comments removed and its whitespace collapsed: what a change to
    the kernel's code changes, and a change to its comments does not."""
    code = _TOKEN.sub(lambda t: t.group(0) if t.group(0)[0] in "\"'" else " ", src)
    return " ".join(code.split())


def sources_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel)) as f:
            h.update(code_text(f.read()).encode())
    with open(os.path.join(ROOT, TUNING_FILE)) as f:
        force = [e for e in json.load(f)["entries"]
                 if e.get("kernel") == 0 and e.get("bucket") == 17]
    h.update(json.dumps(sorted(force, key=lambda e: (e["precision"], e["bucket"])),
                        sort_keys=True).encode())
    return h.hexdigest()[:16]


def committed_record():
    """The counter record of the pair kernel in the committed summary (HBM bytes per launch,
    sustained clock), or None when the kernel sources or shape changed since."""
    try:
        text = open(TRAFFIC_SUMMARY).read()
    except OSError:
        return None
    m = re.search(r"<!-- traffic: (\{.*?\}) -->", text)
    if not m:
        return None
    rec = json.loads(m.group(1))
    return rec if rec.get("sources_hash") == sources_hash() else None


def committed_traffic():
    """HBM bytes per launch of the pair kernel from the committed counter summary, or None."""
    rec = committed_record()
    return rec["bytes_per_launch"] if rec else None


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def parse(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed warm-up steps (default: enough to keep the GPU busy for "
                         "about %.2f s, at least 2)" % WARM_SECONDS)
    ap.add_argument("--workload", default="plummer_131072",
                    choices=["plummer_131072", "plummer_2048", "stress_1m", "clusters_2048",
                             "adjoint_16384", "jerk_131072", "shard8_131072",
                             "active8_131072"])
    ap.add_argument("--no-configs", action="store_true",
                    help="measure only the selected workload (no per-configuration entries)")
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the FP64 oracle leg (no errors, no CPU rate)")
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="i-particles the oracle evaluates (0 = the workload's default)")
    ap.add_argument("--modes", default="comp,plain,fp64red")
    ap.add_argument("--symmetric", action="store_true",
                    help="run the N = 131072 workload on the opt-in symmetric engine (each "
                         "unordered pair once) instead of the library's default shape")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="first run one device-to-device copy of this many MiB from a source "
                         "evicted from the caches (a plain copy kernel of known size, to "
                         "calibrate hardware byte counters)")
    return ap.parse_args(argv)


class Timer:
    """HIP events around calls on the current stream."""

    def __init__(self, torch):
        self.torch = torch
        self.stream = torch.cuda.current_stream()

    def run(self, call, reps, warmup=None):
        torch = self.torch
        warm_up(torch, call, warmup)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(reps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for a, b in ev:
            a.record(self.stream)
            call()
            b.record(self.stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return wall, [a.elapsed_time(b) for a, b in ev]


WARM_SECONDS = 0.25
WARMED = []
GRAPH_CALLS = 50    # evaluations per graph replay in the small-system timing
GRAPH_REPLAYS = 40  # timed replays; the median is reported (a replay's 50 launches are
                    # submitted by the host, whose pace varies from run to run)


def warm_up(torch, call, count):
    """Untimed warm-up calls: ``count`` of them, or, for ``count=None``, as many as keep the
    GPU busy for about WARM_SECONDS (at least two).  Launches shorter than a millisecond
    reach their steady rate only after tens of milliseconds of continuous load (the 1/8
    shard of N = 131072: 0.76 ms per evaluation for the first few, 0.65 ms after 50 ms).
    Returns the number of calls made, also appended to WARMED."""
    if count is not None:
        for _ in range(count):
            call()
        torch.cuda.synchronize()
        WARMED.append(count)
        return count
    call()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    call()
    torch.cuda.synchronize()
    more = max(0, int(np.ceil(WARM_SECONDS / max(time.perf_counter() - t0, 1e-6))) - 2)
    for _ in range(more):
        call()
    torch.cuda.synchronize()
    WARMED.append(more + 2)
    return more + 2


def one_thread(cpu, call, pairs, what):
    """Add the oracle's single-thread rate on a smaller piece of the same work to ``cpu``."""
    import oracle
    old = oracle.set_threads(1)
    try:
        t0 = time.perf_counter()
        call()
        ct = time.perf_counter() - t0
    finally:
        oracle.set_threads(old)
    cpu["value_1_thread"] = pairs / ct
    cpu["sample_1_thread"] = "%s (%.2f s)" % (what, ct)


def cpu_entry(value, sample):
    import oracle
    return {"value": value, "unit": "pair-interactions/s", "cores": oracle.threads(),
            "cpu_model": cpu_model(), "kind": "oracle", "sample": sample}


def errors_of(metrics, acc, pot, ra, rp):
    ea = metrics.rel_errors(acc, ra)
    out = {"acc_rel_rms": ea["rel_rms"], "acc_e_max": ea["e_max"], "acc_normwise": ea["normwise"],
           "sample": int(ea["count"])}
    if pot is not None:
        ep = metrics.rel_errors(pot, rp)
        out.update({"pot_rel_rms": ep["rel_rms"], "pot_e_max": ep["e_max"]})
    return out


def roofline(kind, pairs_per_launch, kernel_ms, kernel_name, traffic=None):
    """Roofline of one kernel: algorithmic TFLOP/s against the published FP32 vector peak
    (``frac``), and the pair rate against the issue model (``issue_model``)."""
    pairs_s = pairs_per_launch / (kernel_ms * 1e-3)
    achieved = pairs_s * FLOPS[kind] / 1e12
    return {"bound": "alu", "achieved": achieved, "peak": FP32_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": achieved / FP32_VECTOR_PEAK_TFLOPS, "traffic": traffic,
            "kernel": kernel_name, "kernel_ms": kernel_ms, "flops_per_pair": FLOPS[kind],
            "pairs_per_s": pairs_s,
            "issue_model": {"peak_pairs_per_s": peak_pairs(kind),
                            "peak_tflops": peak_pairs(kind) * FLOPS[kind] / 1e12,
                            "issue_slots_per_pair": SLOTS[kind],
                            "frac": pairs_s / peak_pairs(kind)}}


def fractions(kind, pairs_per_launch, kernel_ms):
    """Both roofline fractions of one kernel timing (compact form)."""
    r = roofline(kind, pairs_per_launch, kernel_ms, "")
    return {"kernel_ms": kernel_ms, "pairs_per_s": r["pairs_per_s"], "frac": r["frac"],
            "issue_frac": r["issue_model"]["frac"]}


def modes_of(args):
    return [s for s in args.modes.split(",") if s]


# --------------------------------------------------------------------------- workloads
def bench_plummer(args, torch, w):
    """The headline: graph-replayed KDK steps of the N = 131072 sphere, every mode."""
    from paper_astro_ph_0703100_amd import _lib, api, ics, metrics
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
    sp = torch.cuda.current_stream().cuda_stream
    timer = Timer(torch)
    pairs = float(n) * float(n)
    eng = dict(symmetric=2) if args.symmetric else {}
    res = {}
    for precision in modes_of(args):
        x, v = x0.clone(), v0.clone()
        acc, _, _ = api.leapfrog(x, v, m, eps, dt, 0, precision=precision, **eng)
        pot = torch.empty(n, dtype=torch.float64, device=dev)
        g = api.LeapfrogGraph(x, v, m, eps, dt, 1, acc, pot=pot, precision=precision, **eng)
        warm_up(torch, g.launch, args.warmup)
        x.copy_(x0)
        v.copy_(v0)
        api.leapfrog(x, v, m, eps, dt, 0, acc=acc, precision=precision, **eng)
        wall, step_ms = timer.run(g.launch, args.steps, warmup=0)
        g.close()
        fa = torch.empty((3, n), dtype=torch.float64, device=dev)
        fp = torch.empty(n, dtype=torch.float64, device=dev)
        opts = api.make_opts(precision=precision, **eng)
        _, kms = timer.run(lambda: _lib.nbody_force_ex(n, p32.data_ptr(), m.data_ptr(), eps,
                                                       fa.data_ptr(), fp.data_ptr(), opts, sp),
                           max(args.steps, 3), warmup=args.warmup)
        a64, p64 = api.force_f64(x0, m, eps, precision=precision, **eng)
        torch.cuda.synchronize()
        res[precision] = {"wall": wall, "step_ms": step_ms, "kernel_ms": float(np.mean(kms)),
                          "acc": a64.cpu().numpy().T.copy(), "pot": p64.cpu().numpy().copy()}
        print("bench: %-8s %d steps  %.3f ms/step (wall)  force kernel %.3f ms"
              % (precision, args.steps, wall / args.steps * 1e3, np.mean(kms)),
              file=sys.stderr, flush=True)
    cpu, errors = None, {}
    if not args.no_cpu_baseline:
        import oracle
        k = n if args.cpu_sample <= 0 else min(n, args.cpu_sample)
        idx = np.arange(n) if k == n else ics.sample_indices(n, k, seed=w.seed + 1000)
        t0 = time.perf_counter()
        ra, rp = oracle.force_sampled(pos, m32.astype(np.float64), eps, idx)
        ct = time.perf_counter() - t0
        cpu = cpu_entry(k * pairs / n / ct,
                        "force+potential of %d i-particles from all %d particles of the same "
                        "sphere at the initial positions, FP64 (%.1f s)" % (k, n, ct))
        i1 = ics.sample_indices(n, 512, seed=w.seed + 2000)
        one_thread(cpu, lambda: oracle.force_sampled(pos, m32.astype(np.float64), eps, i1),
                   512.0 * n, "force+potential of 512 sampled i-particles from all %d" % n)
        for p, r in res.items():
            errors[p] = errors_of(metrics, r["acc"][idx], r["pot"][idx], ra, rp)
    head = next(iter(res))
    r0 = res[head]
    # The committed counter record is the grid engine's pair kernel.
    rec = None if args.symmetric else committed_record()
    kname = ("sym_kernel (+ sym_finalize_kernel), each unordered pair once" if args.symmetric
             else "tile_kernel<Gravity> (+ finalize_kernel)")
    roof = roofline("gravity", pairs, r0["kernel_ms"], kname,
                    rec["bytes_per_launch"] if rec else None)
    if rec and rec.get("sustained_clock_ghz"):
        # The issue model at the engine clock the counters measured under this load.
        roof["issue_model"]["sustained_clock_ghz"] = rec["sustained_clock_ghz"]
        roof["issue_model"]["frac_at_sustained_clock"] = (
            roof["issue_model"]["frac"] * CLOCK_HZ / (rec["sustained_clock_ghz"] * 1e9))
    return {
        "value": pairs * args.steps / r0["wall"], "ms_per_step": r0["wall"] / args.steps * 1e3,
        "config": {"workload": w.name, "n": n, "eps": eps, "seed": w.seed, "dt": dt,
                   "precision": head, "engine": "symmetric" if args.symmetric else "default",
                   "step": "one graph-replayed KDK leapfrog step: FP64 state, FP32 pair "
                           "arithmetic relative to the system centre, one N^2 force+potential "
                           "evaluation", "description": w.description},
        "roofline": roof,
        "cpu_baseline": cpu,
        "modes": {p: {"value": pairs * args.steps / r["wall"],
                      "ms_per_step": r["wall"] / args.steps * 1e3,
                      "step_ms_events": float(np.mean(r["step_ms"])),
                      "force_kernel_ms": r["kernel_ms"],
                      **{"roofline_" + k: v for k, v in
                         fractions("gravity", pairs, r["kernel_ms"]).items()
                         if k in ("frac", "issue_frac")},
                      "errors": errors.get(p)} for p, r in res.items()},
        "gflops_38": pairs * 38 / (r0["kernel_ms"] * 1e-3) / 1e9,
        "gflops_20": pairs * 20 / (r0["kernel_ms"] * 1e-3) / 1e9,
        # The paper's Table 3 at the same N on a GeForce 8800GTX (2.548 s per force call
        # including host transfers, eps^2 = 0.01, no potential): context only, another
        # machine and not the same workload, hence vs_baseline stays null.
        "paper_context": {"pairs_per_s": 131072.0 ** 2 / 2.548, "gflops_38": 256.0,
                          "ratio": pairs * args.steps / r0["wall"] / (131072.0 ** 2 / 2.548)},
    }


def bench_small(args, torch, w):
    """N = 2048 sphere: one force+potential evaluation per step (FP32 inputs), every mode,
    against the oracle on all N^2 pairs.  A step is timed inside a HIP graph of
    GRAPH_CALLS back-to-back evaluations (the GPU's own rate: from Python each eager call
    costs about 8 us of host time, more than the evaluation); the eager per-call time is
    reported beside it."""
    from paper_astro_ph_0703100_amd import _lib, api, ics, metrics
    n = w.n
    pos, _, mass = ics.plummer(n, seed=w.seed, velocities=False)
    p32 = np.ascontiguousarray(pos.T.astype(np.float32))
    m32 = mass.astype(np.float32)
    eps = float(np.float32(w.eps))
    dev = torch.device("cuda:0")
    p, m = torch.from_numpy(p32).to(dev), torch.from_numpy(m32).to(dev)
    acc = torch.empty((3, n), dtype=torch.float64, device=dev)
    pot = torch.empty(n, dtype=torch.float64, device=dev)
    sp = torch.cuda.current_stream().cuda_stream
    timer = Timer(torch)
    pairs = float(n) * n
    reps = max(args.steps, 200)
    res = {}
    side = torch.cuda.Stream()
    for precision in modes_of(args):
        shape = _lib.nbody_tune_get(_lib.NBODY_KERNEL_FORCE, _lib.PRECISIONS[precision], n)
        opts = api.make_opts(precision=precision)
        ws = torch.empty(max(_lib.nbody_workspace_size(n, opts), 256), dtype=torch.uint8,
                         device=dev)
        gopts = api.make_opts(precision=precision, workspace=ws)
        call = lambda: _lib.nbody_force_ex(n, p.data_ptr(), m.data_ptr(), eps, acc.data_ptr(),
                                           pot.data_ptr(), opts, sp)
        _, kms = timer.run(call, reps, warmup=args.warmup)
        eager_ms = float(np.mean(kms))
        res_eager = (acc.cpu().numpy().T.copy(), pot.cpu().numpy().copy())
        # the same evaluations replayed from a graph
        graph = torch.cuda.CUDAGraph()
        torch.cuda.synchronize()
        with torch.cuda.stream(side):
            with torch.cuda.graph(graph, stream=side):
                for _ in range(GRAPH_CALLS):
                    _lib.nbody_force_ex(n, p.data_ptr(), m.data_ptr(), eps, acc.data_ptr(),
                                        pot.data_ptr(), gopts, side.cuda_stream)
        torch.cuda.synchronize()
        _, gms = timer.run(graph.replay, GRAPH_REPLAYS, warmup=args.warmup)
        kernel_ms = float(np.median(gms)) / GRAPH_CALLS
        graph_res = (acc.cpu().numpy().T.copy(), pot.cpu().numpy().copy())
        assert np.array_equal(graph_res[0], res_eager[0]) and \
            np.array_equal(graph_res[1], res_eager[1]), "graph replay differs from eager calls"
        res[precision] = {"kernel_ms": kernel_ms, "eager_ms": eager_ms, "shape": shape,
                          "acc": graph_res[0], "pot": graph_res[1]}
        del graph
        print("bench: %-8s N=%d  %.2f us per evaluation in a graph, %.2f us eager (shape "
              "ipl %d jtile %d nseg %d jlanes %d symmetric %d)" % ((precision, n, kernel_ms * 1e3,
                                                       eager_ms * 1e3) + tuple(shape)),
              file=sys.stderr, flush=True)
    # The launch floor: the same graph of evaluations of a one-particle system (one block,
    # no pairs), i.e. what a launch costs the GPU whatever it computes.
    one = torch.zeros((3, 1), dtype=torch.float32, device=dev)
    one_m = torch.ones(1, dtype=torch.float32, device=dev)
    graph = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        with torch.cuda.graph(graph, stream=side):
            for _ in range(GRAPH_CALLS):
                _lib.nbody_force_ex(1, one.data_ptr(), one_m.data_ptr(), eps, acc.data_ptr(),
                                    pot.data_ptr(), api.make_opts(), side.cuda_stream)
    torch.cuda.synchronize()
    _, fms = timer.run(graph.replay, GRAPH_REPLAYS, warmup=args.warmup)
    floor_ms = float(np.median(fms)) / GRAPH_CALLS
    del graph
    print("bench: launch floor (N = 1 evaluations in a graph) %.2f us" % (floor_ms * 1e3),
          file=sys.stderr, flush=True)
    cpu, errors = None, {}
    if not args.no_cpu_baseline:
        import oracle
        x64, m64 = p32.T.astype(np.float64), m32.astype(np.float64)
        t0 = time.perf_counter()
        ra, rp = oracle.force_all(x64, m64, eps)
        ct = time.perf_counter() - t0
        cpu = cpu_entry(pairs / ct, "all %d^2 pairs, FP64 (%.2f s)" % (n, ct))
        for q, r in res.items():
            errors[q] = errors_of(metrics, r["acc"], r["pot"], ra, rp)
    head = next(iter(res))
    r0 = res[head]
    kname = ("split_kernel<Gravity, ForceOut> (one launch per evaluation)" if r0["shape"][3] > 1
             else "tile_kernel<Gravity> + finalize_kernel")
    return {
        "value": pairs / (r0["kernel_ms"] * 1e-3), "ms_per_step": r0["kernel_ms"],
        "config": {"workload": w.name, "n": n, "eps": eps, "seed": w.seed, "precision": head,
                   "step": "one force+potential evaluation (nbody_force_ex, FP32 inputs), "
                           "%d per HIP graph replay" % GRAPH_CALLS,
                   "description": w.description},
        "roofline": roofline("gravity", pairs, r0["kernel_ms"], kname),
        "launch_floor_ms": floor_ms,
        "cpu_baseline": cpu,
        "modes": {q: {"ms_per_step": r["kernel_ms"], "eager_ms_per_call": r["eager_ms"],
                      "shape": dict(zip(("ipl", "jtile", "nseg", "jlanes", "symmetric"), r["shape"])),
                      **fractions("gravity", pairs, r["kernel_ms"]),
                      "errors": errors.get(q)} for q, r in res.items()},
    }


def _tile_rounded_rows(pos, centres_of, idx, itile):
    """The FP32-rounded relative positions the tile-centre kernel sees for i-particles
    ``idx``: every particle converted relative to the centre of i's tile (the FP64 mean
    of the tile, here summed by numpy: it may differ from the kernel's fixed-order sum
    in the last bit, so this is the representation error to that accuracy)."""
    out = {}
    for t in np.unique(idx // itile):
        c = centres_of(t)
        out[int(t)] = (pos - c).astype(np.float32).astype(np.float64)
    return out


def bench_stress(args, torch, w):
    """2^20 precision-stress system from FP64 positions: modes x reference centres."""
    from paper_astro_ph_0703100_amd import _lib, api, ics, metrics
    n = w.n
    pos, mass, core = ics.stress_system(n, seed=w.seed)
    dev = torch.device("cuda:0")
    perm = api.morton_order(torch.from_numpy(np.ascontiguousarray(pos.T)).to(dev))
    perm = perm.cpu().numpy().astype(np.int64)
    pos, mass, core = pos[perm], mass[perm], core[perm]
    m32 = mass.astype(np.float32)
    eps = float(np.float32(w.eps))
    x = torch.from_numpy(np.ascontiguousarray(pos.T)).to(dev)
    m = torch.from_numpy(m32).to(dev)
    timer = Timer(torch)
    pairs = float(n) * float(n)
    centres = ("tile", "system", "none")
    res = {}
    for precision in modes_of(args):
        out = {}
        for centre in centres:
            acc = torch.empty((3, n), dtype=torch.float64, device=dev)
            pot = torch.empty(n, dtype=torch.float64, device=dev)
            call = lambda: api.force_f64(x, m, eps, precision=precision, centre=centre,
                                         out=(acc, pot))
            wall, kms = timer.run(call, max(2, min(args.steps, 3)), warmup=1)
            out[centre] = {"wall": wall, "kernel_ms": float(np.mean(kms)),
                           "acc": acc.cpu().numpy().T.copy(), "pot": pot.cpu().numpy().copy()}
        res[precision] = out
        print("bench: %-8s %s" % (precision, "  ".join("%s %.2f ms" % (c, out[c]["kernel_ms"])
                                                      for c in centres)),
              file=sys.stderr, flush=True)
    cpu, errors, split = None, {}, {}
    if not args.no_cpu_baseline:
        import oracle
        m64 = m32.astype(np.float64)
        k = args.cpu_sample if args.cpu_sample > 0 else 2048
        idx = ics.stratified_indices(core, k, seed=w.seed + 1000)
        t0 = time.perf_counter()
        ra, rp = oracle.force_sampled(pos, m64, eps, idx)
        ct = time.perf_counter() - t0
        cpu = cpu_entry(idx.size * pairs / n / ct,
                        "%d stratified i-particles (half core, half halo) from all %d, FP64 "
                        "(%.1f s)" % (idx.size, n, ct))
        one_thread(cpu, lambda: oracle.force_sampled(pos, m64, eps, idx[::16]),
                   float(idx[::16].size) * n, "%d of those i-particles" % idx[::16].size)
        for p, out in res.items():
            for centre, r in out.items():
                errors["%s/%s" % (p, centre)] = errors_of(metrics, r["acc"][idx], r["pot"][idx],
                                                          ra, rp)
        # Representation error apart from arithmetic error: the oracle on the FP32-rounded
        # relative positions each centre mode hands the pair kernel.  none: fp32(x);
        # system: fp32(x - c), c the FP64 mean; tile: fp32(x - c_I) of each sampled i's
        # tile (on 256 of the sampled particles, one conversion of all N per tile).
        rounded = {"none": pos.astype(np.float32).astype(np.float64),
                   "system": (pos - pos.mean(0)).astype(np.float32).astype(np.float64)}
        for centre in ("none", "system"):
            rx = rounded[centre]
            ca, cp = oracle.force_sampled(rx, m64, eps, idx)
            rep = errors_of(metrics, ca, cp, ra, rp)
            split[centre] = {"representation": rep, "arithmetic": {
                p: errors_of(metrics, res[p][centre]["acc"][idx], res[p][centre]["pot"][idx],
                             ca, cp) for p in res}}
        itile = 256 * _lib.nbody_tune_get(0, 2, n)[0]
        sub = idx[:: max(1, idx.size // 256)]
        ta, tp = np.empty((sub.size, 3)), np.empty(sub.size)
        for t, rows in _tile_rounded_rows(pos, lambda t: pos[t * itile:(t + 1) * itile].mean(0),
                                          sub, itile).items():
            sel = np.nonzero(sub // itile == t)[0]
            a_, p_ = oracle.force_sampled(rows, m64, eps, sub[sel])
            ta[sel], tp[sel] = a_, p_
        ra_sub, rp_sub = oracle.force_sampled(pos, m64, eps, sub)
        split["tile"] = {"representation": errors_of(metrics, ta, tp, ra_sub, rp_sub),
                         "arithmetic": {p: errors_of(metrics, res[p]["tile"]["acc"][sub],
                                                     res[p]["tile"]["pot"][sub], ta, tp)
                                        for p in res},
                         "sample": int(sub.size)}
    head = next(iter(res))
    r0 = res[head]["tile"]
    return {
        "value": pairs / (r0["kernel_ms"] * 1e-3), "ms_per_step": r0["kernel_ms"],
        "config": {"workload": w.name, "n": n, "eps": eps, "seed": w.seed, "precision": head,
                   "centre": "tile (Morton order)",
                   "step": "one force+potential evaluation from FP64 positions, FP32 pair "
                           "arithmetic relative to per-i-tile FP64 centres",
                   "description": w.description},
        "roofline": roofline("gravity", pairs, r0["kernel_ms"],
                             "tile_kernel<GravityTile> (+ centres, finalize)"),
        "cpu_baseline": cpu,
        "modes": {"%s/%s" % (p, c): {"ms_per_step": r["kernel_ms"],
                                     **fractions("gravity", pairs, r["kernel_ms"]),
                                     "errors": errors.get("%s/%s" % (p, c))}
                  for p, out in res.items() for c, r in out.items()},
        "error_split": split or None,
    }


def bench_clusters(args, torch, w):
    """2048 ragged clusters: graph-replayed batched KDK steps (persistent kernel)."""
    from paper_astro_ph_0703100_amd import api, ics, metrics
    b = ics.cluster_batch(w.n, seed=w.seed, eps=w.eps)
    dev = torch.device("cuda:0")
    m32 = b.mass.astype(np.float32)
    epsk = b.eps.astype(np.float32)
    x0 = torch.from_numpy(np.ascontiguousarray(b.pos.T)).to(dev)
    v0 = torch.from_numpy(np.ascontiguousarray(b.vel.T)).to(dev)
    m = torch.from_numpy(m32).to(dev)
    e = torch.from_numpy(epsk).to(dev)
    p32 = torch.from_numpy(np.ascontiguousarray(b.pos.T.astype(np.float32))).to(dev)
    timer = Timer(torch)
    res = {}
    pairs = None
    for precision in modes_of(args):
        plan = api.BatchPlan(b.offsets, precision=precision)
        info = plan.info()
        pairs = float(info["pairs"])
        x, v = x0.clone(), v0.clone()
        acc, pot0 = plan.leapfrog(x, v, m, e, w.dt, 0, with_pot=True)
        a0 = acc.cpu().numpy().T.copy()
        p0 = pot0.cpu().numpy().copy()
        pot = torch.empty_like(pot0)
        g = plan.graph(x, v, m, e, w.dt, 1, acc, pot)
        warm_up(torch, g.launch, args.warmup)
        x.copy_(x0)
        v.copy_(v0)
        plan.leapfrog(x, v, m, e, w.dt, 0, acc=acc)
        wall, step_ms = timer.run(g.launch, args.steps, warmup=0)
        g.close()
        torch.cuda.synchronize()
        res[precision] = {"wall": wall, "step_ms": step_ms, "info": info,
                          "a0": a0, "p0": p0, "aT": acc.cpu().numpy().T.copy(),
                          "pT": pot.cpu().numpy().copy(), "xT": x.cpu().numpy().T.copy()}
        _, kms = timer.run(lambda: plan.force(p32, m, e), max(args.steps, 3), warmup=args.warmup)
        res[precision]["kernel_ms"] = float(np.mean(kms))
        plan.close()
        print("bench: %-8s %d steps  %.3f ms/step  batched force %.3f ms  %s"
              % (precision, args.steps, wall / args.steps * 1e3, np.mean(kms), info),
              file=sys.stderr, flush=True)
    cpu, errors = None, {}
    if not args.no_cpu_baseline:
        import oracle
        rng = np.random.default_rng(w.seed + 1000)
        pick = sorted(set([int(np.argmin(b.sizes)), int(np.argmax(b.sizes))] +
                          list(rng.choice(b.nsys, size=14, replace=False))))
        sel = np.concatenate([np.arange(b.offsets[k], b.offsets[k + 1]) for k in pick])

        def refs(pos):
            out = [oracle.force_all(pos[b.offsets[k]:b.offsets[k + 1]],
                                    m32[b.offsets[k]:b.offsets[k + 1]].astype(np.float64),
                                    float(epsk[k])) for k in pick]
            return np.concatenate([a for a, _ in out]), np.concatenate([p for _, p in out])

        t0 = time.perf_counter()
        ra0, rp0 = refs(b.pos)
        ct = time.perf_counter() - t0
        cpairs = float(sum(int(b.sizes[k]) ** 2 for k in pick))
        cpu = cpu_entry(cpairs / ct, "%d of the clusters (incl. smallest and largest), %.3g "
                                     "pairs, FP64 (%.1f s)" % (len(pick), cpairs, ct))
        for p, r in res.items():
            raT, rpT = refs(r["xT"])
            errors[p] = {"step0": errors_of(metrics, r["a0"][sel], r["p0"][sel], ra0, rp0),
                         "after_timed_steps": errors_of(metrics, r["aT"][sel], r["pT"][sel],
                                                        raT, rpT),
                         "systems": len(pick), "smallest_n": int(min(b.sizes[k] for k in pick))}
    head = next(iter(res))
    r0 = res[head]
    return {
        "value": pairs * args.steps / r0["wall"], "ms_per_step": r0["wall"] / args.steps * 1e3,
        "config": {"workload": w.name, "systems": w.n, "particles": int(b.offsets[-1]),
                   "pairs_per_step": pairs, "eps": w.eps, "dt": w.dt, "precision": head,
                   "step": "one graph-replayed batched KDK step (one persistent launch over "
                           "cost-sorted work items)", "plan": r0["info"],
                   "description": w.description},
        "roofline": roofline("gravity", pairs, r0["kernel_ms"],
                             "persistent_kernel<Gravity> (+ batched finalize)"),
        "cpu_baseline": cpu,
        "modes": {p: {"value": pairs * args.steps / r["wall"],
                      "ms_per_step": r["wall"] / args.steps * 1e3,
                      "force_kernel_ms": r["kernel_ms"],
                      **{"roofline_" + k: v for k, v in
                         fractions("gravity", pairs, r["kernel_ms"]).items()
                         if k in ("frac", "issue_frac")},
                      "errors": errors.get(p)} for p, r in res.items()},
    }


def bench_adjoint(args, torch, w, big=True):
    """N = 16384 loss and gradient through a 32-step checkpointed KDK rollout."""
    from paper_astro_ph_0703100_amd import _lib, api, autograd, ics, metrics
    n = w.n
    x0, v0, mass = ics.plummer(n, seed=w.seed)
    m64 = mass.astype(np.float32).astype(np.float64)
    y = ics.perturbed_target(x0, seed=5001)
    eps = float(np.float32(w.eps))
    dev = torch.device("cuda:0")
    xt = torch.from_numpy(np.ascontiguousarray(x0.T)).to(dev)
    vt = torch.from_numpy(np.ascontiguousarray(v0.T)).to(dev)
    mt = torch.from_numpy(m64).to(dev)
    yt = torch.from_numpy(np.ascontiguousarray(y.T)).to(dev)
    timer = Timer(torch)
    state = {}

    def step():
        xi = xt.clone().requires_grad_(True)
        vi = vt.clone().requires_grad_(True)
        mi = mt.clone().requires_grad_(True)
        xT, _ = autograd.rollout(xi, vi, mi, eps, w.dt, w.steps)
        loss = ((xT - yt) ** 2).sum() / n
        loss.backward()
        state["g"] = (float(loss.detach()), xi.grad, vi.grad, mi.grad)

    wall, step_ms = timer.run(step, args.steps, warmup=args.warmup)
    # The adjoint kernel alone.
    p32 = torch.from_numpy(np.ascontiguousarray(x0.T.astype(np.float32))).to(dev)
    m32 = mt.float()
    g = torch.from_numpy(np.random.default_rng(1).standard_normal((3, n))).to(dev)
    gx = torch.empty((3, n), dtype=torch.float64, device=dev)
    gm = torch.empty(n, dtype=torch.float64, device=dev)
    opts = api.make_opts()
    sp = torch.cuda.current_stream().cuda_stream
    _, kms = timer.run(lambda: _lib.nbody_force_vjp(n, p32.data_ptr(), m32.data_ptr(), eps,
                                                    g.data_ptr(), None, gx.data_ptr(),
                                                    gm.data_ptr(), opts, sp), 8, warmup=args.warmup)
    extra = {}
    if big:
        # The same kernel on the N = 131072 sphere, where the grid holds many rounds of blocks.
        nb = 131072
        xb, _, mb = ics.plummer(nb, seed=2, velocities=False)
        pb = torch.from_numpy(np.ascontiguousarray(xb.T.astype(np.float32))).to(dev)
        mbt = torch.from_numpy(mb.astype(np.float32)).to(dev)
        gb = torch.from_numpy(np.random.default_rng(2).standard_normal((3, nb))).to(dev)
        gxb = torch.empty((3, nb), dtype=torch.float64, device=dev)
        gmb = torch.empty(nb, dtype=torch.float64, device=dev)
        eb = float(np.float32(ics.plummer_131072_eps(nb)))
        _, kmb = timer.run(lambda: _lib.nbody_force_vjp(nb, pb.data_ptr(), mbt.data_ptr(), eb,
                                                        gb.data_ptr(), None, gxb.data_ptr(),
                                                        gmb.data_ptr(), opts, sp), 3,
                           warmup=args.warmup)
        extra["adjoint_kernel_131072"] = fractions("adjoint", float(nb) * nb, float(np.mean(kmb)))
    pairs_step = float(n) * n * 2 * (w.steps + 1)
    print("bench: rollout+gradient %.3f ms/step, adjoint kernel %.3f ms" %
          (wall / args.steps * 1e3, np.mean(kms)), file=sys.stderr, flush=True)
    cpu, errors = None, {}
    if not args.no_cpu_baseline:
        import oracle
        t0 = time.perf_counter()
        lo, rx, rv, rm = oracle.rollout_loss_grad(x0, v0, m64, eps, w.dt, w.steps, y)
        ct = time.perf_counter() - t0
        cpu = cpu_entry(pairs_step / ct,
                        "the whole loss and gradient (%d forward + %d adjoint evaluations of "
                        "%d^2 pairs), FP64 (%.1f s)" % (w.steps + 1, w.steps + 1, n, ct))
        if big:
            g1 = np.random.default_rng(w.seed + 2000).standard_normal((4096, 3))
            one_thread(cpu, lambda: oracle.vjp(x0[:4096], m64[:4096], eps, g1), 4096.0 ** 2,
                       "one adjoint evaluation on the first 4096 particles")
        loss, gxg, gvg, gmg = state["g"]
        errors["comp"] = {
            "loss_rel": abs(loss - lo) / abs(lo),
            "grad_x0_normwise": metrics.rel_errors(gxg.cpu().numpy().T, rx)["normwise"],
            "grad_v0_normwise": metrics.rel_errors(gvg.cpu().numpy().T, rv)["normwise"],
            "grad_m_normwise": metrics.rel_errors(gmg.cpu().numpy(), rm)["normwise"],
            "oracle_pinned_by": "central FP64 finite differences on this workload (64 position "
                                "coordinates, 16 masses; CPU slow test)"}
    return {
        "value": pairs_step * args.steps / wall, "ms_per_step": wall / args.steps * 1e3,
        "config": {"workload": w.name, "n": n, "eps": eps, "dt": w.dt, "steps": w.steps,
                   "precision": "comp",
                   "step": "loss and gradient: %d-step checkpointed KDK rollout and the reverse "
                           "pass with the adjoint kernel; pairs counted: forward + adjoint"
                           % w.steps, "description": w.description},
        "roofline": roofline("adjoint", float(n) * n, float(np.mean(kms)),
                             "tile_kernel<Adjoint> (+ finalize)"),
        "cpu_baseline": cpu,
        "modes": {"comp": {"value": pairs_step * args.steps / wall,
                           "ms_per_step": wall / args.steps * 1e3,
                           **fractions("adjoint", float(n) * n, float(np.mean(kms))),
                           "errors": errors.get("comp")}},
        **extra,
    }


def bench_shard(args, torch, w):
    from paper_astro_ph_0703100_amd import _lib, api, ics, metrics
    n, ni = w.n, w.n // 8
    pos, _, mass = ics.plummer(n, seed=w.seed, velocities=False)
    m32 = mass.astype(np.float32)
    eps = float(np.float32(w.eps))
    dev = torch.device("cuda:0")
    p32 = np.ascontiguousarray(pos.T.astype(np.float32))
    pj = torch.from_numpy(p32).to(dev)
    pi = pj[:, :ni].contiguous()
    m = torch.from_numpy(m32).to(dev)
    acc = torch.empty((3, ni), dtype=torch.float64, device=dev)
    pot = torch.empty(ni, dtype=torch.float64, device=dev)
    sp = torch.cuda.current_stream().cuda_stream
    timer = Timer(torch)
    pairs = float(ni) * float(n)
    res = {}
    for precision in modes_of(args):
        opts = api.make_opts(precision=precision)
        call = lambda: _lib.nbody_force_ij(ni, pi.data_ptr(), None, n, pj.data_ptr(), m.data_ptr(),
                                           eps, acc.data_ptr(), pot.data_ptr(), opts, sp)
        wall, kms = timer.run(call, args.steps, warmup=args.warmup)
        res[precision] = {"wall": wall, "kernel_ms": float(np.mean(kms)),
                          "acc": acc.cpu().numpy().T.copy(), "pot": pot.cpu().numpy().copy()}
        print("bench: %-8s %d evaluations  %.3f ms each (wall)  %.3f ms (events)"
              % (precision, args.steps, wall / args.steps * 1e3, np.mean(kms)),
              file=sys.stderr, flush=True)
    cpu, errors = None, {}
    if not args.no_cpu_baseline:
        import oracle
        k = ni if args.cpu_sample <= 0 else min(ni, args.cpu_sample)
        idx = np.arange(ni) if k == ni else ics.sample_indices(ni, k, seed=w.seed + 1000)
        x64 = p32.T.astype(np.float64)
        t0 = time.perf_counter()
        ra, rp = oracle.force_ij(x64, m32.astype(np.float64), x64[idx], eps)
        ct = time.perf_counter() - t0
        cpu = cpu_entry(k * float(n) / ct,
                        "force+potential of %s i-particles of the shard from all %d, FP64 "
                        "(%.1f s)" % ("all %d" % k if k == ni else "%d sampled" % k, n, ct))
        i1 = idx[::8]
        one_thread(cpu, lambda: oracle.force_ij(x64, m32.astype(np.float64), x64[i1], eps),
                   float(i1.size) * n, "%d of those i-particles" % i1.size)
        for p, r in res.items():
            errors[p] = errors_of(metrics, r["acc"][idx], r["pot"][idx], ra, rp)
    head = next(iter(res))
    r0 = res[head]
    return {
        "value": pairs * args.steps / r0["wall"], "ms_per_step": r0["wall"] / args.steps * 1e3,
        "config": {"workload": w.name, "n": n, "n_i": ni, "eps": eps, "seed": w.seed,
                   "precision": head,
                   "step": "one force+potential evaluation of the first 16384 particles from all "
                           "131072 (nbody_force_ij, FP32 inputs); the self pair counts in the "
                           "potential as for any separate i-set",
                   "description": w.description},
        "roofline": roofline("gravity", pairs, r0["kernel_ms"],
                             "tile_kernel<GravityIJ> (+ finalize_kernel)"),
        "cpu_baseline": cpu,
        "modes": {p: {"value": pairs * args.steps / r["wall"],
                      "ms_per_step": r["wall"] / args.steps * 1e3,
                      **fractions("gravity", pairs, r["kernel_ms"]),
                      "errors": errors.get(p)} for p, r in res.items()},
    }


def bench_jerk(args, torch, w):
    from paper_astro_ph_0703100_amd import _lib, api, ics, metrics
    n = w.n
    pos, vel, mass = ics.plummer(n, seed=w.seed)
    m32 = mass.astype(np.float32)
    eps = float(np.float32(w.eps))
    dev = torch.device("cuda:0")
    x = torch.from_numpy(np.ascontiguousarray(pos.T)).to(dev)
    v = torch.from_numpy(np.ascontiguousarray(vel.T)).to(dev)
    m = torch.from_numpy(m32).to(dev)
    p32 = torch.from_numpy(np.ascontiguousarray(pos.T.astype(np.float32))).to(dev)
    v32 = torch.from_numpy(np.ascontiguousarray(vel.T.astype(np.float32))).to(dev)
    acc = torch.empty((3, n), dtype=torch.float64, device=dev)
    jerk = torch.empty((3, n), dtype=torch.float64, device=dev)
    pot = torch.empty(n, dtype=torch.float64, device=dev)
    sp = torch.cuda.current_stream().cuda_stream
    timer = Timer(torch)
    pairs = float(n) * float(n)
    dt = w.dt or 1.0 / 256
    res = {}
    for precision in modes_of(args):
        opts = api.make_opts(precision=precision)
        xs, vs = x.clone(), v.clone()
        ha, hj = api.hermite(xs, vs, m, eps, dt, 0, precision=precision)
        g = api.HermiteGraph(xs, vs, m, eps, dt, 1, ha, hj, precision=precision)
        warm_up(torch, g.launch, args.warmup)
        xs.copy_(x)
        vs.copy_(v)
        api.hermite(xs, vs, m, eps, dt, 0, acc=ha, jerk=hj, precision=precision)
        wall, _ = timer.run(g.launch, args.steps, warmup=0)
        g.close()
        _lib.nbody_force_jerk_f64(n, x.data_ptr(), v.data_ptr(), m.data_ptr(), eps, acc.data_ptr(),
                                  jerk.data_ptr(), pot.data_ptr(), opts, sp)
        host = (acc.cpu().numpy().T.copy(), jerk.cpu().numpy().T.copy(), pot.cpu().numpy().copy())
        _, kms = timer.run(lambda: _lib.nbody_force_jerk(n, p32.data_ptr(), v32.data_ptr(),
                                                         m.data_ptr(), eps, acc.data_ptr(),
                                                         jerk.data_ptr(), pot.data_ptr(), opts, sp),
                           max(args.steps, 3), warmup=args.warmup)
        res[precision] = {"wall": wall, "kernel_ms": float(np.mean(kms)), "out": host}
        print("bench: %-8s %d Hermite steps  %.3f ms/step (wall)  jerk kernel %.3f ms"
              % (precision, args.steps, wall / args.steps * 1e3, np.mean(kms)),
              file=sys.stderr, flush=True)
    cpu, errors = None, {}
    if not args.no_cpu_baseline:
        import oracle
        k = 32768 if args.cpu_sample <= 0 else min(n, args.cpu_sample)
        idx = ics.sample_indices(n, k, seed=w.seed + 1000)
        t0 = time.perf_counter()
        ra, rj, rp = oracle.force_jerk(pos, vel, m32.astype(np.float64), eps, idx=idx)
        ct = time.perf_counter() - t0
        cpu = cpu_entry(k * float(n) / ct,
                        "force+jerk+potential of %d sampled i-particles from all %d, FP64 "
                        "(%.1f s)" % (k, n, ct))
        i1 = idx[::16]
        one_thread(cpu, lambda: oracle.force_jerk(pos, vel, m32.astype(np.float64), eps, idx=i1),
                   float(i1.size) * n, "%d of those i-particles" % i1.size)
        for p, r in res.items():
            a, j, ph = r["out"]
            e = errors_of(metrics, a[idx], ph[idx], ra, rp)
            ej = metrics.rel_errors(j[idx], rj)
            e.update({"jerk_rel_rms": ej["rel_rms"], "jerk_e_max": ej["e_max"],
                      "jerk_normwise": ej["normwise"]})
            errors[p] = e
    head = next(iter(res))
    r0 = res[head]
    return {
        "value": pairs * args.steps / r0["wall"], "ms_per_step": r0["wall"] / args.steps * 1e3,
        "config": {"workload": w.name, "n": n, "eps": eps, "seed": w.seed, "dt": dt,
                   "precision": head, "engine": "symmetric" if args.symmetric else "default",
                   "step": "one graph-replayed fourth-order Hermite step: FP64 predictor, one "
                           "N^2 force+jerk evaluation (FP32 pair arithmetic relative to the "
                           "mean position and velocity), FP64 corrector",
                   "description": w.description},
        "roofline": roofline("jerk", pairs, r0["kernel_ms"],
                             "tile_kernel<GravityJerk> (+ jerk_finalize_kernel)"),
        "cpu_baseline": cpu,
        "modes": {p: {"value": pairs * args.steps / r["wall"],
                      "ms_per_step": r["wall"] / args.steps * 1e3,
                      **fractions("jerk", pairs, r["kernel_ms"]),
                      "errors": errors.get(p)} for p, r in res.items()},
        "gflops_60": pairs * 60 / (r0["kernel_ms"] * 1e-3) / 1e9,
    }


def bench_active(args, torch, w):
    """Force + jerk + potential of the active eighth of the N = 131072 sphere (a seeded
    sample of 16384 particles, as a Hermite code with individual steps would evaluate)
    from all 131072: one nbody_force_jerk_ij call per step."""
    from paper_astro_ph_0703100_amd import _lib, api, ics, metrics
    n, ni = w.n, w.n // 8
    pos, vel, mass = ics.plummer(n, seed=w.seed)
    act = ics.sample_indices(n, ni, seed=w.seed + 3000)
    m32 = mass.astype(np.float32)
    eps = float(np.float32(w.eps))
    dev = torch.device("cuda:0")
    p32 = np.ascontiguousarray(pos.T.astype(np.float32))
    v32 = np.ascontiguousarray(vel.T.astype(np.float32))
    pj, vj = torch.from_numpy(p32).to(dev), torch.from_numpy(v32).to(dev)
    pi = torch.from_numpy(np.ascontiguousarray(p32[:, act])).to(dev)
    vi = torch.from_numpy(np.ascontiguousarray(v32[:, act])).to(dev)
    m = torch.from_numpy(m32).to(dev)
    acc = torch.empty((3, ni), dtype=torch.float64, device=dev)
    jerk = torch.empty((3, ni), dtype=torch.float64, device=dev)
    pot = torch.empty(ni, dtype=torch.float64, device=dev)
    sp = torch.cuda.current_stream().cuda_stream
    timer = Timer(torch)
    pairs = float(ni) * float(n)
    res = {}
    for precision in modes_of(args):
        opts = api.make_opts(precision=precision)
        call = lambda: _lib.nbody_force_jerk_ij(ni, pi.data_ptr(), vi.data_ptr(), n, pj.data_ptr(),
                                                vj.data_ptr(), m.data_ptr(), eps, acc.data_ptr(),
                                                jerk.data_ptr(), pot.data_ptr(), opts, sp)
        wall, kms = timer.run(call, args.steps, warmup=args.warmup)
        res[precision] = {"wall": wall, "kernel_ms": float(np.mean(kms)),
                          "out": (acc.cpu().numpy().T.copy(), jerk.cpu().numpy().T.copy(),
                                  pot.cpu().numpy().copy())}
        print("bench: %-8s %d evaluations  %.3f ms each (wall)  %.3f ms (events)"
              % (precision, args.steps, wall / args.steps * 1e3, np.mean(kms)),
              file=sys.stderr, flush=True)
    cpu, errors = None, {}
    if not args.no_cpu_baseline:
        import oracle
        k = ni if args.cpu_sample <= 0 else min(ni, args.cpu_sample)
        x64, v64 = p32.T.astype(np.float64), v32.T.astype(np.float64)
        mj = m32.astype(np.float64)
        sel = act[:k]
        t0 = time.perf_counter()
        ra, rj, rp = oracle.force_jerk_ij(x64, v64, mj, x64[sel], v64[sel], eps)
        ct = time.perf_counter() - t0
        cpu = cpu_entry(k * float(n) / ct,
                        "force+jerk+potential of %d of the active particles from all %d, FP64 "
                        "(%.1f s)" % (k, n, ct))
        s1 = sel[::16]
        one_thread(cpu, lambda: oracle.force_jerk_ij(x64, v64, mj, x64[s1], v64[s1], eps),
                   float(s1.size) * n, "%d of those i-particles" % s1.size)
        for p, r in res.items():
            a, j, ph = r["out"]
            e = errors_of(metrics, a[:k], ph[:k], ra, rp)
            ej = metrics.rel_errors(j[:k], rj)
            e.update({"jerk_rel_rms": ej["rel_rms"], "jerk_e_max": ej["e_max"],
                      "jerk_normwise": ej["normwise"]})
            errors[p] = e
    head = next(iter(res))
    r0 = res[head]
    return {
        "value": pairs * args.steps / r0["wall"], "ms_per_step": r0["wall"] / args.steps * 1e3,
        "config": {"workload": w.name, "n": n, "n_i": ni, "eps": eps, "seed": w.seed,
                   "precision": head,
                   "step": "one force+jerk+potential evaluation of 16384 active particles (a "
                           "seeded sample) from all 131072 (nbody_force_jerk_ij, FP32 inputs); "
                           "the active particles' own pairs count as for any separate i-set",
                   "description": w.description},
        "roofline": roofline("jerk", pairs, r0["kernel_ms"],
                             "tile_kernel<GravityJerkIJ> (+ jerk_finalize_kernel)"),
        "cpu_baseline": cpu,
        "modes": {p: {"value": pairs * args.steps / r["wall"],
                      "ms_per_step": r["wall"] / args.steps * 1e3,
                      **fractions("jerk", pairs, r["kernel_ms"]),
                      "errors": errors.get(p)} for p, r in res.items()},
    }


BENCHES = {"plummer_131072": bench_plummer, "plummer_2048": bench_small,
           "stress_1m": bench_stress, "clusters_2048": bench_clusters,
           "adjoint_16384": bench_adjoint, "jerk_131072": bench_jerk,
           "shard8_131072": bench_shard, "active8_131072": bench_active}


def compact(body):
    """The per-configuration entry of the default line: step time, pair rate, both roofline
    fractions of the dominant kernel, and the accuracy against the oracle."""
    roof = body["roofline"]
    out = {"workload": body["config"]["workload"], "step": body["config"]["step"],
           "ms_per_step": body["ms_per_step"], "pairs_per_s": body["value"],
           "kernel": roof["kernel"], "kernel_ms": roof["kernel_ms"],
           "roofline_frac": roof["frac"], "issue_frac": roof["issue_model"]["frac"],
           "modes": {k: {kk: vv for kk, vv in v.items() if kk != "value"}
                     for k, v in body["modes"].items()},
           "oracle_sample": (body.get("cpu_baseline") or {}).get("sample")}
    for key in ("error_split", "adjoint_kernel_131072", "launch_floor_ms"):
        if body.get(key) is not None:
            out[key] = body[key]
    return out


def run_configs(args, torch):
    """Every configuration of the workload set besides the headline, in compact form."""
    from paper_astro_ph_0703100_amd import ics
    out = {}
    for name in CONFIG_WORKLOADS:
        sub = parse(["--steps", "4" if name != "plummer_2048" else "200",
                     "--modes", "comp,plain,fp64red" if name != "adjoint_16384" else "comp"]
                    + (["--no-cpu-baseline"] if args.no_cpu_baseline else []))
        t0 = time.perf_counter()
        fn = BENCHES[name]
        body = fn(sub, torch, ics.WORKLOADS[name], big=False) if name == "adjoint_16384" \
            else fn(sub, torch, ics.WORKLOADS[name])
        out[name] = compact(body)
        out[name]["bench_seconds"] = time.perf_counter() - t0
        print("bench: config %s done (%.1f s)" % (name, out[name]["bench_seconds"]),
              file=sys.stderr, flush=True)
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this path runs on one GPU; --gpus %d is not supported "
              "(a system would shard by i-range with nbody_force_ij; not built)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_astro_ph_0703100_amd import ics

    if args.calib_copy_mb > 0:
        nb = args.calib_copy_mb * (1 << 20) // 4
        src = torch.ones(nb, dtype=torch.float32, device="cuda:0")
        evict = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")  # 1 GiB through the caches
        del evict
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    w = ics.WORKLOADS[args.workload]
    body = BENCHES[w.name](args, torch, w)
    warmed = WARMED[0] if WARMED else args.warmup
    if w.name == "plummer_131072" and not args.no_configs:
        body["configs"] = run_configs(args, torch)
    line = {
        "metric": METRIC if w.name == "plummer_131072" else "pair interactions/s, " + w.name,
        "value": body["value"],
        "unit": "pair-interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": warmed,
        "ms_per_step": body["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
    }
    line.update({k: v for k, v in body.items() if k not in ("value", "ms_per_step")})
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
