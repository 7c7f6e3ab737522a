"""Autotuner: measure launch shapes on the GPU and write the library's tuning table.

For each workload it sweeps i-particles per lane (1, 2, 4, 8), j-tile (64 .. 512)
and, for the single-system kernels (force, force-jerk, adjoint), the number of
j-segments of the grid engine; for the force and the adjoint up to 2^15 particles
also the split engine's shapes (lanes per i-particle 8 .. 64, i-particles per lane 1
or 2, j-tile 256 .. 2048).  Every shape is timed with HIP events on the launch stream
(median of ``reps`` runs, after a warm-up call): the force and the adjoint as HIP graphs
of back-to-back calls (the GPU's own time; a small evaluation takes less than the
host's launch cost), the others as runs of back-to-back calls; and admits
a shape only if its result matches a reference computed on the same GPU with FP64
reduction at the built-in shape (relative RMS <= 1e-6, plain FP32 <= 2e-5).  The
fastest admitted shape is stored with ``nbody_tune_set`` and the table is written
with ``nbody_tune_save``; the library loads ``tuning_gfx950.json`` next to itself.

    python -m paper_astro_ph_0703100_amd.tune --out paper_astro_ph_0703100_amd/tuning_gfx950.json
"""
from __future__ import annotations

import argparse
import json
import os
import sys

import numpy as np
import torch

from . import _lib, api, ics
from .metrics import rel_errors

IPLS = (1, 2, 4, 8)
JTILES = (64, 128, 256, 512)
SEGS = (0, 4, 8, 10, 12, 16, 20, 24, 32, 40, 48, 64, 96, 128)
# Split engine: (ipl, jlanes, jtile); the adjoint's 32-byte j-records stop at 512.
SPLIT_MAX_N = 1 << 15
SPLIT = [(ipl, jl, jt) for ipl in (1, 2) for jl in (8, 16, 32, 64) for jt in (256, 512, 1024, 2048)
         if jt < 2048 or jl >= 32]
GATE = {"comp": 1e-6, "fp64red": 1e-6, "plain": 2e-5}


def shapes(n: int, kernel: str):
    """Launch shapes to sweep for ``n`` particles: dicts of ipl, jtile, nseg, jlanes."""
    out = []
    for ipl in IPLS:
        for jt in JTILES:
            jtiles = (n + jt - 1) // jt
            for nseg in SEGS:
                if nseg <= jtiles:
                    out.append({"ipl": ipl, "jtile": jt, "nseg": nseg, "jlanes": 1})
    if kernel in ("force", "vjp") and n <= SPLIT_MAX_N:
        for ipl, jl, jt in SPLIT:
            if kernel == "vjp" and jt > 512:
                continue
            if jt == 2048 and n > 8192:
                continue  # one block per CU pair of tiles: only for the smallest systems
            out.append({"ipl": ipl, "jtile": jt, "nseg": 0, "jlanes": jl})
    return out


def _time(call, reps: int) -> float:
    """Median milliseconds per call (events on the current stream around runs of
    back-to-back calls, each run about a millisecond or longer)."""
    call()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(s)
    call()
    b.record(s)
    b.synchronize()
    inner = max(1, min(200, int(1.0 / max(a.elapsed_time(b), 1e-3))))
    times = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(s)
        for _ in range(inner):
            call()
        b.record(s)
        b.synchronize()
        times.append(a.elapsed_time(b) / inner)
    return float(np.median(times))


def _time_graph(make_call, reps: int) -> float:
    """Median milliseconds per call of ``make_call(stream)()`` replayed from a HIP graph of
    back-to-back calls (about half a millisecond or more per replay): the GPU's own time
    per call, without the host's launch cost, which exceeds a small evaluation's."""
    side = torch.cuda.Stream()
    s = torch.cuda.current_stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        call = make_call(side.cuda_stream)
        call()
        side.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(side)
        call()
        b.record(side)
        b.synchronize()
        k = max(1, min(50, int(np.ceil(0.5 / max(a.elapsed_time(b), 1e-3)))))
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=side):
            for _ in range(k):
                call()
    torch.cuda.synchronize()
    g.replay()
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(s)
        g.replay()
        b.record(s)
        b.synchronize()
        times.append(a.elapsed_time(b) / k)
    del g
    return float(np.median(times))


def _workspace(nbytes):
    return torch.empty(max(256, nbytes), dtype=torch.uint8, device="cuda:0")


def _host(t):
    return t.detach().cpu().numpy()


def tune_force(n: int, seed: int, eps: float, precision: str, reps: int = 3, log=None):
    """Sweep the single-system force kernel (with potential) for ``n`` particles."""
    pos, _, mass = ics.plummer(n, seed=seed)
    dev = "cuda:0"
    p = torch.from_numpy(np.ascontiguousarray(pos.T.astype(np.float32))).to(dev)
    m = torch.from_numpy(mass.astype(np.float32)).to(dev)
    ref_a, ref_p = api.force(p, m, eps, precision="fp64red", ipl=1, jtile=64, nseg=1)
    ref_a, ref_p = _host(ref_a).T, _host(ref_p)
    acc = torch.empty((3, n), dtype=torch.float64, device=dev)
    pot = torch.empty(n, dtype=torch.float64, device=dev)
    best = None
    rows = []
    for sh in shapes(n, "force"):
        ws = _workspace(_lib.nbody_workspace_size(n, api.make_opts(precision=precision, **sh)))
        opts = api.make_opts(precision=precision, workspace=ws, **sh)
        ms = _time_graph(lambda st: lambda: _lib.nbody_force_ex(
            n, p.data_ptr(), m.data_ptr(), eps, acc.data_ptr(), pot.data_ptr(), opts, st), reps)
        ea = rel_errors(_host(acc).T, ref_a)["rel_rms"]
        ep = rel_errors(_host(pot), ref_p)["rel_rms"]
        ok = ea <= GATE[precision] and ep <= GATE[precision]
        row = dict({"kernel": "force", "precision": precision, "n": n}, **sh)
        row.update({"ms": ms, "acc_rel_rms": ea, "ok": ok, "pairs_per_s": n * n / (ms * 1e-3)})
        rows.append(row)
        if log:
            log(row)
        if ok and (best is None or ms < best["ms"]):
            best = row
    return best, rows


def tune_jerk(n: int, seed: int, eps: float, precision: str, reps: int = 3, log=None):
    """Sweep the force-jerk-potential kernel for ``n`` particles (with velocities)."""
    pos, vel, mass = ics.plummer(n, seed=seed)
    dev = "cuda:0"
    p = torch.from_numpy(np.ascontiguousarray(pos.T.astype(np.float32))).to(dev)
    v = torch.from_numpy(np.ascontiguousarray(vel.T.astype(np.float32))).to(dev)
    m = torch.from_numpy(mass.astype(np.float32)).to(dev)
    ref_a, ref_j, _ = api.force_jerk(p, v, m, eps, precision="fp64red", ipl=1, jtile=64, nseg=1)
    ref_a, ref_j = _host(ref_a).T.copy(), _host(ref_j).T.copy()
    acc = torch.empty((3, n), dtype=torch.float64, device=dev)
    jerk = torch.empty((3, n), dtype=torch.float64, device=dev)
    pot = torch.empty(n, dtype=torch.float64, device=dev)
    best, rows = None, []
    for ipl in IPLS:
        for jt in JTILES:
            jtiles = (n + jt - 1) // jt
            for nseg in SEGS:
                if nseg > jtiles:
                    continue
                opts = api.make_opts(precision=precision, ipl=ipl, jtile=jt, nseg=nseg)
                call = lambda: _lib.nbody_force_jerk(n, p.data_ptr(), v.data_ptr(), m.data_ptr(),
                                                     eps, acc.data_ptr(), jerk.data_ptr(),
                                                     pot.data_ptr(), opts, api.stream_ptr())
                ms = _time(call, reps)
                ea = rel_errors(_host(acc).T, ref_a)["rel_rms"]
                ej = rel_errors(_host(jerk).T, ref_j)["normwise"]
                ok = ea <= GATE[precision] and ej <= 10 * GATE[precision]
                row = {"kernel": "jerk", "precision": precision, "n": n, "ipl": ipl, "jtile": jt,
                       "nseg": nseg, "ms": ms, "acc_rel_rms": ea, "jerk_normwise": ej, "ok": ok,
                       "pairs_per_s": n * n / (ms * 1e-3)}
                rows.append(row)
                if log:
                    log(row)
                if ok and (best is None or ms < best["ms"]):
                    best = row
    return best, rows


def tune_vjp(n: int, seed: int, eps: float, precision: str, reps: int = 3, log=None):
    pos, _, mass = ics.plummer(n, seed=seed)
    dev = "cuda:0"
    rng = np.random.default_rng(seed + 1)
    p = torch.from_numpy(np.ascontiguousarray(pos.T.astype(np.float32))).to(dev)
    m = torch.from_numpy(mass.astype(np.float32)).to(dev)
    g = torch.from_numpy(rng.standard_normal((3, n))).to(dev)
    gx = torch.empty((3, n), dtype=torch.float64, device=dev)
    gm = torch.empty(n, dtype=torch.float64, device=dev)

    def run(opts, stream=None):
        return lambda: _lib.nbody_force_vjp(n, p.data_ptr(), m.data_ptr(), eps, g.data_ptr(),
                                            None, gx.data_ptr(), gm.data_ptr(), opts,
                                            stream if stream is not None else api.stream_ptr())
    run(api.make_opts(precision="fp64red", ipl=1, jtile=64, nseg=1))()
    torch.cuda.synchronize()
    ref = _host(gx).T.copy()
    best, rows = None, []
    for sh in shapes(n, "vjp"):
        ws = _workspace(_lib.nbody_workspace_size_vjp(n, api.make_opts(precision=precision, **sh)))
        opts = api.make_opts(precision=precision, workspace=ws, **sh)
        ms = _time_graph(lambda st: run(opts, st), reps)
        e = rel_errors(_host(gx).T, ref)["normwise"]
        ok = e <= 1e-6
        row = dict({"kernel": "vjp", "precision": precision, "n": n}, **sh)
        row.update({"ms": ms, "normwise": e, "ok": ok, "pairs_per_s": n * n / (ms * 1e-3)})
        rows.append(row)
        if log:
            log(row)
        if ok and (best is None or ms < best["ms"]):
            best = row
    return best, rows


def tune_batched(nsys: int, seed: int, eps: float, precision: str, reps: int = 3, log=None):
    b = ics.cluster_batch(nsys, seed=seed, eps=eps)
    dev = "cuda:0"
    p = torch.from_numpy(np.ascontiguousarray(b.pos.T.astype(np.float32))).to(dev)
    m = torch.from_numpy(b.mass.astype(np.float32)).to(dev)
    e = torch.from_numpy(b.eps.astype(np.float32)).to(dev)
    ref_plan = api.BatchPlan(b.offsets, precision="fp64red", ipl=1, jtile=64)
    ref_a, _ = ref_plan.force(p, m, e)
    ref_a = _host(ref_a).T.copy()
    ref_plan.close()
    best, rows = None, []
    mean_n = int(b.offsets[-1] // max(1, nsys))
    for ipl in IPLS:
        for jt in JTILES:
            plan = api.BatchPlan(b.offsets, precision=precision, ipl=ipl, jtile=jt)
            info = plan.info()
            acc, pot = plan.force(p, m, e)
            ms = _time(lambda: plan.force(p, m, e, with_pot=True), reps)
            acc, _ = plan.force(p, m, e)
            err = rel_errors(_host(acc).T, ref_a)["rel_rms"]
            ok = err <= GATE[precision]
            row = {"kernel": "batched", "precision": precision, "n": mean_n, "nsys": nsys,
                   "ipl": ipl, "jtile": jt, "nseg": 0, "ms": ms, "acc_rel_rms": err, "ok": ok,
                   "pairs_per_s": info["pairs"] / (ms * 1e-3), "items": info["items"],
                   "padded_pairs": info["padded_pairs"]}
            rows.append(row)
            if log:
                log(row)
            if ok and (best is None or ms < best["ms"]):
                best = row
            plan.close()
    return best, rows


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--out", default=_lib.TUNING_PATH)
    ap.add_argument("--report", default="", help="write every measured shape here (JSON lines)")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--quick", action="store_true", help="force kernel at N=131072 only")
    ap.add_argument("--only", default="",
                    help="comma-separated kernels to tune (force, jerk, vjp, batched); the other "
                         "entries of the table at --out are kept")
    args = ap.parse_args(argv)

    _lib.load()
    only = [k for k in args.only.split(",") if k]
    if only and os.path.exists(args.out):
        _lib.nbody_tune_reset()
        _lib.nbody_tune_load(args.out)  # keep the entries that are not re-tuned
    else:
        _lib.nbody_tune_reset()  # measure against the built-in shapes, not an old table
    rep = open(args.report, "w") if args.report else None

    def log(row):
        if rep:
            rep.write(json.dumps(row) + "\n")
            rep.flush()

    jobs = []
    w = ics.WORKLOADS["plummer_131072"]
    eps = float(np.float32(w.eps))
    for prec in ("comp", "plain", "fp64red"):
        jobs.append(("force", prec, lambda prec=prec: tune_force(w.n, w.seed, eps, prec, args.reps, log)))
    if not args.quick:
        # Below 2^13 particles the built-in split-engine shapes are used (they depend on n
        # within a size bucket: the 2048-record tile only while the blocks fit one round).
        for n in (8192, 16384, 32768):
            jobs.append(("force", "comp", lambda n=n: tune_force(n, 10 + n, 0.01, "comp", args.reps, log)))
        jobs.append(("jerk", "comp", lambda: tune_jerk(w.n, w.seed, eps, "comp", args.reps, log)))
        wa = ics.WORKLOADS["adjoint_16384"]
        jobs.append(("vjp", "comp", lambda: tune_vjp(wa.n, wa.seed, float(np.float32(wa.eps)), "comp",
                                                     args.reps, log)))
        wb = ics.WORKLOADS["clusters_2048"]
        jobs.append(("batched", "comp", lambda: tune_batched(wb.n, wb.seed, wb.eps, "comp",
                                                             args.reps, log)))
    if only:
        jobs = [j for j in jobs if j[0] in only]
    summary = []
    for kernel, prec, job in jobs:
        best, rows = job()
        if best is None:
            print("tune: no shape passed the parity gate for %s/%s" % (kernel, prec), file=sys.stderr)
            continue
        _lib.nbody_tune_set(_lib.KERNELS[kernel], _lib.PRECISIONS[prec], best["n"], best["ipl"],
                            best["jtile"], best["nseg"], best.get("jlanes", 1))
        default = [r for r in rows if r["ok"]]
        print("tune: %-7s %-7s n=%-7d best ipl=%d jtile=%d nseg=%d jlanes=%d  %.4f ms  %.3g "
              "pairs/s (%d shapes, slowest admitted %.3f ms)"
              % (kernel, prec, best["n"], best["ipl"], best["jtile"], best["nseg"],
                 best.get("jlanes", 1), best["ms"], best["pairs_per_s"], len(rows),
                 max(r["ms"] for r in default)), flush=True)
        summary.append(best)
    _lib.nbody_tune_save(args.out)
    print("tune: wrote %s" % args.out, flush=True)
    if rep:
        rep.close()
    return summary


if __name__ == "__main__":
    main()
