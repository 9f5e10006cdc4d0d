"""Benchmark of the coupled f+g D2Q9 MRT step on one MI355X.

Workload: the differentially heated cavity of Sec. 4.3 at 2048 x 2048 nodes,
eps = 0.6, Ra = 1e8, Pr = 0.71, gamma = 1.4, Sutherland viscosity, tau0 = 0.8,
first-order wall extrapolation, all cubic corrections on; synthetic state
(rest + 1e-6 density noise from splitmix64 seed 1), resident in HBM before
the timed region.  One step = one fused launch that streams and collides both
DFs of every node, walls included.

Headline value: FP32-storage MLUPS (million node updates per second).  The
FP16-offset path, the FP32-f / FP16-g path and the FP64 path are timed on
the same workload and reported under "paths".  Roofline: algorithmic HBM
bytes per node and step = 9 f values + 9 g values, each read and written
once, over the average kernel time measured with HIP events on the launch
stream, against 8 TB/s.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "coupled f+g MLUPS and % of HBM roofline, 2048² cavity, FP32/FP16 vs FP64"
PEAK_HBM_GBS = 8000.0
BYTES_PER_NODE = {"f64": 288, "f32": 144, "f16s": 72, "f32g16": 108}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_sha():
    """Hash of the HIP sources with comments and whitespace removed, and of
    the compiler flags, so that a change of comments alone keeps a counter
    record valid."""
    import hashlib
    import glob
    import re
    from paper_1809_08683_amd import build as _build
    src = os.path.join(ROOT, "paper_1809_08683_amd", "csrc")
    h = hashlib.sha256()
    h.update(" ".join(_build.HIPFLAGS).encode())
    for f in sorted(glob.glob(os.path.join(src, "*.hip")) + glob.glob(os.path.join(src, "*.hpp"))):
        h.update(os.path.basename(f).encode())
        with open(f, encoding="utf-8") as fh:
            code = fh.read()
        code = re.sub(r"/\*.*?\*/", " ", code, flags=re.S)
        code = re.sub(r"//[^\n]*", " ", code)
        h.update(" ".join(code.split()).encode())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of the FP32 step kernel from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE record, if it was taken on the current
    kernel sources; None otherwise."""
    path = os.path.join(ROOT, "profiles", "step_kernel_cavity2048_traffic.md")
    try:
        with open(path) as fh:
            for line in fh:
                if line.startswith("traffic_record:"):
                    rec = json.loads(line.split(":", 1)[1])
                    if rec.get("source_sha") == kernel_source_sha():
                        return rec["bytes_per_launch"]
    except OSError:
        pass
    return None


def _timed(ctx, nodes, prec, steps, warmup):
    """Warm-up, then `steps` timed steps (HIP events on the launch stream and
    the host clock around them)."""
    import torch

    # The 2048^2 Ra = 1e8 cavity leaves the stable range of the scheme
    # between steps 1000 and 2000 from rest (its buoyancy velocity passes
    # Mach 0.25); the cost of a step does not depend on the values, so a
    # longer run is still timed, and the divergence is reported.
    diverged_at = None
    if warmup:
        ctx.step_timed(warmup, allow_diverged=True)
        if ctx.diverged:
            diverged_at = "warmup"
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kernel_ms = ctx.step_timed(steps, allow_diverged=True)
    torch.cuda.synchronize()
    wall_s = time.perf_counter() - t0
    if ctx.diverged and diverged_at is None:
        diverged_at = "timed steps"
    if diverged_at:
        log(f"bench: {prec}: the lattice state diverged during the {diverged_at} "
            f"(the timing covers complete steps)")
    per_step_kernel_s = kernel_ms * 1e-3 / steps
    res = {
        "mlups": nodes * steps / wall_s / 1e6,
        "ms_per_step": wall_s * 1e3 / steps,
        "kernel_ms_per_step": per_step_kernel_s * 1e3,
        "kernel_mlups": nodes / per_step_kernel_s / 1e6,
        "bytes_per_node": BYTES_PER_NODE[prec],
        "achieved_GBs": BYTES_PER_NODE[prec] * nodes / per_step_kernel_s / 1e9,
        "work_items": ctx.work_items,
        "state_diverged": diverged_at,
    }
    res["frac_hbm"] = res["achieved_GBs"] / PEAK_HBM_GBS
    return res


def time_path(case, prec, steps, warmup, seg_rows=0, tune=True):
    """Times the step in the default launch configuration, then in the one
    the autotuner picks (its cache file, or trials on this context when the
    cache has no entry), from the same start state."""
    import torch
    from paper_1809_08683_amd import lbm

    c = dict(case, prec=prec)
    stream = torch.cuda.Stream()
    ctx = lbm.Context(c, stream=stream, seg_rows=seg_rows)
    nodes = c["nx"] * c["ny"]
    ctx.init(**c["init"])
    res = _timed(ctx, nodes, prec, steps, warmup)
    if tune:
        ctx.init(**c["init"])
        t = ctx.autotune(trial_steps=100)
        log(f"bench: {prec}: launch configuration {t}")
        ctx.init(**c["init"])
        tuned = _timed(ctx, nodes, prec, steps, warmup)
        default = res
        res = dict(tuned)
        res["tune"] = {k: (round(v, 5) if isinstance(v, float) else v) for k, v in t.items()}
        res["default_config"] = {k: default[k] for k in ("mlups", "ms_per_step", "kernel_ms_per_step", "frac_hbm")}
    ctx.close()
    return res


def time_batch(steps, warmup, prec="f32"):
    """The batched sweep: 64 cavities of uneven size (N in {128..1024}) and
    Rayleigh number, one launch per step for all of them."""
    import torch
    from paper_1809_08683_amd import inputs, lbm

    cases = inputs.batch_cases(seed=2, n=64, prec=prec)
    nodes = sum(c["nx"] * c["ny"] for c in cases)
    stream = torch.cuda.Stream()
    b = lbm.Batch(cases, stream=stream)

    def start():
        for k, c in enumerate(cases):
            b.init(k, rho=1.0 + 1e-6 * inputs.noise(3 + k, c["nx"] * c["ny"]).reshape(c["ny"], c["nx"]))

    def run(graph, persistent=False):
        start()
        if warmup:
            b.step(warmup, allow_diverged=True)
        if graph:                       # capture the graph of `steps` steps outside the timed region
            b.step_ex(steps, graph=True, allow_diverged=True, persistent=persistent)
            start()
            b.step(warmup, allow_diverged=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ms = b.step_ex(steps, graph=graph, allow_diverged=True, persistent=persistent)
        torch.cuda.synchronize()
        return ms, time.perf_counter() - t0

    default_ms, default_wall = run(False)
    start()
    tune = b.autotune(trial_steps=20)
    log(f"bench: batch launch configuration {tune}")
    kernel_ms, wall_s = run(True)
    flags = b.flags()
    # the same steps in one persistent launch (per-case step barriers), replayed as a graph
    persistent = None
    try:
        p_ms, p_wall = run(True, persistent=True)
        persistent = {"mlups": nodes * steps / p_wall / 1e6,
                      "kernel_mlups": nodes / (p_ms * 1e-3 / steps) / 1e6,
                      "frac_hbm": BYTES_PER_NODE[prec] * nodes / (p_ms * 1e-3 / steps) / 1e9 / PEAK_HBM_GBS,
                      "stepping": "one persistent launch with per-case step barriers, replayed as a captured graph"}
    except lbm.LBMError as e:
        persistent = {"skipped": str(e)}
    log(f"bench: batch persistent {persistent}")
    per_step_s = kernel_ms * 1e-3 / steps
    res = {
        "workload": "64 cavities, N in {128,256,512,1024} (seed 2), Ra log-uniform in [1e3,1e8], "
                    "eps in [0.1,0.6], Pr in {0.71,1,7}, buoyancy Mach 0.05 (nu0 >= 0.1)",
        "prec": prec,
        "nodes": nodes,
        "mlups": nodes * steps / wall_s / 1e6,
        "ms_per_step": wall_s * 1e3 / steps,
        "kernel_mlups": nodes / per_step_s / 1e6,
        "achieved_GBs": BYTES_PER_NODE[prec] * nodes / per_step_s / 1e9,
        "diverged_cases": int(sum(flags)),
        "work_items": b.work_items,
        "stepping": "launch configuration from the autotuner, steps replayed as one captured HIP graph",
        "tune": {k: (round(v, 5) if isinstance(v, float) else v) for k, v in tune.items()},
        "default_config": {"mlups": nodes * steps / default_wall / 1e6,
                           "kernel_mlups": nodes / (default_ms * 1e-3 / steps) / 1e6,
                           "frac_hbm": BYTES_PER_NODE[prec] * nodes / (default_ms * 1e-3 / steps) / 1e9 / PEAK_HBM_GBS,
                           "stepping": "default configuration, one launch per step"},
        "persistent": persistent,
    }
    res["frac_hbm"] = res["achieved_GBs"] / PEAK_HBM_GBS
    b.close()
    return res


def batch_accuracy(steps, prec="f32"):
    """Per-case mean Nusselt number of the batched sweep in `prec` against the
    same sweep stepped in FP64 on the GPU, after `steps` steps from the same
    start, with the a-priori flag of each case (no viscosity keeps the paired
    relaxation rates below 1.75 at both walls) and the Rayleigh number the
    case runs at (Ra_eff, where its viscosity was moved into that window)."""
    from paper_1809_08683_amd import inputs, lbm

    runs = {}
    for pr in (prec, "f64"):
        cases = inputs.batch_cases(seed=2, n=64, prec=pr)
        b = lbm.Batch(cases)
        for k, c in enumerate(cases):
            b.init(k, rho=1.0 + 1e-6 * inputs.noise(3 + k, c["nx"] * c["ny"]).reshape(c["ny"], c["nx"]))
        done = 0
        while done < steps:
            n = min(1000, steps - done)
            b.step(n, allow_diverged=True)
            done += n
        flags = b.flags()
        nu = [None if flags[k] else b.nusselt(k, 0) for k in range(len(cases))]
        runs[pr] = (cases, flags, nu)
        b.close()
        log(f"bench: batch accuracy {pr}: {steps} steps, {sum(flags)} cases diverged")
    cases, f_lo, nu_lo = runs[prec]
    _, f_64, nu_64 = runs["f64"]
    rows, errs = [], []
    for k, c in enumerate(cases):
        err = None
        if nu_lo[k] is not None and nu_64[k] is not None:
            err = abs(nu_lo[k] - nu_64[k]) / abs(nu_64[k])
            errs.append(err)
        rows.append([k, c["nx"], float(f"{c['Ra']:.4g}"), float(f"{c['Ra_eff']:.4g}"), round(c["eps"], 4), c["Pr"],
                     round(c["nu0"], 5), bool(c["window_empty"]),
                     None if nu_64[k] is None else round(nu_64[k], 6),
                     None if err is None else float(f"{err:.3g}"), bool(f_lo[k]), bool(f_64[k])])
    return {
        "steps": steps,
        "prec": prec,
        "columns": ["case", "N", "Ra", "Ra_eff", "eps", "Pr", "nu0", "flagged_a_priori", "Nu_f64",
                    f"Nu_rel_err_{prec}_vs_f64", f"diverged_{prec}", "diverged_f64"],
        "cases": rows,
        "flagged_a_priori": int(sum(r[7] for r in rows)),
        "max_Nu_rel_err": None if not errs else float(f"{max(errs):.3g}"),
        "cases_within_0.5pct": int(sum(e <= 5e-3 for e in errs)),
        "cases_compared": len(errs),
    }


def format_accuracy(precs, cases=((256, 1e5, 100000), (1024, 1e6, 50000))):
    """Mean hot-wall Nusselt number of each storage format against the FP64
    path on the same cavity (eps = 0.6, tau0 = 0.8, seeded noise) after the
    same number of steps: the 256^2 Ra = 1e5 cavity near steady state and the
    1024^2 Ra = 1e6 cavity during its transient."""
    from paper_1809_08683_amd import inputs, lbm

    out = {}
    for N, Ra, steps in cases:
        nu = {}
        for prec in ["f64"] + [p for p in precs if p != "f64"]:
            c = inputs.cavity(N=N, Ra=Ra, eps=0.6, prec=prec, noise_seed=1)
            g = lbm.Context(c).init(**c["init"])
            g.step_ex(steps, allow_diverged=True)
            nu[prec] = None if g.diverged else g.nusselt(0)
            g.close()
        key = f"{N}x{N} Ra {Ra:.0e}, {steps} steps"
        out[key] = {"Nu_f64": round(nu["f64"], 6)}
        for prec, v in nu.items():
            if prec != "f64":
                out[key][f"Nu_rel_err_{prec}"] = None if v is None else float(f"{(v - nu['f64']) / nu['f64']:.3g}")
        log(f"bench: accuracy {key}: {json.dumps(out[key])}")
    return out


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(seconds_target=12.0):
    """The FP64 CPU oracle as written, on a bounded sample: a 256 x 256 cavity
    (eps 0.6, Ra 1e5) stepped for about `seconds_target` seconds on one host
    thread and again on all the host threads this process may use (its node
    loops run under OpenMP with bitwise the serial result)."""
    import oracle
    from paper_1809_08683_amd import inputs

    def run(threads):
        c = inputs.cavity(N=256, Ra=1e5, prec="f64", noise_seed=1)
        o = oracle.Oracle(c).set_threads(threads).init(**c["init"])
        steps = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < seconds_target:
            o.step(5)
            steps += 5
        dt = time.perf_counter() - t0
        return 256 * 256 * steps / dt / 1e6, steps, dt

    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    threads = max(1, min(avail, int(os.environ.get("OMP_NUM_THREADS") or avail)))
    v1, s1, t1 = run(1)
    vn, sn, tn = run(threads)
    return {"value": round(vn, 3), "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": f"256x256 cavity (eps 0.6, Ra 1e5), FP64: {sn} steps in {tn:.1f} s on {threads} threads; "
                      f"{s1} steps in {t1:.1f} s on one thread",
            "value_1core": round(v1, 3), "nproc": os.cpu_count(), "threads_available": avail,
            "cpu_model": _cpu_model()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--paths", default="f32,f16s,f32g16,f64")
    ap.add_argument("--seg-rows", type=int, default=0)
    ap.add_argument("--no-tune", action="store_true", help="time the default launch configuration only")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--batch-acc-steps", type=int, default=20000,
                    help="steps of the per-case FP32-vs-FP64 Nusselt comparison of the batched sweep (0: skip)")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the per-format Nusselt comparison with the FP64 path")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: runs on one GPU only (a multi-GPU slab decomposition is designed "
              "but not built); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1809_08683_amd import inputs, lbm

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    lbm.load_library()

    case = inputs.cavity(N=args.n, Ra=1e8, eps=0.6, prec="f32", noise_seed=1)
    paths = {}
    for prec in args.paths.split(","):
        log(f"bench: {args.n}^2 cavity {prec}: warmup {args.warmup}, timed {args.steps} steps")
        paths[prec] = time_path(case, prec, args.steps, args.warmup, args.seg_rows, tune=not args.no_tune)
        log(f"bench: {prec}: {json.dumps(paths[prec])}")
    batch = None
    if not args.no_batch:
        log("bench: 64-cavity batch f32: warmup 20, timed 100 steps")
        batch = time_batch(100, 20)
        log(f"bench: batch: {json.dumps(batch)}")
        if args.batch_acc_steps > 0:
            batch["accuracy"] = batch_accuracy(args.batch_acc_steps)
            log(f"bench: batch accuracy: {json.dumps(batch['accuracy'])}")
    accuracy = None
    if not args.no_accuracy and "f64" in paths:
        accuracy = format_accuracy(list(paths))
    copy_gbs, _ = lbm.copy_bandwidth(1 << 30, iters=20)
    log(f"bench: device copy bandwidth {copy_gbs:.0f} GB/s")

    head = "f32" if "f32" in paths else list(paths)[0]
    h = paths[head]
    out = {
        "metric": METRIC,
        "value": round(h["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(h["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": head,
        "data": "synthetic",
        "config": {
            "workload": f"differentially heated cavity {args.n}x{args.n}, eps 0.6, Ra 1e8, Pr 0.71, "
                        f"gamma 1.4, Sutherland, tau0 0.8, bulk/shear 4, 1st-order walls, "
                        f"cubic corrections on, {head} storage",
            "nx": args.n, "ny": args.n, "prec": head,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(h["achieved_GBs"], 1),
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": round(h["frac_hbm"], 4),
            # the committed counter record covers the FP32 kernel at 2048 x 2048
            "traffic": measured_traffic() if head == "f32" and args.n == 2048 and args.seg_rows == 0 else None,
        },
        "paths": {k: {kk: (round(vv, 4) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                  for k, v in paths.items()},
        "copy_bandwidth_GBs": round(copy_gbs, 1),
    }
    if accuracy is not None:
        out["format_accuracy"] = accuracy
    if batch is not None:
        out["batch"] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in batch.items()}
    if "f64" in paths:
        out["speedup_vs_f64"] = {k: round(v["mlups"] / paths["f64"]["mlups"], 3) for k, v in paths.items()}
    if not args.no_cpu:
        log("bench: cpu_baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
