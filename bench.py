"""Throughput of the micro-macro ES-BGK step on one MI355X.

Workload (default): the 256 x 256 x 32 x 32 cavity box (67,108,864 phase-space
points; walls, moving lid, seeded density/temperature perturbations, eps =
1e-2), FP64.  A step is one full micro-macro step over the whole grid.  The
same line reports the mixed-precision form (g stored in FP32) and the
learned-closure form (network trained on the GPU before the timed region, on
snapshots of the solver's own runs) on the same workload, each form's
macro-moment error against the FP64 oracle after 100 steps, the phase-space
pass's HBM roofline fraction, and the oracle timed on the host cores.

Prints one JSON line.  Usage:
  python bench.py [--gpus 1] [--steps K] [--warmup W] [--forms fp64,mixed,closure] [--no-cpu]
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import mm_workloads as W  # noqa: E402

HBM_PEAK_GBS = 8000.0     # MI355X HBM3E
GOLDEN = os.path.join(ROOT, "tests", "golden", "c3_cavity_100steps.npz")
# sources of the phase-space pass; the committed counter figures are valid only for this hash
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2509_21832_amd", "csrc", f)
                  for f in ("mm_fused2d.hip", "mm_fused2d_lk.hip", "mm_fused_common.h", "mm_internal.h")]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def bytes_per_point(precision):
    """Algorithmic HBM bytes per phase-space point per step: read g once, write g once."""
    return 16 if precision == "fp64" else 8


def make_solver(B, p, Q, G, closure):
    s = B.Solver(p, Q, G)
    if p["precision"] == "closure":
        s.closure_attach(closure["net"], closure["kn_max"], residual=closure["residual"])
    return s


def time_form(B, torch, p, Q, G, steps, warmup, closure=None):
    s = make_solver(B, p, Q, G, closure)
    s.step(warmup)
    torch.cuda.synchronize()
    s.timing(True)
    t0 = time.perf_counter()
    s.step_async(steps)
    s.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    n_micro, ms_micro = s.timing_get(0)
    n_prep, ms_prep = s.timing_get(1)
    n_macro, ms_macro = s.timing_get(2)
    n_wall, ms_wall = s.timing_get(3)
    n_cl, ms_cl = s.timing_get(4)
    s.timing(False)
    # the same number of steps without event timing (the headline figure)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    s.step_async(steps)
    s.sync()
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    frac = None
    if p["precision"] == "closure":
        ncl, _ = s.closure_cells()
        frac = ncl / ((warmup + 2 * steps) * p["nx"] * p["ny"])
    s.close()
    return {"seconds": t3 - t2, "seconds_timed_run": t1 - t0,
            "micro_ms": ms_micro / max(n_micro, 1), "prep_ms": ms_prep / max(n_prep, 1),
            "macro_ms": ms_macro / max(n_macro, 1), "wall_ms": ms_wall / max(n_wall, 1),
            "closure_ms": ms_cl / max(n_cl, 1), "launches": n_micro,
            "closure_fraction": frac}


def oracle_error(B, p, eps, seed=0, closure=None):
    """Macro rel-L1 after 100 steps against the oracle's stored result (sampled cells)."""
    if not os.path.exists(GOLDEN):
        return None
    ref = np.load(GOLDEN)
    key = f"eps{eps:g}"
    if key + "_sample" not in ref:
        return None
    st = int(ref["stride"])
    p0, Q0, G0 = W.cavity2d(seed=seed, eps=eps)
    p0["precision"] = p["precision"]
    with make_solver(B, p0, Q0, G0, closure) as s:
        s.step(int(ref["steps"]))
        Q = s.moments().reshape(p0["ny"], p0["nx"], 6)
    a = Q[::st, ::st, :]
    b = ref[key + "_sample"]
    return float(np.abs(a - b).sum() / np.abs(b).sum())


def cpu_baseline(p, Q, G, budget_s=20.0):
    """The oracle on the host cores, on a bounded sample of the workload: full-size steps."""
    import oracle
    threads = oracle.threads()
    t0 = time.perf_counter()
    Qc, Gc, H = oracle.run(p, Q.reshape(-1), G.reshape(-1), 1)
    t1 = time.perf_counter()
    per = t1 - t0
    n = max(0, min(4, int(budget_s / per) - 1))
    if n:
        t0 = time.perf_counter()
        oracle.run(p, Qc, Gc, n)
        per = (time.perf_counter() - t0) / n
    steps = n if n else 1
    pts = p["nx"] * p["ny"] * p["nv1"] * p["nv2"]
    # one more full step on a single thread
    oracle.set_threads(1)
    try:
        t0 = time.perf_counter()
        oracle.run(p, Qc, Gc, 1)
        per1 = time.perf_counter() - t0
    finally:
        oracle.set_threads(threads)
    return {"value": pts / per, "unit": "phase-space cell-updates/s", "cores": threads, "kind": "oracle",
            "value_1thread": pts / per1,
            "sample": f"{steps} full step(s) of the {p['nx']}x{p['ny']}x{p['nv1']}x{p['nv2']} workload "
                      f"({per:.2f} s per step, {threads} OpenMP threads), then 1 step on 1 thread "
                      f"({per1:.2f} s)"}


def copy_bandwidth(torch, gib=1.0, reps=10):
    """Device-to-device copy rate of this GPU (bytes read + written per second, GB/s):
    the attainable bandwidth for a stream that reads and writes equal amounts, as
    the phase-space pass does."""
    n = int(gib * (1 << 30)) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2 * n * 8 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return gbs


def traffic_entry(precision):
    """HBM bytes of the phase-space pass from committed rocprofv3 counter runs, if they
    were taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    e = d.get(precision)
    if not e or e.get("kernel_hash") != kernel_hash():
        return None
    return e.get("bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--forms", default="fp64,mixed,closure")
    ap.add_argument("--eps", type=float, default=1e-2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-error", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="first run one plain device-to-device copy of MIB MiB (the reference kernel that "
                         "scales the HBM byte counters of a profiler run)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the solver has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2509_21832_amd import binding as B
    assert torch.cuda.is_available(), "no GPU"

    if args.copy_probe:
        n = args.copy_probe * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"copy probe: {args.copy_probe} MiB read, {args.copy_probe} MiB written")
        del a, b

    copy_gbs = copy_bandwidth(torch)
    log(f"device copy: {copy_gbs:.0f} GB/s (read + write)")

    p, Q, G = W.cavity2d(seed=0, eps=args.eps)
    pts = p["nx"] * p["ny"] * p["nv1"] * p["nv2"]
    forms = {}
    closure = None
    for form in [f for f in args.forms.split(",") if f]:
        pf = dict(p)
        pf["precision"] = form
        if form == "closure" and closure is None:
            # the network, trained on the GPU by the library's kernels (not timed)
            from paper_2509_21832_amd import closure as CL
            t0 = time.perf_counter()
            net, losses, nsamp = CL.trained_closure()
            closure = {"net": net, "kn_max": CL.KN_MAX, "residual": CL.RESIDUAL,
                       "train_seconds": time.perf_counter() - t0, "train_samples": nsamp,
                       "final_loss": float(losses[-1])}
            log(f"closure network: {nsamp} samples, {closure['train_seconds']:.1f} s, loss {losses[-1]:.4f}")
        try:
            r = time_form(B, torch, pf, Q, G, args.steps, args.warmup, closure)
        except B.MMError as e:
            log(f"form {form}: {e}")
            continue
        r["value"] = pts * args.steps / r["seconds"]
        r["ms_per_step"] = 1e3 * r["seconds"] / args.steps
        r["err_vs_oracle"] = None if args.no_error else oracle_error(B, pf, args.eps, closure=closure)
        bpp = bytes_per_point(form)
        # dominant kernel: the fused phase-space pass (one launch per step, every point
        # read once and written once); its duration from HIP events on the solver's stream
        r["roofline"] = {"bound": "hbm", "kernel": "k_fused2d_lk", "bytes_per_launch": bpp * pts,
                         "achieved": bpp * pts / (r["micro_ms"] * 1e-3) / 1e9,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s"}
        r["roofline"]["frac"] = r["roofline"]["achieved"] / HBM_PEAK_GBS
        r["roofline"]["copy_gbs"] = copy_gbs
        r["roofline"]["frac_of_copy"] = r["roofline"]["achieved"] / copy_gbs
        r["roofline"]["traffic"] = traffic_entry(form)
        if form == "closure":
            r["roofline"] = None      # the closure pass touches only the solved cells
        forms[form] = r
        log(f"{form}: {r['ms_per_step']:.3f} ms/step, {r['value']:.3e} updates/s, micro pass "
            f"{r['micro_ms']:.3f} ms, err {r['err_vs_oracle']}")

    main_form = forms.get("fp64") or next(iter(forms.values()))
    out = {
        "metric": "phase-space cell-updates/s: FP64 vs mixed vs learned closure, at macro rel-L1 err",
        "value": main_form["value"],
        "unit": "phase-space cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_form["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"2D2V cavity box {p['nx']}x{p['ny']} cells x {p['nv1']}x{p['nv2']} velocity "
                               f"nodes on [-7,7]^2, walls + moving lid u_w=0.2, eps={args.eps:g}, FP64",
                   "phase_points": pts, "eps": args.eps, "seed": 0},
        "roofline": main_form["roofline"],
        "err_vs_oracle": main_form["err_vs_oracle"],
        "forms": {k: {"value": v["value"], "ms_per_step": v["ms_per_step"], "err_vs_oracle": v["err_vs_oracle"],
                      "speedup_vs_fp64": v["value"] / forms["fp64"]["value"] if "fp64" in forms else None,
                      "micro_pass_ms": v["micro_ms"], "wall_cells_ms": v["wall_ms"], "prep_ms": v["prep_ms"],
                      "macro_ms": v["macro_ms"], "closure_kernels_ms": v["closure_ms"],
                      "closure_fraction": v["closure_fraction"],
                      "roofline_frac": v["roofline"]["frac"] if v["roofline"] else None}
                  for k, v in forms.items()},
        "kernel_hash": kernel_hash(),
    }
    if closure is not None:
        out["closure_training"] = {k: closure[k] for k in ("train_seconds", "train_samples", "final_loss")}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(p, Q, G)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
