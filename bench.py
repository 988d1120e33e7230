"""Throughput of the micro-macro ES-BGK step on one MI355X.

Workload (default): the 256 x 256 x 32 x 32 cavity box (67,108,864 phase-space
points; walls, moving lid, seeded density/temperature perturbations, eps =
1e-2), FP64.  A step is one full micro-macro step over the whole grid.  The
same line reports the mixed-precision form (g stored in FP32) and the
learned-closure form (network trained on the GPU before the timed region, on
snapshots of the solver's own runs; its first 40 steps solve every cell while
the micro part relaxes from g = 0) on the same workload, each form's
macro-moment error against the FP64 oracle after 100 steps, the phase-space
pass's HBM roofline fraction, and the oracle timed on the host cores.

Beside the headline the line carries `sweeps`: the same step timed on the
cavity box at every Knudsen number of its sweep (FP64 and g in FP32), on the
512 x 512 x 48 x 48 Gaussian blast (g in FP32, and FP64 for the speedup), and
in the learned-closure form at three Knudsen numbers, each with its error
against a stored oracle result and its phase-space pass against the roofline.

Every timed form first runs at least 200 ms of warm-up steps (and at least W
steps), so clocks and caches are in their steady state.

Prints one JSON line.  Usage:
  python bench.py [--gpus 1] [--steps K] [--warmup W] [--forms fp64,mixed,closure] [--no-cpu] [--no-sweep]
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
GOLDEN_C4 = os.path.join(ROOT, "tests", "golden", "c4_blast_checkpoints.npz")
WARMUP_SECONDS = 0.2
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
    """A solver of the form; the closure form runs through its initial layer with every
    cell solved first.  Returns (solver, steps already run)."""
    s = B.Solver(p, Q, G)
    done = 0
    if p["precision"] == "closure":
        from paper_2509_21832_amd import closure as CL
        done = CL.start(s, closure["net"], closure["kn_max"], residual=closure["residual"])
    return s, done


def time_form(B, torch, p, Q, G, steps, warmup, closure=None, warmup_seconds=WARMUP_SECONDS):
    s, done = make_solver(B, p, Q, G, closure)
    closure_start = done              # the initial layer has no closure cells
    # warm-up: at least `warmup` steps and at least warmup_seconds of them
    s.step(max(warmup, 1))
    done += max(warmup, 1)
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < warmup_seconds:
        s.step(5)
        done += 5
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
        ncl, _ = s.closure_cells()          # counted since the threshold was attached
        frac = ncl / ((done - closure_start + 2 * steps) * p["nx"] * p["ny"])
    s.close()
    return {"seconds": t3 - t2, "seconds_timed_run": t1 - t0,
            "micro_ms": ms_micro / max(n_micro, 1), "prep_ms": ms_prep / max(n_prep, 1),
            "macro_ms": ms_macro / max(n_macro, 1), "wall_ms": ms_wall / max(n_wall, 1),
            "closure_ms": ms_cl / max(n_cl, 1), "launches": n_micro,
            "closure_fraction": frac, "warmup_steps": done}


def _golden_cells(ref, key, ny, nx):
    """Stored oracle values on every stride-th cell and (where stored) the boundary ring:
    (mask [ny][nx], values [ny][nx][6] with NaN off the mask)."""
    st = int(ref["stride"])
    vals = np.full((ny, nx, 6), np.nan)
    vals[::st, ::st] = ref[key + "_sample"]
    if key + "_row_lo" in ref:
        vals[0] = ref[key + "_row_lo"]
        vals[-1] = ref[key + "_row_hi"]
        vals[:, 0] = ref[key + "_col_lo"]
        vals[:, -1] = ref[key + "_col_hi"]
    return ~np.isnan(vals[:, :, 0]), vals


def oracle_error(B, p, eps, seed=0, closure=None):
    """Macro rel-L1 after 100 steps of the cavity box against the oracle's stored result
    (every 4th cell in x and y, and the whole boundary ring)."""
    if not os.path.exists(GOLDEN):
        return None
    ref = np.load(GOLDEN)
    key = f"eps{eps:g}"
    if key + "_sample" not in ref:
        return None
    p0, Q0, G0 = W.cavity2d(seed=seed, eps=eps)
    p0["precision"] = p["precision"]
    s, done = make_solver(B, p0, Q0, G0, closure)
    with s:
        s.step(int(ref["steps"]) - done)
        Q = s.moments().reshape(p0["ny"], p0["nx"], 6)
    mask, vals = _golden_cells(ref, key, p0["ny"], p0["nx"])
    return float(np.abs(Q[mask] - vals[mask]).sum() / np.abs(vals[mask]).sum())


def oracle_error_c4(B, p, steps=10):
    """Macro rel-L1 of the 512^2 x 48^2 blast after `steps` steps against the oracle's
    stored checkpoint (every 8th cell)."""
    if not os.path.exists(GOLDEN_C4):
        return None
    ref = np.load(GOLDEN_C4)
    key = f"step{steps}"
    if key + "_sample" not in ref:
        return None
    p0, Q0, G0 = W.blast2d(seed=0)
    p0["precision"] = p["precision"]
    with B.Solver(p0, Q0, G0) as s:
        s.step(steps)
        Q = s.moments().reshape(p0["ny"], p0["nx"], 6)
    st = int(ref["stride"])
    a, b = Q[::st, ::st, :], ref[key + "_sample"]
    return float(np.abs(a - b).sum() / np.abs(b).sum())


def cpu_baseline(p, seeds=(0, 1, 2), gen=None, one_thread=True):
    """The oracle on the host cores, on a bounded sample of the workload: one full-size
    step from each seeded initial state (all OpenMP threads; the median is the value),
    then one full step on a single thread."""
    import oracle
    gen = gen or (lambda sd: W.cavity2d(seed=sd, eps=p["eps"]))
    threads = oracle.threads()
    pts = p["nx"] * p["ny"] * p["nv1"] * p["nv2"]
    per = []
    for sd in seeds:
        p0, Q, G = gen(sd)
        t0 = time.perf_counter()
        oracle.run(p0, Q.reshape(-1), G.reshape(-1), 1)
        per.append(time.perf_counter() - t0)
    med = float(np.median(per))
    out = {"value": pts / med, "unit": "phase-space cell-updates/s", "cores": threads, "kind": "oracle",
           "sample": f"1 full step of the {p['nx']}x{p['ny']}x{p['nv1']}x{p['nv2']} workload from each of seeds "
                     f"{list(seeds)} ({', '.join(f'{x:.2f}' for x in per)} s; median {med:.2f} s per step, "
                     f"{threads} OpenMP threads)"}
    if one_thread:
        oracle.set_threads(1)
        try:
            p0, Q, G = gen(seeds[0])
            t0 = time.perf_counter()
            oracle.run(p0, Q.reshape(-1), G.reshape(-1), 1)
            per1 = time.perf_counter() - t0
        finally:
            oracle.set_threads(threads)
        out["value_1thread"] = pts / per1
        out["sample"] += f", then 1 step on 1 thread ({per1:.2f} s)"
    return out


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


def traffic_entry(precision, workload="cavity"):
    """HBM bytes of the phase-space pass from committed rocprofv3 counter runs, if they
    were taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    e = d.get(precision if workload == "cavity" else f"{workload}_{precision}")
    if not e or e.get("kernel_hash") != kernel_hash():
        return None
    return e.get("bytes_per_launch")


def roofline(form, pts, micro_ms, copy_gbs):
    """Roofline object of the fused phase-space pass: algorithmic bytes (read g once,
    write g once) over its mean duration from HIP events on the solver's stream."""
    bpp = bytes_per_point(form)
    r = {"bound": "hbm", "kernel": "k_fused2d_lk", "bytes_per_launch": bpp * pts,
         "achieved": bpp * pts / (micro_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    r["frac"] = r["achieved"] / HBM_PEAK_GBS
    r["copy_gbs"] = copy_gbs
    r["frac_of_copy"] = r["achieved"] / copy_gbs
    r["traffic"] = None
    return r


def run_form(B, torch, form, p, Q, G, steps, warmup, copy_gbs, closure=None, err=None, warmup_seconds=WARMUP_SECONDS):
    pf = dict(p)
    pf["precision"] = form
    pts = pf["nx"] * pf["ny"] * pf["nv1"] * pf["nv2"]
    r = time_form(B, torch, pf, Q, G, steps, warmup, closure, warmup_seconds)
    r["value"] = pts * steps / r["seconds"]
    r["ms_per_step"] = 1e3 * r["seconds"] / steps
    r["err_vs_oracle"] = err(pf) if err else None
    r["roofline"] = roofline(form, pts, r["micro_ms"], copy_gbs) if form != "closure" else None
    return r


def summary(r, base=None):
    """The figures of one timed form that go into the JSON line."""
    out = {"value": r["value"], "ms_per_step": r["ms_per_step"], "err_vs_oracle": r["err_vs_oracle"],
           "micro_pass_ms": r["micro_ms"], "wall_cells_ms": r["wall_ms"], "prep_ms": r["prep_ms"],
           "macro_ms": r["macro_ms"], "closure_kernels_ms": r["closure_ms"],
           "closure_fraction": r["closure_fraction"], "warmup_steps": r["warmup_steps"],
           "roofline_frac": r["roofline"]["frac"] if r["roofline"] else None,
           "achieved_gbs": r["roofline"]["achieved"] if r["roofline"] else None}
    out["speedup_vs_fp64"] = r["value"] / base["value"] if base else None
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--forms", default="fp64,mixed,closure")
    ap.add_argument("--eps", type=float, default=1e-2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-error", action="store_true")
    ap.add_argument("--no-sweep", action="store_true",
                    help="time only the headline workload (no eps sweeps, no 512^2 x 48^2 blast)")
    ap.add_argument("--warmup-seconds", type=float, default=WARMUP_SECONDS,
                    help="least time of warm-up steps per form (0 for profiler runs)")
    ap.add_argument("--workload", default="cavity", choices=("cavity", "blast"),
                    help="headline workload: the 256^2 x 32^2 cavity box (default) or the 512^2 x 48^2 Gaussian "
                         "blast (forms fp64 and mixed only; implies --no-sweep)")
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

    def c3_err(eps, closure=None):
        return None if args.no_error else (lambda pf: oracle_error(B, pf, eps, closure=closure))

    if args.workload == "blast":
        p, Q, G = W.blast2d(seed=0)
        args.no_sweep = True
        args.forms = ",".join(f for f in args.forms.split(",") if f != "closure")

        def c3_err(eps, closure=None):       # noqa: F811 (the blast's own stored checkpoint)
            return None if args.no_error else (lambda pf: oracle_error_c4(B, pf))
    else:
        p, Q, G = W.cavity2d(seed=0, eps=args.eps)
    pts = p["nx"] * p["ny"] * p["nv1"] * p["nv2"]
    forms = {}
    closure = None

    def get_closure():
        nonlocal closure
        if closure is None:
            # the network, trained on the GPU by the library's kernels (not timed)
            from paper_2509_21832_amd import closure as CL
            t0 = time.perf_counter()
            net, losses, nsamp = CL.trained_closure()
            closure = {"net": net, "kn_max": CL.KN_MAX, "residual": CL.RESIDUAL,
                       "train_seconds": time.perf_counter() - t0, "train_samples": nsamp,
                       "final_loss": float(losses[-1])}
            log(f"closure network: {nsamp} samples, {closure['train_seconds']:.1f} s, loss {losses[-1]:.4f}")
        return closure

    for form in [f for f in args.forms.split(",") if f]:
        cl = get_closure() if form == "closure" else None
        try:
            r = run_form(B, torch, form, p, Q, G, args.steps, args.warmup, copy_gbs, cl, c3_err(args.eps, cl),
                         args.warmup_seconds)
        except B.MMError as e:
            log(f"form {form}: {e}")
            continue
        if r["roofline"]:
            r["roofline"]["traffic"] = traffic_entry(form, args.workload)
        forms[form] = r
        log(f"{form}: {r['ms_per_step']:.3f} ms/step, {r['value']:.3e} updates/s, micro pass "
            f"{r['micro_ms']:.3f} ms, err {r['err_vs_oracle']}")

    sweeps = None
    if not args.no_sweep:
        sweeps = {"c3_cavity_eps": [], "c4_blast": {}, "c5_closure_eps": []}
        base = {}
        # the cavity box at every eps of its sweep (and 3e-3 for the closure's baseline)
        for eps in (1e-3, 3e-3, 1e-2, 1e-1, 1.0):
            pe, Qe, Ge = W.cavity2d(seed=0, eps=eps)
            row = {"eps": eps}
            for form in ("fp64", "mixed"):
                if eps == args.eps and form in forms:
                    r = forms[form]
                else:
                    r = run_form(B, torch, form, pe, Qe, Ge, args.steps, args.warmup, copy_gbs,
                                 err=c3_err(eps), warmup_seconds=args.warmup_seconds)
                row[form] = summary(r, base.get(eps))
                if form == "fp64":
                    base[eps] = r
                log(f"c3 eps={eps:g} {form}: {r['ms_per_step']:.3f} ms/step, pass {r['micro_ms']:.3f} ms, "
                    f"err {r['err_vs_oracle']}")
            sweeps["c3_cavity_eps"].append(row)
        # the learned closure at three eps, against the FP64 step at the same eps
        if "closure" in args.forms:
            for eps in (1e-3, 3e-3, 1e-2):
                pe, Qe, Ge = W.cavity2d(seed=0, eps=eps)
                cl = get_closure()
                if eps == args.eps and "closure" in forms:
                    r = forms["closure"]
                else:
                    r = run_form(B, torch, "closure", pe, Qe, Ge, args.steps, args.warmup, copy_gbs, cl,
                                 c3_err(eps, cl), args.warmup_seconds)
                row = {"eps": eps, "closure": summary(r, base.get(eps))}
                sweeps["c5_closure_eps"].append(row)
                log(f"c5 eps={eps:g}: {r['ms_per_step']:.3f} ms/step, closure cells {r['closure_fraction']}, "
                    f"err {r['err_vs_oracle']}")
        # the 512^2 x 48^2 blast: g in FP32, and FP64 for the speedup
        pb, Qb, Gb = W.blast2d(seed=0)
        c4 = {}
        for form in ("fp64", "mixed"):
            errf = None if args.no_error else (lambda pf: oracle_error_c4(B, pf))
            r = run_form(B, torch, form, pb, Qb, Gb, max(10, args.steps // 4), args.warmup, copy_gbs, err=errf,
                         warmup_seconds=args.warmup_seconds)
            c4[form] = r
            log(f"c4 {form}: {r['ms_per_step']:.3f} ms/step, pass {r['micro_ms']:.3f} ms, err {r['err_vs_oracle']}")
        sweeps["c4_blast"] = {
            "workload": f"2D2V Gaussian blast {pb['nx']}x{pb['ny']} cells x {pb['nv1']}x{pb['nv2']} velocity nodes "
                        f"on [-8,8]^2, walls, eps={pb['eps']:g}",
            "phase_points": pb["nx"] * pb["ny"] * pb["nv1"] * pb["nv2"],
            "err_steps": 10,
            "fp64": summary(c4["fp64"]), "mixed": summary(c4["mixed"], c4["fp64"]),
            "roofline_mixed": c4["mixed"]["roofline"], "roofline_fp64": c4["fp64"]["roofline"]}
        del Qb, Gb

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
        "config": {"workload": (f"2D2V cavity box {p['nx']}x{p['ny']} cells x {p['nv1']}x{p['nv2']} velocity "
                                f"nodes on [-7,7]^2, walls + moving lid u_w=0.2, eps={args.eps:g}, FP64"
                                if args.workload == "cavity" else
                                f"2D2V Gaussian blast {p['nx']}x{p['ny']} cells x {p['nv1']}x{p['nv2']} velocity "
                                f"nodes on [-8,8]^2, walls, eps={p['eps']:g}, FP64"),
                   "phase_points": pts, "eps": p["eps"], "seed": 0},
        "roofline": main_form["roofline"],
        "err_vs_oracle": main_form["err_vs_oracle"],
        "forms": {k: summary(v, forms.get("fp64")) for k, v in forms.items()},
        "sweeps": sweeps,
        "kernel_hash": kernel_hash(),
    }
    if closure is not None:
        out["closure_training"] = {k: closure[k] for k in ("train_seconds", "train_samples", "final_loss")}
    if not args.no_cpu:
        if args.workload == "blast":
            out["cpu_baseline"] = cpu_baseline(p, seeds=(0,), gen=lambda sd: W.blast2d(seed=sd), one_thread=False)
        else:
            out["cpu_baseline"] = cpu_baseline(p)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
