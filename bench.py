#!/usr/bin/env python3
"""Throughput of the SSN kernel-OT solver on one MI355X.

A step is one full solve of one synthetic problem with inputs resident in HBM: setup (Gram matrices, mean
embeddings, q^2, Cholesky factor) and Algorithm 2 to |R(w)| <= 1e-6.  The workload is ``mix1000`` (n = 5000
samples per side, d = 10, two 4-component Gaussian mixtures, l = 1000 filling points), one instance per
seed.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--arm fp64|warm|mixed32|mixed16|mixed|all]
                    [--lanes L] [--no-cpu-baseline]

Each arm's K solves run twice: one at a time on one context, then as independent solves in flight together on
L lanes of ``kot_solve_batched`` (child contexts with a stream and a host thread each; default 8).  The rates
reported are those of the lanes pass (whole-job throughput); the one-at-a-time rate is kept beside them.

Arms: ``fp64`` cold start, FP64 everywhere; ``warm`` learned warm start, FP64; ``mixed32``, ``mixed16`` and
``mixed``: learned warm start with the CG matvec chain in FP32, BF16 and split BF16 (three BF16 products per
FP32 product) on the matrix cores, FP32 accumulation, inside FP64 iterative refinement.  ``value`` is the rate
of the last arm run (``mixed`` by default); every arm's rate is in ``config.arms``.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

TRAFFIC_FILE = os.path.join(ROOT, "profiles", "gemm_f64_mix1000_traffic.md")
GEMM_SOURCE = os.path.join(ROOT, "paper_2310_14087_amd", "csrc", "k_gemm.hip")

PEAK = {  # MI355X published dense peaks
    "fp64_tflops": 78.6,
    "fp32_tflops": 157.3,
    "bf16_tflops": 2500.0,
    "hbm_gbs": 8000.0,
}


# profiler class -> (bound, published peak, unit)
CLASS_ROOF = {
    "gemm_f64": ("mfma", PEAK["fp64_tflops"], "TFLOP/s"),
    "eig_sweep": ("mfma", PEAK["fp64_tflops"], "TFLOP/s"),
    "gemv_f64": ("hbm", PEAK["hbm_gbs"], "GB/s"),
    "gemm_f32": ("mfma", PEAK["fp32_tflops"], "TFLOP/s"),
    "gemm_bf16": ("mfma", PEAK["bf16_tflops"], "TFLOP/s"),
    "potential": ("alu", PEAK["fp64_tflops"], "TFLOP/s"),
}


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(workload: str):
    """Time the CPU oracle (as it stands) on one full solve of instance 0 of the same workload."""
    import numpy as np
    from threadpoolctl import threadpool_info
    from oracle import kot_oracle as ko
    from paper_2310_14087_amd.inputs import make_problem

    p = make_problem(workload, 0)
    t0 = time.perf_counter()
    core = ko.setup(p.xs, p.ys, p.xf, p.yf, p.sigma, p.lam1, p.lam2)
    res = ko.solve(core, ko.Params(tol=p.tol))
    dt = time.perf_counter() - t0
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    return dict(value=1.0 / dt, unit="solves/s", cores=threads, kind="oracle",
                sample=f"1 full oracle solve (setup + Algorithm 2, {res['iters']} iterations, status "
                       f"{res['status']}) of {workload} instance 0, {dt:.1f} s wall, numpy/OpenBLAS FP64",
                cpu=_cpu_model())


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def gemm_traffic():
    """HBM bytes per FP64 GEMM call from the committed counter summary (FETCH_SIZE + WRITE_SIZE, scaled by a
    plain copy of known size), or None when there is none or the GEMM source changed since it was taken."""
    import hashlib
    try:
        with open(TRAFFIC_FILE) as f:
            kv = dict(line.strip().lstrip("- ").split(": ", 1) for line in f if ": " in line)
        with open(GEMM_SOURCE, "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
        if kv.get("gemm_source_sha256") != sha:
            return None
        return float(kv["traffic_bytes_per_call"])
    except (OSError, KeyError, ValueError):
        return None


def copy_calibrate(mb):
    """Device-to-device copies of a known size, for scaling the HBM byte counters."""
    import torch
    n = int(mb * (1 << 20) // 8)
    src = torch.ones(n, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration": {"bytes_read_per_copy": 8 * n, "bytes_written_per_copy": 8 * n,
                                           "copies": 3}}), flush=True)


def sweep_bench(a):
    """Section 5's synthetic sweep, SSN side: 3- vs 5-Gaussian mixtures in d = 2, 5, 10 with Sobol filling points
    and l = n in {100, 200, 500, 1000}, stopped at |R(w)| < 0.005; mean wall time per solve for the paper's FP64
    SSN (plain CG) and for the accelerated configuration (Jacobi CG, BF16x3 chain, learned start)."""
    import numpy as np
    import torch
    from paper_2310_14087_amd import kotssn, warmstart
    from paper_2310_14087_amd.inputs import make_problem
    dev = torch.device("cuda:0")
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    theta, F, H, _ = warmstart.load()
    theta_dev = torch.from_numpy(theta).to(dev)
    ctx = kotssn.Context(0)
    reps = max(1, a.steps // 2)
    rows = []
    for d in (2, 5, 10):
        for l in (100, 200, 500, 1000):
            probs = [make_problem(f"sweep_d{d}", s, l=l, n=l) for s in range(reps)]
            inputs = [(t(p.xs), t(p.ys), t(p.xf), t(p.yf)) for p in probs]
            row = dict(d=d, l=l, n=l)
            for arm in ("fp64", "fast"):
                def prm(p):
                    kw = dict(sigma=p.sigma, lambda1=p.lam1, lambda2=p.lam2, tol=p.tol)
                    if arm == "fast":
                        kw.update(precond=kotssn.KOT_PRECOND_JACOBI, precision=kotssn.KOT_MIXED_BF16X3,
                                  ws_F=kotssn.N_FEATURES, ws_H=H, ws_theta=theta_dev.data_ptr())
                    return kotssn.default_params(**kw)
                ctx.solve(*inputs[0], prm(probs[0]))  # warm-up (workspace sizing)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                out = []
                for i, p in enumerate(probs):
                    out.append(ctx.solve(*inputs[i], prm(p))[2])
                    _log(f"sweep d={d} l={l} {arm} instance {i}: iters={out[-1].iters} status={out[-1].status}")
                torch.cuda.synchronize()
                dt = (time.perf_counter() - t0) / len(probs)
                row[arm] = dict(ms=1e3 * dt, iters=[r.iters for r in out], residual=max(r.residual for r in out),
                                converged=sum(1 for r in out if r.status == kotssn.KOT_OK))
                _log(f"sweep d={d} l={l} {arm}: {1e3 * dt:.2f} ms/solve iters={row[arm]['iters']}")
            rows.append(row)
    ctx.close()
    print(json.dumps({"metric": "mean SSN solve time to |R(w)| < 0.005 on Section 5's synthetic sweep",
                      "unit": "ms/solve", "higher_is_better": False, "data": "synthetic",
                      "config": {"workload": "sweep: mixtures of 3 vs 5 Gaussians, d in {2,5,10}, Sobol filling, "
                                             "sigma^2=0.005, lambda1=1/l, lambda2=1/sqrt(n), n=l",
                                 "instances_per_point": reps},
                      "rows": rows}), flush=True)


def batch_bench(a):
    """Uneven batch (n ~ U{200..2000}, l ~ U{100..400}, d ~ U{2..10}): solves/s through kot_solve_batched with
    `lanes` concurrent streams vs one lane; FP32 CG chain, FP64 projections."""
    import numpy as np
    import torch
    from paper_2310_14087_amd import kotssn
    from paper_2310_14087_amd.inputs import make_problem
    dev = torch.device("cuda:0")
    probs = [make_problem("batch", s) for s in range(a.batch)]
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    inputs = [(t(p.xs), t(p.ys), t(p.xf), t(p.yf)) for p in probs]
    prms = [kotssn.default_params(sigma=p.sigma, lambda1=p.lam1, lambda2=p.lam2, tol=p.tol, precision=1, max_iter=60)
            for p in probs]
    ctx = kotssn.Context(0)
    if a.tune:
        if os.path.exists(a.tune):
            ctx.autotune_load(a.tune)
        else:
            ctx.autotune(sorted({p.l for p in probs}), a.tune)
    res = {}
    for lanes in sorted({1, a.lanes}):
        ctx.solve_batched(inputs[:min(4, len(inputs))], prms[:min(4, len(inputs))], lanes=lanes)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = ctx.solve_batched(inputs, prms, lanes=lanes)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        conv = sum(1 for _, r in out if r.status == kotssn.KOT_OK)
        res[f"lanes{lanes}"] = dict(solves_per_s=len(probs) / dt, seconds=dt, converged=conv,
                                    iters=[r.iters for _, r in out])
        _log(f"lanes={lanes}: {len(probs) / dt:.2f} solves/s, {conv}/{len(probs)} converged")
    ctx.close()
    print(json.dumps({"metric": "batched SSN solves/s (uneven problems)", "problems": len(probs),
                      "sizes": {"l": [p.l for p in probs], "n": [p.n_src for p in probs], "d": [p.d for p in probs]},
                      "results": res}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=24)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="mix1000",
                    help="mix1000 (the metric line) or sweep (Section 5's synthetic sweep, its own JSON line)")
    ap.add_argument("--arm", default="all", choices=["fp64", "warm", "mixed32", "mixed16", "mixed", "all"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="skip the roofline pass")
    ap.add_argument("--roofline-solves", type=int, default=3,
                    help="solves of the final arm in the roofline pass (after the timed run)")
    ap.add_argument("--overlap", type=int, default=1, choices=[0, 1],
                    help="1: extragradient branch on a second stream (the default of the library)")
    ap.add_argument("--precond", default="auto", choices=["auto", "none", "jacobi"],
                    help="Schur-system CG as in the paper (none) or Jacobi-preconditioned; auto: none on the "
                         "plain fp64 arm, jacobi on the accelerated arms")
    ap.add_argument("--batch", type=int, default=0,
                    help="instead of the metric line: time kot_solve_batched on this many 'batch' problems")
    ap.add_argument("--lanes", type=int, default=8,
                    help="independent solves in flight (kot_solve_batched lanes, one stream and host thread each); "
                         "1: one solve at a time on the main context")
    ap.add_argument("--tune", default=None, help="autotune table to load (or create when missing)")
    ap.add_argument("--copy-calibrate", type=float, default=0.0,
                    help="instead of the metric line: copy this many MiB device-to-device three times")
    a = ap.parse_args()

    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(json.dumps({"error": "this solver runs on one GPU; --gpus must be 1 (a multi-GPU run would only "
                                   "repeat independent solves per GPU and is not part of this build)"}))
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2310_14087_amd import kotssn
    from paper_2310_14087_amd.inputs import make_problem

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if a.batch:
        return batch_bench(a)
    if a.workload == "sweep":
        return sweep_bench(a)
    if a.copy_calibrate > 0:
        return copy_calibrate(a.copy_calibrate)
    n_inst = max(1, a.steps)
    _log(f"generating {n_inst} {a.workload} instances")
    probs = [make_problem(a.workload, s) for s in range(n_inst)]
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    dev_inputs = [(t(p.xs), t(p.ys), t(p.xf), t(p.yf)) for p in probs]
    torch.cuda.synchronize()

    ctx = kotssn.Context(0)
    base = [dict(sigma=p.sigma, lambda1=p.lam1, lambda2=p.lam2, tol=p.tol) for p in probs]
    arms = ["fp64", "warm", "mixed32", "mixed16", "mixed"] if a.arm == "all" else [a.arm]
    theta_dev, H = None, 0
    if any(x != "fp64" for x in arms):
        from paper_2310_14087_amd import warmstart
        theta, F, H, meta = warmstart.load()
        theta_dev = torch.from_numpy(theta).to(dev)

    def params(i, arm):
        jac = a.precond == "jacobi" or (a.precond == "auto" and arm != "fp64")
        kw = dict(base[i], overlap=a.overlap,
                  precond=kotssn.KOT_PRECOND_JACOBI if jac else kotssn.KOT_PRECOND_NONE)
        if arm != "fp64":
            kw.update(ws_F=kotssn.N_FEATURES, ws_H=H, ws_theta=theta_dev.data_ptr())
        if arm == "mixed":
            kw.update(precision=kotssn.KOT_MIXED_BF16X3)
        elif arm == "mixed16":
            kw.update(precision=kotssn.KOT_MIXED_BF16)
        elif arm == "mixed32":
            kw.update(precision=kotssn.KOT_FP32)
        return kotssn.default_params(**kw)

    def run_arm(arm):
        """The arm's `steps` solves one after another on the main context (`overlap` as given), then, with
        lanes > 1, the same solves again through kot_solve_batched: independent instances on `lanes` child
        contexts, each with its own stream and host thread.  Returns (sequential results, seconds), and the
        lanes' (results, seconds) or None."""
        for w in range(a.warmup):
            _log(f"{arm} warmup {w}")
            ctx.solve(*dev_inputs[w % n_inst], params(w % n_inst, arm))
        torch.cuda.synchronize()
        results = []
        t0 = time.perf_counter()
        for k in range(a.steps):
            i = k % n_inst
            _, _, r = ctx.solve(*dev_inputs[i], params(i, arm))
            results.append(r)
            _log(f"{arm} step {k}: instance {i} status={r.status} iters={r.iters} warm_used={r.warm_used} "
                 f"residual={r.residual:.2e} ot={r.ot:.10g} device_ms={r.time_ms:.1f}")
        torch.cuda.synchronize()
        seq = (results, time.perf_counter() - t0)
        if a.lanes <= 1:
            return seq, None
        idx = [k % n_inst for k in range(a.steps)]
        batch_in = [dev_inputs[i] for i in idx]
        batch_prm = [params(i, arm) for i in idx]
        nw = min(a.lanes, a.steps)
        for w in range(a.warmup):  # every lane gets a solve: its workspace and GEMM unit lists exist before timing
            ctx.solve_batched(batch_in[:nw], batch_prm[:nw], lanes=a.lanes)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = ctx.solve_batched(batch_in, batch_prm, lanes=a.lanes)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        lres = [r for _, r in out]
        for k, r in enumerate(lres):
            _log(f"{arm} lanes solve {k}: instance {idx[k]} status={r.status} iters={r.iters} "
                 f"residual={r.residual:.2e} ot={r.ot:.10g}")
        return seq, (lres, el)

    def roofline_pass(arm):
        """Per-class launch timing with HIP events around every launch, outside the timed loop and on one
        stream (overlap=0), so that each launch's duration is its own and no event lands in the timed run."""
        ctx.profile_start()
        t0 = time.perf_counter()
        for k in range(a.roofline_solves):
            i = k % n_inst
            prm = params(i, arm)
            prm.overlap = 0
            ctx.solve(*dev_inputs[i], prm)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return ctx.profile_stop(), wall

    out_arms = {}
    prof = None
    elapsed = None
    for arm in arms:
        (sres, sel), lan = run_arm(arm)
        results, el = lan if lan else (sres, sel)
        ok = lambda rs: sum(1 for r in rs if r.status == kotssn.KOT_OK and r.residual <= 1e-6)
        conv = ok(results)
        out_arms[arm] = dict(solves_per_s=a.steps / el, ms_per_solve=1e3 * el / a.steps, converged=conv,
                             iters=[r.iters for r in results], eig_sweeps=[r.eig_sweeps_total for r in results],
                             cg_iters=[r.cg_iters_total for r in results],
                             lowp_directions=[r.lowp_directions for r in results], ot=[r.ot for r in results])
        if lan:
            out_arms[arm]["sequential"] = dict(
                solves_per_s=a.steps / sel, ms_per_solve=1e3 * sel / a.steps, converged=ok(sres),
                ot_max_abs_diff_vs_lanes=max(abs(x.ot - y.ot) for x, y in zip(sres, results)))
        if arm == arms[-1]:
            elapsed, final = el, arm
            if not a.no_profile:
                _log(f"{arm}: roofline pass ({a.roofline_solves} solves, one stream, events on every launch)")
                prof, prof_wall = roofline_pass(arm)
        _log(f"{arm}: {a.steps / el:.2f} solves/s, {conv}/{a.steps} converged"
             + (f" ({a.lanes} lanes; one at a time {a.steps / sel:.2f} solves/s)" if lan else ""))
    ctx.close()
    if "fp64" in out_arms:
        for arm in ("warm", "mixed32", "mixed16", "mixed"):
            if arm in out_arms:
                out_arms[arm]["ot_rel_dev_vs_fp64"] = max(
                    abs(x - y) / abs(y) for x, y in zip(out_arms[arm]["ot"], out_arms["fp64"]["ot"]))
                out_arms[f"speedup_{arm}_vs_fp64"] = out_arms[arm]["solves_per_s"] / out_arms["fp64"]["solves_per_s"]
    value = a.steps / elapsed
    out = {
        "metric": "SSN solves/s to residual<=1e-6 at l=1000: plain FP64 vs warm-start+mixed",
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * elapsed / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{a.workload}: n=5000/side, d=10, two 4-component mixtures, l=1000, "
                               f"sigma^2=0.005 on unit-cube data, lambda1=1/l, lambda2=1/sqrt(n), tol 1e-6",
                   "arm": final, "instances": n_inst, "lanes": max(1, a.lanes), "overlap": a.overlap,
                   "precond": a.precond,
                   "arms": out_arms},
    }
    if prof:
        dom = max(prof, key=lambda c: prof[c]["ms"])
        pc = prof[dom]
        bound, peak, unit = CLASS_ROOF[dom]
        sec = pc["ms"] * 1e-3
        if bound == "hbm":
            ach = pc["bytes"] / sec / 1e9 if sec > 0 else 0.0
        else:
            ach = pc["flops"] / sec / 1e12 if sec > 0 else 0.0
        nl = max(1, pc["launches"])
        out["roofline"] = {"bound": bound, "achieved": ach, "peak": peak, "unit": unit, "frac": ach / peak,
                           "traffic": gemm_traffic() if dom == "gemm_f64" else None,
                           "traffic_unit": "HBM bytes per call", "kernel": dom, "launches": pc["launches"],
                           "avg_launch_us": 1e6 * sec / nl, "flops_per_launch": pc["flops"] / nl,
                           "algorithmic_bytes_per_launch": pc["bytes"] / nl, "share_of_pass": sec / prof_wall,
                           "measured_on": f"{a.roofline_solves} solves of the {final} arm after the timed run, "
                                          "one stream, HIP events around each launch"}
        out["profile"] = {c: {"launches": v["launches"], "ms": round(v["ms"], 3),
                              "tflops": (v["flops"] / (v["ms"] * 1e-3) / 1e12) if v["ms"] > 0 else 0.0}
                          for c, v in prof.items()}
    if not a.no_cpu_baseline:
        _log("timing the CPU oracle")
        out["cpu_baseline"] = cpu_baseline(a.workload)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
