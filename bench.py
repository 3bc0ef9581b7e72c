"""Benchmark of the matrix-free Jacobian action (Eq. (2)) on one MI355X.

One step = one Jacobian-vector apply J(u) v (G -> B -> dual-number D -> B^T ->
G^T) in FP64 on the workload's seeded random u, v, with the inputs already
resident in HBM.  value = n_dofs * steps / elapsed / 1e9 (GDOF/s).

Also measured on the same line (not part of ``value``): the mixed-precision
Jacobian apply, the residual, the fused residual + Jacobian apply, the
adjoint-gradient time on the design workload, and the Newton-CG solve time,
each with its own timing; the roofline of the dominant kernel from hipEvents
recorded around every launch by the library; and the CPU oracle timed on a
bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GDOF/s of AD Jacobian-vector apply (FP64 vs mixed) + adjoint-gradient time"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP64_PEAK_TFS = 78.6           # 256 CU * 2.4 GHz * 128 FLOP/clk (vector FP64 FMA)
FP32_PEAK_TFS = 78.6           # scalar (non-packed) FP32 FMA: same lane rate as FP64


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def timed_loop(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    s = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(steps):
        fn()
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / steps  # ms per call


def kernel_profile(prob, fn, steps):
    import torch
    torch.cuda.synchronize()
    prob.profile(True)
    for _ in range(steps):
        fn()
    stats = prob.profile_read()
    prob.profile(False)
    return {k: {"launches": n, "avg_ms": ms / n} for k, (n, ms) in stats.items()}


def roofline(prob, op, prec, stats, kernel):
    bytes_, flops = prob.kernel_cost(op, prec)
    avg_s = stats[kernel]["avg_ms"] * 1e-3
    gbs = bytes_ / avg_s / 1e9
    tfs = flops / avg_s / 1e12
    peak_alu = FP64_PEAK_TFS if prec == "fp64" else FP32_PEAK_TFS
    t_mem = bytes_ / (HBM_PEAK_GBS * 1e9)
    t_alu = flops / (peak_alu * 1e12)
    if t_mem >= t_alu:
        r = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS}
    else:
        r = {"bound": "alu", "achieved": tfs, "peak": peak_alu, "unit": "TFLOP/s", "frac": tfs / peak_alu}
    r.update({"kernel": kernel, "avg_us": avg_s * 1e6, "algorithmic_bytes": bytes_,
              "algorithmic_flops": flops, "achieved_GBs": gbs, "achieved_TFLOPs": tfs,
              "traffic": None})
    return r


def cpu_baseline(w, inp, budget_s=12.0):
    """The oracle's Jacobian apply on the same workload, timed on host cores."""
    import threadpoolctl
    from oracle import Discretisation
    d = Discretisation(w.nx, w.ny, w.nz, w.k, w.nq, w.p, w.eps, vertices=inp["vertices"],
                       rho=inp["rho"], compute_load=False)
    threads = max([x.get("num_threads", 1) for x in threadpoolctl.threadpool_info()] + [1])
    n, t0 = 0, time.perf_counter()
    while True:
        d.jvp(inp["u"], inp["v"])
        n += 1
        el = time.perf_counter() - t0
        if el >= budget_s or n >= 5:
            break
    return {"value": w.n_dofs * n / el / 1e9, "unit": "GDOF/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} full Jacobian applies of the {w.name} workload ({el:.1f} s, "
                      f"dense-element NumPy/OpenBLAS, {os.cpu_count()} host CPUs visible)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the subdomain operator P is the identity on one GPU).", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2506_00746_amd as feod
    from workloads import WORKLOADS, make_inputs

    w = WORKLOADS[args.workload]
    inp = make_inputs(w)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    prob = feod.Problem(w.nx, w.ny, w.nz, w.k, w.nq, w.p, w.eps, vertices=inp["vertices"],
                        rho=inp["rho"], device=dev)
    u = torch.as_tensor(inp["u"], device=dev)
    v = torch.as_tensor(inp["v"], device=dev)
    jv = torch.empty_like(u)
    r = torch.empty_like(u)
    N = w.n_dofs

    def jvp64():
        prob.jacobian_apply(u, v, out=jv)

    log(f"[bench] {w.name}: N={N} E={w.n_elems} timed JVP fp64 x{args.steps}")
    ms = timed_loop(jvp64, args.steps, args.warmup)
    value = N / (ms * 1e-3) / 1e9
    stats = kernel_profile(prob, jvp64, min(args.steps, 50))
    roof = roofline(prob, "jvp", "fp64", stats, "element_jvp_f64")
    log(f"[bench] JVP fp64 {ms * 1e3:.1f} us/apply = {value:.2f} GDOF/s; kernels {stats}")

    rows = {"jvp_fp64": {"GDOF/s": value, "us_per_apply": ms * 1e3}}
    if not args.no_extras:
        def jvp32():
            prob.jacobian_apply(u, v, out=jv, prec="mixed")

        def res64():
            prob.residual(u, out=r)

        def resjvp64():
            prob.jacobian_apply(u, v, out=jv, residual_out=r)
        for name, fn, op, prec, kern in [("jvp_mixed", jvp32, "jvp", "mixed", "element_jvp_f32"),
                                         ("residual_fp64", res64, "residual", "fp64", "element_residual_f64"),
                                         ("residual_jvp_fp64", resjvp64, "resjvp", "fp64", "element_resjvp_f64")]:
            t = timed_loop(fn, args.steps, args.warmup)
            st = kernel_profile(prob, fn, min(args.steps, 50))
            rl = roofline(prob, op, prec, st, kern)
            rows[name] = {"GDOF/s": N / (t * 1e-3) / 1e9, "us_per_apply": t * 1e3,
                          "kernel_us": rl["avg_us"], "kernel_frac": rl["frac"], "kernel_bound": rl["bound"]}
            log(f"[bench] {name}: {rows[name]}")
        rows["jvp_mixed"]["speedup_vs_fp64_apply"] = rows["jvp_mixed"]["GDOF/s"] / value

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline ...")
        cpu = cpu_baseline(w, inp)
        log(f"[bench] cpu_baseline {cpu}")

    out = {"metric": METRIC, "value": value, "unit": "GDOF/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"{w.name}: {w.note}", "n_dofs": N, "n_elems": w.n_elems,
                      "order_k": w.k, "nq": w.nq, "p": w.p, "eps": w.eps, "seed": w.seed,
                      "parallelism": "single GPU"},
           "roofline": {k: roof[k] for k in ("bound", "achieved", "peak", "unit", "frac", "traffic")},
           "roofline_detail": roof, "cpu_baseline": cpu, "rows": rows}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
