"""Benchmark of the matrix-free Jacobian action (Eq. (2)) on one MI355X.

One step = one Jacobian-vector apply J(u) v (G -> B -> dual-number D -> B^T ->
G^T) in FP64 on the workload's seeded random u, v, with the inputs already
resident in HBM.  value = n_dofs * steps / elapsed / 1e9 (GDOF/s) on the
64^3 Q4 p = 2.5 workload (16,974,593 DOFs), the largest of the five and the
one the FP64-vs-mixed throughput comparison is made on.  The same K steps are
timed again in --repeats further windows; their median is reported beside
value.

Also reported on the same JSON line (each timed separately, none of it part
of ``value``): the mixed-precision Jacobian apply, the residual, the fused
residual + Jacobian apply, the same applies on the other workloads, the
Newton-CG and adjoint-gradient times (wall and kernel sum), the element
tangent matrices, partial assembly, single applies with the Infinity Cache
flushed, the mixed-precision error at random and smooth inputs, the roofline of
the dominant (element) kernel, whose duration is timed with events over
back-to-back launches of the element stage alone on the library's stream,
its HBM traffic from the committed rocprofv3 summary (when measured on the
current kernel sources), and the CPU oracle timed on a bounded sample.

Before the W warm-up steps the apply runs untimed for --settle seconds (0.5 by
default): an idle GPU raises its clocks during the first milliseconds of work,
and the K timed steps measure the steady state.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c3]
       [--settle S] [--repeats R] [--no-extras] [--no-cpu-baseline]
       [--calibrate-copy] [--cpu-table]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GDOF/s of AD Jacobian-vector apply (FP64 vs mixed) + adjoint-gradient time"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP64_PEAK_TFS = 78.6           # 256 CU * 2.4 GHz * 128 FLOP/clk (vector FP64 FMA)
FP32_PEAK_TFS = 78.6           # non-packed FP32 FMA (packed FP32 is compiled out): same lane rate as FP64
FP32_PUBLISHED_TFS = 157.3     # MI355X's published FP32 vector peak (packed FP32), reported beside


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def settle(fn, seconds):
    """Run fn untimed, in synchronised rounds of 20, for at least `seconds` of
    wall time: an idle GPU raises its clocks over the first milliseconds of
    work, and the timed steps should see the steady state."""
    import torch
    t0 = time.time()
    while time.time() - t0 < seconds:
        for _ in range(20):
            fn()
        torch.cuda.synchronize()


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
    """Per-kernel average durations from the library's own hipEvents."""
    import torch
    torch.cuda.synchronize()
    prob.profile(True)
    for _ in range(steps):
        fn()
    stats = prob.profile_read()
    prob.profile(False)
    return {k: {"launches": n, "avg_ms": ms / n} for k, (n, ms) in stats.items()}


def element_kernel_ms(prob, u, v, op, prec, steps, warmup):
    """Average duration of the element kernel alone: back-to-back launches
    timed with events on the stream the library launches on."""
    return timed_loop(lambda: prob.element_vectors(op, u, v, prec=prec), steps, warmup)


def ad_overhead(prob, u, v, args):
    """The FP64 Jacobian element kernel with J_D from dual numbers and with the
    hand-coded J_D (the paper's Table 1 compares AD with hand-coded, HND);
    the two timings are interleaved twice."""
    d = h = 0.0
    for _ in range(2):
        d += element_kernel_ms(prob, u, v, "jvp", "fp64", args.steps, args.warmup)
        prob.set_tangent_mode("hand")
        h += element_kernel_ms(prob, u, v, "jvp", "fp64", args.steps, args.warmup)
        prob.set_tangent_mode("dual")
    return {"dual_us": d / 2 * 1e3, "hand_us": h / 2 * 1e3, "dual_vs_hand": d / h}


def stored_traffic(workload, kernel):
    """HBM bytes per launch from the committed rocprofv3 summary, if it was
    measured on the current kernel sources (else None)."""
    from paper_2506_00746_amd import profiling
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}.md")
    b, sha = profiling.read_traffic(path)
    return b if (b is not None and sha == profiling.kernel_source_sha256()) else None


def roofline(prob, op, prec, stats, kernel, kernel_ms=None):
    bytes_, flops = prob.kernel_cost(op, prec)
    avg_s = (kernel_ms if kernel_ms is not None else stats[kernel]["avg_ms"]) * 1e-3
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
    if prec != "fp64":
        r["frac_vs_published_fp32"] = tfs / FP32_PUBLISHED_TFS
    return r


def apply_rows(prob, u, v, w, args, only=None):
    """GDOF/s and kernel roofline of the applies of one workload."""
    import torch
    jv = torch.empty_like(u)
    r = torch.empty_like(u)
    N = w.n_dofs
    cases = [("jvp_fp64", lambda: prob.jacobian_apply(u, v, out=jv), "jvp", "fp64", "element_jvp_f64"),
             ("jvp_mixed", lambda: prob.jacobian_apply(u, v, out=jv, prec="mixed"), "jvp", "mixed",
              "element_jvp_f32"),
             ("residual_fp64", lambda: prob.residual(u, out=r), "residual", "fp64", "element_residual_f64"),
             ("residual_jvp_fp64", lambda: prob.jacobian_apply(u, v, out=jv, residual_out=r),
              "resjvp", "fp64", "element_resjvp_f64")]
    out = {}
    for name, fn, op, prec, kern in cases:
        if only is not None and name not in only:
            continue
        settle(fn, min(args.settle, 0.2))
        t = timed_loop(fn, args.steps, args.warmup)
        st = kernel_profile(prob, fn, min(args.steps, 50))
        k_ms = element_kernel_ms(prob, u, v, op, prec, args.steps, args.warmup)
        rl = roofline(prob, op, prec, st, kern, kernel_ms=k_ms)
        gt = st.get("gather_transpose", st.get("gather_transpose2", {"avg_ms": 0.0}))
        out[name] = {"GDOF/s": N / (t * 1e-3) / 1e9, "us_per_apply": t * 1e3, "kernel_us": rl["avg_us"],
                     "kernel_bound": rl["bound"], "kernel_frac": rl["frac"],
                     "kernel_frac_vs_published_fp32": rl.get("frac_vs_published_fp32"),
                     "kernel_TFLOPs": rl["achieved_TFLOPs"], "kernel_GBs": rl["achieved_GBs"],
                     "gather_t_us": gt["avg_ms"] * 1e3, "roofline": rl}
    if "jvp_fp64" in out and "jvp_mixed" in out:
        out["jvp_mixed"]["speedup_vs_fp64_apply"] = out["jvp_mixed"]["GDOF/s"] / out["jvp_fp64"]["GDOF/s"]
    return out


def _newton_row(pb, torch, **opts):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    u, rep = pb.newton_solve(rtol=1e-10, **opts)
    torch.cuda.synchronize()
    return u, {"ms": (time.perf_counter() - t0) * 1e3, "newton_iters": rep["newton_iters"],
               "cg_iters": rep["cg_iters_total"], "res_final_rel": rep["res_final"] / rep["ref_norm"],
               "status": rep["status"]}


def _adjoint_row(pb, torch, u, b, **opts):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g, lam, rep = pb.adjoint_gradient(u, b, rtol=1e-10, **opts)
    torch.cuda.synchronize()
    row = {"ms": (time.perf_counter() - t0) * 1e3, "cg_iters": rep["cg_iters_total"],
           "refine_iters": rep["refine_iters"], "res_final_rel": rep["res_final"] / rep["ref_norm"],
           "status": rep["status"]}
    # the same solve again with every launch timed by events: GPU kernel time
    pb.profile(True)
    pb.adjoint_gradient(u, b, rtol=1e-10, **opts)
    row["kernel_sum_ms"] = sum(ms for _, ms in pb.profile_read().values())
    pb.profile(False)
    return g, row


def solve_rows(feod, WORKLOADS, make_inputs, dev, names=("c3", "c4", "c2", "c5")):
    """Newton-CG and adjoint-gradient wall times (synchronised).  Every solve
    stops at the same FP64 relative residual 1e-10 (the residual is FP64 in
    both precisions), so FP64 and mixed are compared at equal final accuracy.
    64^3 Q4: FP64 vs mixed (the solver defaults: fused Jacobian action, Jacobi).
    16^3 Q7 curved: also with partial assembly.
    48^3 Q2 and 32^3 Q3: also with partial assembly and without Jacobi.
    48^3 Q2 and 16^3 Q7 curved: the adjoint design gradient (compliance) in
    FP64 and mixed, fused and with partial assembly, and the gradient kernel
    alone in FP64 and FP32."""
    import torch
    out = {}
    for name in names:
        w = WORKLOADS[name]
        ii = make_inputs(w)
        pb = feod.Problem(w.nx, w.ny, w.nz, w.k, w.nq, w.p, w.eps, vertices=ii["vertices"], rho=ii["rho"],
                          device=dev)
        b = torch.as_tensor(feod.HostSetup(w.nx, w.ny, w.nz, w.k, w.nq, vertices=ii["vertices"]).load,
                            device=dev)
        combos = {"c3": [(0, 1)], "c5": [(0, 1), (1, 1)]}.get(name, [(pa, jac) for pa in (0, 1) for jac in (0, 1)])
        u_ref = None
        t_ref = {}
        for prec in ("fp64", "mixed"):
            for pa, jac in combos:
                u, row = _newton_row(pb, torch, prec=prec, partial_assembly=pa, jacobi=jac)
                if u_ref is None:
                    u_ref = u.clone()
                else:
                    row["u_rel_diff_vs_fp64"] = float(torch.linalg.norm(u - u_ref) / torch.linalg.norm(u_ref))
                if prec == "fp64":
                    t_ref[(pa, jac)] = row["ms"]
                else:
                    row["speedup_vs_fp64_at_equal_residual"] = t_ref[(pa, jac)] / row["ms"]
                out[f"{name}_newton_{prec}_pa{pa}_jacobi{jac}"] = row
        if name in ("c4", "c5"):
            g_ref = None
            for prec in ("fp64", "mixed"):
                for pa in (0, 1):
                    g, row = _adjoint_row(pb, torch, u_ref, b, prec=prec, partial_assembly=pa)
                    if g_ref is None:
                        g_ref = g.clone()
                    else:
                        row["grad_rel_diff_vs_fp64"] = float(torch.linalg.norm(g - g_ref) / torch.linalg.norm(g_ref))
                    out[f"{name}_adjoint_gradient_{prec}_pa{pa}"] = row
            # the gradient kernel alone at (u, lambda = u): FP64 vs FP32
            g64 = pb.grad_rho(u_ref, u_ref)
            krow = {}
            for prec in ("fp64", "mixed"):
                ms = timed_loop(lambda: pb.grad_rho(u_ref, u_ref, prec=prec), 50, 5)
                gk = pb.grad_rho(u_ref, u_ref, prec=prec)
                krow[prec] = {"us": ms * 1e3,
                              "rel_err_vs_fp64": float(torch.linalg.norm(gk - g64) / torch.linalg.norm(g64))}
            out[f"{name}_grad_kernel"] = krow
        del pb, b, u_ref
        torch.cuda.empty_cache()
    for k, v in out.items():
        log(f"[bench] solve {k}: {v}")
    return out


def tangent_flops_per_element(k, nq):
    """Algorithmic FLOPs of one element tangent matrix (Eq. 3) as the kernel
    computes it.  Sum-factorised kernel: dense reference gradients (12 nq^3 (k+1)^3), the pointwise
    tangent by three dual evaluations plus transform (~150 per point), and the
    sum-factorised B^T Chat B, 3 FLOP per term of each stage (two factors and
    the accumulate): x and y stages for the 9 tensor terms, 27 (nq^3 D1^2 +
    nq^2 D1^4), and the z stage once per z-factor pair, 12 nq D1^6."""
    d1 = k + 1
    if d1 == 3:
        # matrix-core path: K = G^T W with G the 3 nq^3 x 27 table of
        # reference derivatives and W = Chat G (3 FMA per entry); the
        # symmetric product is computed on 3 of the 4 16x16 tiles (553 of the
        # 729 entries, the rest written by symmetry); plus the gradient of u
        # at the points and Chat
        kd, ne = 3 * nq ** 3, 27
        return 2 * kd * ne + 150 * nq ** 3 + 6 * kd * ne + 2 * kd * (16 * 16 + 16 * 11 + 11 * 11)
    return (12 * nq ** 3 * d1 ** 3 + 150 * nq ** 3
            + 27 * (nq ** 3 * d1 ** 2 + nq ** 2 * d1 ** 4) + 12 * nq * d1 ** 6)


def tangent_rows(feod, WORKLOADS, make_inputs, dev, args):
    """Element tangent matrices K_e = B^T J_D B (Eq. 3) for every element."""
    import torch
    out = {}
    for name in ("c4", "c2"):
        w = WORKLOADS[name]
        ii = make_inputs(w)
        pb = feod.Problem(w.nx, w.ny, w.nz, w.k, w.nq, w.p, w.eps, vertices=ii["vertices"], rho=ii["rho"],
                          device=dev)
        u = torch.as_tensor(ii["u"], device=dev)
        ne = (w.k + 1) ** 3
        Ke = torch.empty((w.n_elems, ne, ne), dtype=torch.float64, device=dev)
        ms = timed_loop(lambda: pb.element_tangents(u, out=Ke), max(3, args.steps // 10), 2)
        flops = tangent_flops_per_element(w.k, w.nq) * w.n_elems
        bytes_ = Ke.numel() * 8 + 8 * w.n_dofs
        out[name] = {"path": "mfma" if w.k == 2 else "vector", "ms_per_launch": ms,
                     "ns_per_element": ms * 1e6 / w.n_elems,
                     "TFLOP/s": flops / (ms * 1e-3) / 1e12, "frac_fp64_peak": flops / (ms * 1e-3) / 1e12 / FP64_PEAK_TFS,
                     "GB/s": bytes_ / (ms * 1e-3) / 1e9, "matrix_entries": Ke.numel()}
        # the paper's ELM variant (Table 1): forward AD through the element
        # residual, one Jacobian action per local DOF; FLOPs from the cost model
        ms_elm = timed_loop(lambda: pb.element_tangents(u, out=Ke, method="elm"), max(3, args.steps // 10), 2)
        f_elm = pb.kernel_cost("elm")[1]
        out[name]["elm"] = {"ms_per_launch": ms_elm, "ns_per_element": ms_elm * 1e6 / w.n_elems,
                            "TFLOP/s": f_elm / (ms_elm * 1e-3) / 1e12,
                            "frac_fp64_peak": f_elm / (ms_elm * 1e-3) / 1e12 / FP64_PEAK_TFS,
                            "time_vs_quadrature_point_ad": ms_elm / ms}
        log(f"[bench] element tangents {name}: {out[name]}")
        del pb, u, Ke
        torch.cuda.empty_cache()
    return out


def partial_assembly_rows(feod, WORKLOADS, make_inputs, dev, args):
    """Fused Jacobian apply vs the partial-assembly one (stored gradients of u)."""
    import torch
    out = {}
    for name in ("c2", "c4", "c5"):
        w = WORKLOADS[name]
        ii = make_inputs(w)
        pb = feod.Problem(w.nx, w.ny, w.nz, w.k, w.nq, w.p, w.eps, vertices=ii["vertices"], rho=ii["rho"],
                          device=dev)
        u = torch.as_tensor(ii["u"], device=dev)
        v = torch.as_tensor(ii["v"], device=dev)
        jv = torch.empty_like(u)
        row = {}
        for prec in ("fp64", "mixed"):
            t_fused = timed_loop(lambda: pb.jacobian_apply(u, v, out=jv, prec=prec), args.steps, args.warmup)
            t_setup = timed_loop(lambda: pb.pa_setup(u, prec=prec), 5, 1)
            t_pa = timed_loop(lambda: pb.jacobian_apply_pa(v, out=jv, prec=prec), args.steps, args.warmup)
            row[prec] = {"fused_us": t_fused * 1e3, "pa_us": t_pa * 1e3, "pa_setup_us": t_setup * 1e3,
                         "pa_speedup": t_fused / t_pa,
                         "stored_MB": 3 * w.nq ** 3 * w.n_elems * (8 if prec == "fp64" else 4) / 1e6}
        out[name] = row
        log(f"[bench] partial assembly {name}: {row}")
        del pb, u, v, jv
        torch.cuda.empty_cache()
    return out


def mall_cold_rows(feod, WORKLOADS, make_inputs, dev, reps=21):
    """Single FP64 Jacobian applies with the 256 MB Infinity Cache flushed
    before each (a 1 GiB buffer is written between applies, outside the timed
    window), against the warm back-to-back rate and a measured device-copy
    bandwidth.  Bytes are the apply's algorithmic bytes: element kernel (unique
    L-vector reads, E-vector write) plus G^T (E-vector read, L-vector write)."""
    import torch
    flush = torch.empty(128 * 1024 * 1024, dtype=torch.float64, device=dev)
    src = torch.ones(64 * 1024 * 1024, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    copy_ms = timed_loop(lambda: dst.copy_(src), 10, 2)
    copy_gbs = 2 * src.numel() * 8 / (copy_ms * 1e-3) / 1e9
    del src, dst
    s = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    out = {"copy_GBs": copy_gbs}
    for name in ("c2", "c4", "c5"):
        w = WORKLOADS[name]
        ii = make_inputs(w)
        pb = feod.Problem(w.nx, w.ny, w.nz, w.k, w.nq, w.p, w.eps, vertices=ii["vertices"], rho=ii["rho"],
                          device=dev)
        u = torch.as_tensor(ii["u"], device=dev)
        v = torch.as_tensor(ii["v"], device=dev)
        jv = torch.empty_like(u)
        warm = timed_loop(lambda: pb.jacobian_apply(u, v, out=jv), 50, 5)
        times = []
        for i in range(reps + 2):
            flush.fill_(float(i))
            s.record()
            pb.jacobian_apply(u, v, out=jv)
            e.record()
            torch.cuda.synchronize()
            if i >= 2:
                times.append(s.elapsed_time(e))
        cold = sorted(times)[len(times) // 2]
        kbytes, _ = pb.kernel_cost("jvp", "fp64")
        nbytes = kbytes + 8 * w.n_elems * (w.k + 1) ** 3 + 8 * w.n_dofs
        # the design's own byte count (u, v, G map, E-vector written and read,
        # G^T map, L-vector written, curved vertices): 28 N + 24 E (k+1)^3 [+ 192 E]
        sbytes = 28 * w.n_dofs + 24 * w.n_elems * (w.k + 1) ** 3 + (192 * w.n_elems if w.perturb else 0)
        out[name] = {"cold_us": cold * 1e3, "warm_us": warm * 1e3, "GDOF/s_cold": w.n_dofs / (cold * 1e-3) / 1e9,
                     "apply_bytes": nbytes, "hbm_frac_cold": nbytes / (cold * 1e-3) / (HBM_PEAK_GBS * 1e9),
                     "copy_frac_cold": nbytes / (cold * 1e-3) / (copy_gbs * 1e9),
                     "design_bytes": sbytes,
                     "hbm_frac_cold_design_bytes": sbytes / (cold * 1e-3) / (HBM_PEAK_GBS * 1e9)}
        log(f"[bench] MALL-cold {name}: {out[name]}")
        del pb, u, v, jv
        torch.cuda.empty_cache()
    log(f"[bench] device copy {copy_gbs:.0f} GB/s")
    del flush
    torch.cuda.empty_cache()
    return out


def mixed_error_rows(feod, WORKLOADS, make_inputs, dev):
    """Relative L2 difference of the mixed-precision Jacobian apply from the
    FP64 one, at the seeded random u and at a smooth u (the Newton solution)."""
    import torch
    out = {}
    for name in ("c2", "c4", "c5"):
        w = WORKLOADS[name]
        ii = make_inputs(w)
        pb = feod.Problem(w.nx, w.ny, w.nz, w.k, w.nq, w.p, w.eps, vertices=ii["vertices"], rho=ii["rho"],
                          device=dev)
        u = torch.as_tensor(ii["u"], device=dev)
        v = torch.as_tensor(ii["v"], device=dev)
        row = {}
        for tag, uu in (("random_u", u), ("newton_u", pb.newton_solve(rtol=1e-10)[0])):
            j64 = pb.jacobian_apply(uu, v)
            j32 = pb.jacobian_apply(uu, v, prec="mixed")
            row[tag] = float(torch.linalg.norm(j32 - j64) / torch.linalg.norm(j64))
        out[name] = row
        log(f"[bench] mixed-vs-FP64 Jacobian apply error {name}: {row}")
        del pb, u, v
        torch.cuda.empty_cache()
    return out


def cpu_baseline(w, inp, budget_s=12.0, chunk=2048):
    """The oracle's Jacobian apply on the same workload, timed on host cores
    over a bounded sample: whole chunks of consecutive elements, as many as
    the time budget allows (at least one), scaled to GDOF/s of a full apply
    (N DOFs per E elements)."""
    import threadpoolctl
    from oracle import Discretisation
    d = Discretisation(w.nx, w.ny, w.nz, w.k, w.nq, w.p, w.eps, vertices=inp["vertices"],
                       rho=inp["rho"], compute_load=False, chunk=chunk)
    threads = max([x.get("num_threads", 1) for x in threadpoolctl.threadpool_info()] + [1])
    n_el, t0 = 0, time.perf_counter()
    while n_el < w.n_elems:
        elems = (n_el + np.arange(min(chunk, w.n_elems - n_el)))
        d.jvp(inp["u"], inp["v"], elems)
        n_el += elems.size
        el = time.perf_counter() - t0
        if el >= budget_s:
            break
    full_s = el * w.n_elems / n_el
    return {"value": w.n_dofs / full_s / 1e9, "unit": "GDOF/s", "cores": threads, "kind": "oracle",
            "sample": f"oracle Jacobian apply over {n_el} of the {w.n_elems} elements of the {w.name} "
                      f"workload in {el:.1f} s (dense-element NumPy/OpenBLAS, {os.cpu_count()} host CPUs "
                      f"visible), scaled to a full apply of {w.n_dofs} DOFs ({full_s:.1f} s)"}


def cpu_table(WORKLOADS, make_inputs):
    """The oracle's residual and Jacobian apply on every workload, full
    applies, median of 3 (one run on the 64^3 Q4 workload, about a minute per
    apply), and its Newton solve on the 4^3 Q2 workload."""
    import threadpoolctl
    from oracle import Discretisation, newton
    threads = max([x.get("num_threads", 1) for x in threadpoolctl.threadpool_info()] + [1])
    out = {"cores": threads}
    for name in ("c1", "c2", "c3", "c4", "c5"):
        w = WORKLOADS[name]
        inp = make_inputs(w)
        d = Discretisation(w.nx, w.ny, w.nz, w.k, w.nq, w.p, w.eps, vertices=inp["vertices"],
                           rho=inp["rho"], compute_load=(name == "c1"))
        if d.b is None:
            d.b = np.zeros(d.N)  # the load is a subtraction; its cost is not the apply's
        row = {}
        for op, fn in (("residual", lambda: d.residual(inp["u"])), ("jvp", lambda: d.jvp(inp["u"], inp["v"]))):
            ts = []
            for _ in range(1 if name == "c3" else 3):
                t0 = time.perf_counter()
                fn()
                ts.append(time.perf_counter() - t0)
            med = sorted(ts)[len(ts) // 2]
            row[op] = {"s": med, "GDOF/s": w.n_dofs / med / 1e9, "runs": len(ts)}
        if name == "c1":
            t0 = time.perf_counter()
            newton(d, tol=1e-10)
            row["newton_s"] = time.perf_counter() - t0
        out[name] = row
        log(f"[bench] oracle {name}: {row}")
        del d
    return out


def summary(rows):
    """The headline figures of every row, in one short object (the JSON line
    leads with it, ahead of the full rows)."""
    out = {"jvp_GDOF/s": {}, "element_kernel_frac": {}, "newton_ms": {}, "adjoint_gradient_ms": {}}
    for w in ("c3", "c2", "c4", "c5"):
        r = rows.get(w, {})
        for prec in ("fp64", "mixed"):
            x = r.get(f"jvp_{prec}")
            if x:
                out["jvp_GDOF/s"][f"{w}_{prec}"] = round(x["GDOF/s"], 3)
                out["element_kernel_frac"][f"{w}_{prec}"] = round(x["kernel_frac"], 4)
                if prec == "mixed" and x.get("kernel_frac_vs_published_fp32") is not None:
                    out["element_kernel_frac"][f"{w}_mixed_vs_published_fp32"] = round(
                        x["kernel_frac_vs_published_fp32"], 4)
        if r.get("jvp_mixed") and r.get("jvp_fp64"):
            out["jvp_GDOF/s"][f"{w}_mixed_speedup"] = round(r["jvp_mixed"]["GDOF/s"] / r["jvp_fp64"]["GDOF/s"], 3)
    sol = rows.get("solves", {})
    for w in ("c3", "c2", "c4", "c5"):
        a, b = sol.get(f"{w}_newton_fp64_pa0_jacobi1"), sol.get(f"{w}_newton_mixed_pa0_jacobi1")
        if a and b:
            out["newton_ms"][w] = {"fp64": round(a["ms"], 2), "mixed": round(b["ms"], 2),
                                   "mixed_speedup_at_equal_residual": round(a["ms"] / b["ms"], 3),
                                   "res_final_rel": [a["res_final_rel"], b["res_final_rel"]]}
        a, b = sol.get(f"{w}_adjoint_gradient_fp64_pa0"), sol.get(f"{w}_adjoint_gradient_mixed_pa0")
        if a and b:
            out["adjoint_gradient_ms"][w] = {"fp64": round(a["ms"], 2), "mixed": round(b["ms"], 2),
                                             "mixed_grad_rel_diff": b.get("grad_rel_diff_vs_fp64")}
    mc = rows.get("mall_cold", {})
    if "c4" in mc:
        out["c4_cold_apply"] = {"us": round(mc["c4"]["cold_us"], 2), "hbm_frac": round(mc["c4"]["hbm_frac_cold"], 4),
                                "hbm_frac_design_bytes": round(mc["c4"]["hbm_frac_cold_design_bytes"], 4),
                                "copy_GBs": round(mc["copy_GBs"], 1)}
    if "mixed_error" in rows:
        out["mixed_vs_fp64_jvp_rel_error"] = rows["mixed_error"]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--prec", default="fp64", choices=["fp64", "mixed"],
                    help="precision of the timed Jacobian apply (the headline is FP64; mixed is for profiling runs)")
    ap.add_argument("--settle", type=float, default=0.5,
                    help="seconds of untimed applies before the warm-up steps (GPU clocks reach steady state)")
    ap.add_argument("--repeats", type=int, default=5,
                    help="further windows of K timed steps; their median is reported beside value")
    ap.add_argument("--cpu-table", action="store_true",
                    help="also time the oracle's full residual and Jacobian applies on every workload "
                         "(median of 3; minutes of CPU time)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one 256 MiB device-to-device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
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
    N = w.n_dofs

    if args.calibrate_copy:
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    prec = args.prec
    kname = "element_jvp_f64" if prec == "fp64" else "element_jvp_f32"

    def jvp64():
        prob.jacobian_apply(u, v, out=jv, prec=prec)

    log(f"[bench] {w.name}: N={N} E={w.n_elems} timed JVP {prec} x{args.steps}")
    settle(jvp64, args.settle)
    ms = timed_loop(jvp64, args.steps, args.warmup)
    value = N / (ms * 1e-3) / 1e9
    stats = kernel_profile(prob, jvp64, min(args.steps, 50))
    k_ms = element_kernel_ms(prob, u, v, "jvp", prec, args.steps, args.warmup)
    roof = roofline(prob, "jvp", prec, stats, kname, kernel_ms=k_ms)
    roof["traffic"] = stored_traffic(w.name, kname)
    reps = sorted(timed_loop(jvp64, args.steps, 0) for _ in range(args.repeats))
    rep_med = reps[len(reps) // 2] if reps else ms
    log(f"[bench] JVP {prec} {ms * 1e3:.1f} us/apply = {value:.2f} GDOF/s (median of {len(reps)} more windows "
        f"{rep_med * 1e3:.1f} us); element kernel {k_ms * 1e3:.2f} us back-to-back; per-launch events {stats}")

    rows = {w.name: {f"jvp_{prec}": {"GDOF/s": value, "us_per_apply": ms * 1e3, "kernel_us": roof["avg_us"],
                                  "kernel_bound": roof["bound"], "kernel_frac": roof["frac"],
                                  "repeat_windows_us": [t * 1e3 for t in reps],
                                  "repeat_median_GDOF/s": N / (rep_med * 1e-3) / 1e9,
                                  "gather_t_us": stats.get("gather_transpose", {"avg_ms": 0.0})["avg_ms"] * 1e3}}}
    if not args.no_extras and prec == "fp64":
        rows[w.name].update(apply_rows(prob, u, v, w, args,
                                       only=("jvp_mixed", "residual_fp64", "residual_jvp_fp64")))
        rows[w.name]["jvp_mixed"]["speedup_vs_fp64_apply"] = rows[w.name]["jvp_mixed"]["GDOF/s"] / value
        rows[w.name]["ad_overhead"] = ad_overhead(prob, u, v, args)
        log(f"[bench] {w.name} rows: {rows[w.name]}")
        del prob, u, v, jv
        torch.cuda.empty_cache()
        for name in [x for x in ("c2", "c3", "c4", "c5") if x != w.name]:
            wl = WORKLOADS[name]
            ii = make_inputs(wl)
            pb = feod.Problem(wl.nx, wl.ny, wl.nz, wl.k, wl.nq, wl.p, wl.eps, vertices=ii["vertices"],
                              rho=ii["rho"], device=dev)
            uu = torch.as_tensor(ii["u"], device=dev)
            vv = torch.as_tensor(ii["v"], device=dev)
            rows[name] = apply_rows(pb, uu, vv, wl, args, only=("jvp_fp64", "jvp_mixed", "residual_fp64"))
            log(f"[bench] {name}: { {k: (x['GDOF/s'], x['kernel_us'], x['kernel_frac']) for k, x in rows[name].items()} }")
            rows[name]["ad_overhead"] = ad_overhead(pb, uu, vv, args)
            log(f"[bench] {name} AD vs hand-coded J_D: {rows[name]['ad_overhead']}")
            del pb, uu, vv
            torch.cuda.empty_cache()
        rows["solves"] = solve_rows(feod, WORKLOADS, make_inputs, dev)
        rows["element_tangents"] = tangent_rows(feod, WORKLOADS, make_inputs, dev, args)
        rows["partial_assembly"] = partial_assembly_rows(feod, WORKLOADS, make_inputs, dev, args)
        rows["mall_cold"] = mall_cold_rows(feod, WORKLOADS, make_inputs, dev)
        rows["mixed_error"] = mixed_error_rows(feod, WORKLOADS, make_inputs, dev)

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline ...")
        cpu = cpu_baseline(w, inp)
        log(f"[bench] cpu_baseline {cpu}")
    if args.cpu_table:
        rows["oracle_table"] = cpu_table(WORKLOADS, make_inputs)

    out = {"metric": METRIC, "value": value, "unit": "GDOF/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64" if prec == "fp64" else "f32 element stage, f64 G^T",
           "data": "synthetic",
           "config": {"workload": f"{w.name}: {w.note}", "n_dofs": N, "n_elems": w.n_elems,
                      "order_k": w.k, "nq": w.nq, "p": w.p, "eps": w.eps, "seed": w.seed,
                      "parallelism": "single GPU", "settle_s": args.settle},
           "roofline": {k: roof[k] for k in ("bound", "achieved", "peak", "unit", "frac", "traffic")},
           "roofline_detail": roof, "cpu_baseline": cpu, "summary": summary(rows), "rows": rows}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
