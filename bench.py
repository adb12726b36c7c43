#!/usr/bin/env python3
"""Throughput of the DG Maxwell hot path on one MI355X.

Workload (default, the largest single-GPU configuration): the 48^3 x 6
jittered Kuhn cube (K = 663,552 tetrahedra), order N = 5 (Np = 56), FP32
state, perfectly conducting walls, upwind flux, fields = the (1,1,0) cavity
mode plus seeded N(0, 1e-3) noise.  One "step" is one LSERK time step: five
right-hand-side evaluations, each fused with its stage update, over the whole
mesh; the K timed steps are one dg_rk_step call.

Metric: GDOF/s per RHS evaluation = 5 * 6 * K * Np * steps / time / 1e9,
inputs resident in HBM, timed with HIP events on the stream the library
launches on.  The "roofline" object describes the dominant kernel, the fused
stage (right-hand side + update), from its algorithmic flop and byte counts
and its average launch time over the timed region (time / (5 steps));
"rhs_only" gives the same for the plain right-hand side.  The same line
carries the split 16-bit precisions on that mesh, the 24^3 x 6, N = 4 mesh in
FP64 and FP32, and the 64-problem batch (graph replay vs one launch per
problem).  "cpu_baseline" times the FP64 CPU oracle on a bounded sample of
the same recipe.
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

import dg_inputs as I  # noqa: E402

PEAKS = {  # MI355X published peaks (dense)
    "hbm_GBs": 8000.0,
    "fp64_TFs": 78.6,
    "fp32_TFs": 157.3,
    "bf16_TFs": 2500.0,   # BF16 and FP16 matrix cores
}


def flops_per_element(N: int, stage: bool = False) -> int:
    """Algorithmic flops of one RHS per element: 18 Np x Np matvecs (Dr, Ds,
    Dt of six fields), 6 Np x 4Nfp matvecs (LIFT), the upwind flux (~60 per
    face node) and metric + curl (~66 per node).  A fused LSERK stage adds the
    update res = a res + dt rhs, u' = u + b res: 5 flops per value."""
    Np = (N + 1) * (N + 2) * (N + 3) // 6
    Nfp = (N + 1) * (N + 2) // 2
    return 36 * Np * Np + 48 * Np * Nfp + 240 * Nfp + 66 * Np + (30 * Np if stage else 0)


def contraction_flops_per_element(N: int) -> int:
    """Flops of the two dense contractions alone (volume and LIFT)."""
    Np = (N + 1) * (N + 2) * (N + 3) // 6
    Nfp = (N + 1) * (N + 2) // 2
    return 36 * Np * Np + 48 * Np * Nfp


def bytes_per_element(N: int, s: int, stage: bool = False) -> int:
    """Algorithmic HBM bytes of one RHS per element: read u, write rhs
    (6 Np scalars each), 25 geometry scalars, 16 bytes of connectivity.  A
    fused LSERK stage reads u and res and writes res and the new state: four
    state arrays instead of two."""
    Np = (N + 1) * (N + 2) * (N + 3) // 6
    return (4 if stage else 2) * 6 * Np * s + 25 * s + 16


def make_problem(dg, k, N, precision):
    VX, EToV = I.kuhn_cube(k, 0.1, 0)
    p = dg.Problem(N, VX, EToV, precision)
    xyz = p.nodes()
    u = I.cavity_mode(xyz[..., 0], xyz[..., 1], xyz[..., 2]) + I.field_noise((6, p.info.K, p.info.Np), 1e-3, 1)
    return p, u, (VX, EToV)


def time_rhs(torch, p, du, out, reps):
    stream = torch.cuda.current_stream()
    for _ in range(3):
        p.rhs(du, out, stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        p.rhs(du, out, stream)
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / 1e3 / reps


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_rate(k, N, budget_s, max_evals):
    """(GDOF/s, evaluations, mean seconds, K) of FP64 oracle RHS evaluations on
    the jittered k^3 x 6 cube at order N with the benchmark's fields."""
    from oracle import maxwell as Mx
    from oracle import mesh as Me
    VX, EToV = I.kuhn_cube(k, 0.1, 0)
    m = Me.Mesh(N, VX, EToV)
    u = I.cavity_mode(m.x, m.y, m.z) + I.field_noise((6, m.K, m.Np), 1e-3, 1)
    t0 = time.perf_counter()
    n = 0
    while True:
        Mx.rhs(m, u)
        n += 1
        if time.perf_counter() - t0 > budget_s or n >= max_evals:
            break
    t = (time.perf_counter() - t0) / n
    return 6 * m.K * m.Np / t / 1e9, n, t, m.K


def cpu_baseline(k, N, k_single):
    """The FP64 CPU oracle on a bounded sample of the benchmark's recipe (the
    per-DOF work of one RHS does not depend on K): all BLAS threads on the
    k^3 x 6 mesh, and one thread on the smaller k_single mesh."""
    from threadpoolctl import threadpool_info, threadpool_limits
    threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    v, n, t, K = _oracle_rate(k, N, 12.0, 4)
    with threadpool_limits(1):
        v1, n1, t1, K1 = _oracle_rate(k_single, N, 4.0, 3)
    return {"value": v, "unit": "GDOF/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} FP64 oracle RHS evaluations on the {k}^3x6 cube (K={K}, N={N}, the same mesh recipe "
                      f"and fields at 1/{(48 // k) ** 3 if 48 % k == 0 else 'n'} of the elements; mean {t:.2f} s "
                      f"each) with {threads} BLAS threads; the oracle's elementwise NumPy work is single-threaded",
            "single_thread": {"value": v1, "unit": "GDOF/s", "cores": 1,
                              "sample": f"{n1} evaluations on the {k_single}^3x6 cube (K={K1}), mean {t1:.2f} s"},
            "host": {"cpu_model": _cpu_model(), "logical_cpus": os.cpu_count()}}


def roofline(prec, N, K, t_rhs, s, stage=False):
    """(bound, achieved, peak, unit) of one RHS (or fused LSERK stage) of K
    elements taking t_rhs s.  FP64/FP32 are priced against the matrix-core
    peak of their dtype; the split precisions against whichever of HBM bytes
    and 16-bit matrix-core work takes longer."""
    flops = flops_per_element(N, stage) * K
    if prec in ("fp64", "fp32"):
        peak = PEAKS["fp64_TFs"] if prec == "fp64" else PEAKS["fp32_TFs"]
        return "mfma", flops / t_rhs / 1e12, peak, "TFLOP/s"
    nprod = int(prec[-1]) if prec[-1].isdigit() else 1
    nbytes = bytes_per_element(N, s, stage) * K
    t_hbm = nbytes / (PEAKS["hbm_GBs"] * 1e9)
    t_mma = nprod * contraction_flops_per_element(N) * K / (PEAKS["bf16_TFs"] * 1e12)
    if t_hbm >= t_mma:
        return "hbm", nbytes / t_rhs / 1e9, PEAKS["hbm_GBs"], "GB/s"
    return "mfma", nprod * contraction_flops_per_element(N) * K / t_rhs / 1e12, PEAKS["bf16_TFs"], "TFLOP/s"


def bench_sweep(args, torch, dg):
    """Order sweep: for each N the cube mesh with about 1e7 nodal values per
    field (k = round((1e7 / (6 Np))^(1/3))), one RHS timed per precision and
    kernel variant; split precisions report their error against the FP64
    path on the same fields."""
    rows = []
    for N in [int(x) for x in args.sweep_orders.split(",")]:
        k = I.k_for_dofs(N)
        VX, EToV = I.kuhn_cube(k, 0.1, 0)
        ref = None
        for prec in args.sweep_precisions.split(","):
            try:
                p = dg.Problem(N, VX, EToV, prec)
            except dg.DgError as e:
                if e.status == dg.DG_EUNSUPPORTED:
                    continue
                raise
            xyz = p.nodes()
            u = I.cavity_mode(xyz[..., 0], xyz[..., 1], xyz[..., 2]) + I.field_noise((6, p.info.K, p.info.Np), 1e-3, 1)
            du = p.pack(u)
            out = p.zeros_state()
            for v in range(dg.dg_variant_count()):
                try:
                    p.set_variant(v)
                except dg.DgError:
                    continue
                t = dg.dg_time_rhs(p.handle, du, out, 3, args.rhs_reps) / 1e3
                bound, ach, peak, unit = roofline(prec, N, p.info.K, t, p.info.elem_bytes)
                row = {"N": N, "K": p.info.K, "precision": prec, "variant": p.variant, "rhs_us": 1e6 * t,
                       "gdofs": 6 * p.info.K * p.info.Np / t / 1e9, "bound": bound, "achieved": ach,
                       "unit": unit, "frac": ach / peak}
                if prec == "fp64" and ref is None:
                    p.rhs(du, out)
                    torch.cuda.synchronize()
                    ref = p.unpack(out)
                if prec != "fp64" and ref is not None:
                    p.rhs(du, out)
                    torch.cuda.synchronize()
                    row["rel_err_vs_fp64"] = float(np.abs(p.unpack(out) - ref).max() / np.abs(ref).max())
                rows.append(row)
                print(json.dumps(row), file=sys.stderr, flush=True)
            p.close()
            del du, out
    best = {}
    for r in rows:
        key = (r["N"], r["precision"])
        if key not in best or r["rhs_us"] < best[key]["rhs_us"]:
            best[key] = r
    line = {"metric": "GDOF/s per DG RHS eval (Maxwell tets) and % of HBM/MFMA roofline",
            "workload": "order sweep, about 1e7 nodal values per field per order", "rows": rows,
            "best": [best[k] for k in sorted(best)]}
    print(json.dumps(line), flush=True)


def batch_modes(torch, dg, steps, warmup):
    """64 independent cavity problems (k ~ U{4..20}, N ~ U{2..7}, FP32) stepped
    together: graph-replayed grouped launches, the same launches issued
    directly, and one launch per problem and stage."""
    draws = I.batch_draws()
    meshes, dofs = [], 0
    for k, N, seed in draws:
        VX, EToV = I.kuhn_cube(k, 0.1, seed)
        meshes.append((N, VX, EToV))
        dofs += 6 * EToV.shape[0] * (N + 1) * (N + 2) * (N + 3) // 6
    b = dg.Batch(meshes, "fp32")
    us, ress, dts = [], [], []
    for (k, N, seed), p in zip(draws, b.problems):
        xyz = p.nodes()
        u = I.cavity_mode(xyz[..., 0], xyz[..., 1], xyz[..., 2]) + I.field_noise((6, p.info.K, p.info.Np), 1e-3, seed)
        us.append(p.pack(u))
        ress.append(p.zeros_state())
        dts.append(0.5 * p.info.dt_cfl1)
    stream = torch.cuda.current_stream()
    out = {}
    for mode in ("graph", "grouped", "per_problem"):
        b.rk_step(us, ress, dts, warmup, mode, stream)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        b.rk_step(us, ress, dts, steps, mode, stream)
        e1.record(stream)
        e1.synchronize()
        wall = time.perf_counter() - t0
        t = e0.elapsed_time(e1) / 1e3
        out[mode] = {"ms_per_step": 1e3 * t / steps, "gdofs": 5 * dofs * steps / t / 1e9,
                     "host_ms_per_step": 1e3 * wall / steps}
    b.close()
    return {"workload": "64 independent PEC-cavity problems, k ~ U{4..20} (K = 6k^3), N ~ U{2..7}, FP32, "
                        "one LSERK step of all of them per step",
            "problems": len(draws), "dofs": dofs, "orders": sorted({n for _, n, _ in draws}), "modes": out,
            "speedup_graph_vs_per_problem": out["per_problem"]["ms_per_step"] / out["graph"]["ms_per_step"]}


def bench_batch(args, torch, dg):
    r = batch_modes(torch, dg, args.steps, args.warmup)
    line = {
        "metric": "GDOF/s per DG RHS eval (Maxwell tets) and % of HBM/MFMA roofline",
        "value": r["modes"]["graph"]["gdofs"], "unit": "GDOF/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": r["modes"]["graph"]["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": r["workload"], "problems": r["problems"], "dofs": r["dofs"], "orders": r["orders"]},
        "modes": r["modes"], "speedup_graph_vs_per_problem": r["speedup_graph_vs_per_problem"],
    }
    print(json.dumps(line), flush=True)


def systems_rhs(torch, k, N, prec, reps):
    """Run-time compiled systems (acoustics, Euler) on the k^3 x 6 cube: one
    right-hand side timed by dg_time_rhs, priced against the binding roofline
    from the contraction flops 2 M Np (3 Np + 4 Nfp) and the bytes of one state
    read, one written, geometry and connectivity per element."""
    from paper_1211_0582_amd import dg
    from paper_1211_0582_amd import systems as S
    out = {}
    VX, EToV = I.kuhn_cube(k, 0.1, 0)
    for spec in (S.acoustics(), S.euler()):
        t0 = time.perf_counter()
        p = S.SystemProblem(spec, N, VX, EToV, prec)
        setup_s = time.perf_counter() - t0
        K, Np, Nfp, M, sz = p.info.K, p.info.Np, p.info.Nfp, spec.M, p.info.elem_bytes
        xyz = p.nodes()
        u = np.ones((M, K, Np)) + I.field_noise((M, K, Np), 1e-2, 1)
        if spec.name == "euler":
            u[1:4] *= 0.1
            u[4] = 2.5 + 0.1 * np.cos(xyz[..., 0])
        du = p.pack(u)
        o = p.zeros_state()
        t = dg.dg_time_rhs(p.handle, du, o, 3, reps) / 1e3
        flops = 2 * M * Np * (3 * Np + 4 * Nfp) * K
        nbytes = (2 * M * Np * sz + 25 * sz + 16) * K
        peak_f = (PEAKS["fp64_TFs"] if prec == "fp64" else PEAKS["fp32_TFs"]) * 1e12
        if flops / peak_f >= nbytes / (PEAKS["hbm_GBs"] * 1e9):
            bound, ach, peak, unit = "mfma", flops / t / 1e12, peak_f / 1e12, "TFLOP/s"
        else:
            bound, ach, peak, unit = "hbm", nbytes / t / 1e9, PEAKS["hbm_GBs"], "GB/s"
        out[spec.name] = {"K": K, "N": N, "fields": M, "rhs_us": 1e6 * t, "gdofs": M * K * Np / t / 1e9,
                          "bound": bound, "achieved": ach, "peak": peak, "unit": unit, "frac": ach / peak,
                          "setup_and_compile_s": setup_s}
        p.close()
        del du, o
    return out


MIX = {"fp64": 0, "fp32": 0, "bf16": 1, "bf16x2": 2, "bf16x3": 3, "f16": 4, "f16x2": 5, "f16x3": 6}


def measure(torch, dg, profiling, k, N, prec, steps, warmup, rhs_reps, variant=None, traffic_file=None):
    """One mesh and precision: the LSERK step over `steps` steps in one call
    (value, fused-stage roofline) and the plain right-hand side."""
    p, u, mesh = make_problem(dg, k, N, prec)
    if variant:
        p.set_variant(variant)
    K, Np = p.info.K, p.info.Np
    s = p.info.elem_bytes
    du = p.pack(u)
    del u
    res = p.zeros_state()
    out = p.zeros_state()
    dt = 0.5 * p.info.dt_cfl1
    stream = torch.cuda.current_stream()
    t_rhs = time_rhs(torch, p, du, out, rhs_reps)
    # Warm-up and timed region: one dg_rk_step call each.  The fused stages
    # ping-pong between two state buffers, so a call of n steps (5 n stages)
    # needs a state copy at the end only when n is odd.
    p.rk_step(du, res, 0.0, dt, warmup, stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    p.rk_step(du, res, 0.0, dt, steps, stream)
    e1.record(stream)
    e1.synchronize()
    torch.cuda.synchronize()
    t_total = e0.elapsed_time(e1) / 1e3
    t_stage = t_total / (5 * steps)   # average fused-stage launch in the timed region
    dofs = 6 * K * Np
    tname = "double" if prec == "fp64" else "float"
    if p.variant.startswith("mfma"):
        cfg = dg.variant_id(p.variant) - dg.variant_id("mfma")   # tuning configuration of the kernel
        kname = f"void dgd::rhs_mfma_kernel<{N}, {tname}, true, {MIX[prec]}, false, {cfg}>(dgd::RhsArgs)"
        kname_rhs = f"void dgd::rhs_mfma_kernel<{N}, {tname}, false, {MIX[prec]}, false, {cfg}>(dgd::RhsArgs)"
    else:
        kname = kname_rhs = f"void dgd::rhs_valu_kernel<{N}, {tname}>(dgd::RhsArgs)"
    traffic_file = traffic_file or os.path.join(ROOT, "profiles", f"rhs_traffic_k{k}_n{N}.txt")
    traffic = profiling.read_traffic(traffic_file, kname)
    bound, achieved, peak, unit = roofline(prec, N, K, t_stage, s, stage=True)
    if prec in ("fp64", "fp32") and not p.variant.startswith("mfma"):
        bound = "alu"
    rb, ra, rp, ru = roofline(prec, N, K, t_rhs, s)
    r = {
        "value": 5 * dofs * steps / t_total / 1e9,
        "ms_per_step": 1e3 * t_total / steps,
        "stage_us": 1e6 * t_stage,
        "rhs_us": 1e6 * t_rhs,
        "rhs_gdofs": dofs / t_rhs / 1e9,
        "roofline": {"bound": bound, "achieved": achieved, "peak": peak,
                     "unit": unit, "frac": achieved / peak, "traffic": traffic,
                     "kernel": kname,
                     "launch_us": 1e6 * t_stage,
                     "algorithmic_flops_per_launch": flops_per_element(N, True) * K,
                     "algorithmic_bytes_per_launch": bytes_per_element(N, s, True) * K,
                     "hbm_GBs_algorithmic": bytes_per_element(N, s, True) * K / t_stage / 1e9},
        "rhs_only": {"kernel": kname_rhs, "launch_us": 1e6 * t_rhs, "bound": rb, "achieved": ra,
                     "peak": rp, "unit": ru, "frac": ra / rp,
                     "traffic": profiling.read_traffic(traffic_file, kname_rhs),
                     "algorithmic_bytes_per_launch": bytes_per_element(N, s) * K},
        "K": K, "Np": Np, "variant": p.variant,
    }
    p.close()
    del du, res, out
    return r


def _summary(r):
    return {kk: r[kk] for kk in ("value", "ms_per_step", "stage_us", "rhs_us", "rhs_gdofs", "roofline", "rhs_only",
                                 "variant", "K", "Np")}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="large", choices=["large", "single", "batch", "sweep"],
                    help="large (default): 48^3 x 6 tets (K = 663,552), N = 5, FP32 headline plus the split "
                         "precisions, the 24^3 x 6 N = 4 mesh and the 64-problem batch as extra keys; "
                         "single: one mesh (--k, --order, --precision); batch: 64 independent problems; "
                         "sweep: orders 1..9 at about 1e7 nodal values per field")
    ap.add_argument("--k", type=int, default=None, help="cube resolution (K = 6 k^3); default 48 (large), 24 (single)")
    ap.add_argument("--order", type=int, default=None, help="default 5 (large), 4 (single)")
    ap.add_argument("--precision", default=None,
                    choices=["fp64", "fp32", "bf16x3", "f16x3", "bf16x2", "f16x2", "bf16", "f16"],
                    help="default fp32 (large), fp64 (single)")
    ap.add_argument("--also", default=None,
                    help="other precisions on the same mesh (comma separated, may be empty); "
                         "default f16x3,bf16x3 (large), fp32,f16x3,bf16x3 (single)")
    ap.add_argument("--no-extras", action="store_true",
                    help="large workload: skip the 24^3 x 6 mesh and the batch")
    ap.add_argument("--rhs-reps", type=int, default=50)
    ap.add_argument("--variant", default=None, help="kernel variant (default: the library's choice)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one torch copy of 256 MiB (scale for the HBM traffic counters)")
    ap.add_argument("--sweep-precisions", default="fp64,fp32,f16x3,bf16x3")
    ap.add_argument("--sweep-orders", default="1,2,3,4,5,6,7,8,9")
    ap.add_argument("--traffic-file", default=None,
                    help="traffic summary written from rocprofv3 --pmc runs (default: profiles/rhs_traffic_k<k>_n<N>.txt)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the multi-GPU path is not part of this build "
              "(see the design notes on how the element partition would shard).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1211_0582_amd import dg

    from paper_1211_0582_amd import profiling

    torch.cuda.set_device(0)
    if args.workload == "batch":
        return bench_batch(args, torch, dg)
    if args.workload == "sweep":
        return bench_sweep(args, torch, dg)
    large = args.workload == "large"
    k = args.k or (48 if large else 24)
    N = args.order or (5 if large else 4)
    prec = args.precision or ("fp32" if large else "fp64")
    also = args.also if args.also is not None else ("f16x3,bf16x3" if large else "fp32,f16x3,bf16x3")
    if args.calibrate_copy:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    others = [x for x in also.split(",") if x and x != prec]
    results = {}
    for pr in [prec] + others:
        print(f"bench: k={k} N={N} {pr}", file=sys.stderr, flush=True)
        results[pr] = measure(torch, dg, profiling, k, N, pr, args.steps, args.warmup, args.rhs_reps, args.variant,
                              args.traffic_file)
        torch.cuda.empty_cache()
    main_r = results[prec]
    line = {
        "metric": "GDOF/s per DG RHS eval (Maxwell tets) and % of HBM/MFMA roofline",
        "value": main_r["value"],
        "unit": "GDOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32"}.get(prec, prec + "+f32acc"),
        "data": "synthetic",
        "config": {"workload": f"jittered Kuhn cube {k}^3x6 tets (K={main_r['K']}), N={N} (Np={main_r['Np']}), "
                               f"{prec.upper()} state, PEC cavity + noise, upwind, "
                               f"LSERK(5,4) step = 5 RHS + 5 updates",
                   "K": main_r["K"], "N": N, "precision": prec, "variant": main_r["variant"]},
        "roofline": main_r["roofline"],
        "rhs_us": main_r["rhs_us"],
        "rhs_gdofs": main_r["rhs_gdofs"],
        "stage_us": main_r["stage_us"],
        "rhs_only": main_r["rhs_only"],
        "other_precision": {o: _summary(results[o]) for o in others},
    }
    if large and not args.no_extras:
        small = {}
        for pr in ("fp64", "fp32"):
            print(f"bench: k=24 N=4 {pr}", file=sys.stderr, flush=True)
            small[pr] = _summary(measure(torch, dg, profiling, 24, 4, pr, args.steps, args.warmup, args.rhs_reps))
        line["mesh_24_n4"] = {"workload": "jittered Kuhn cube 24^3x6 tets (K=82944), N=4 (Np=35), "
                                          "PEC cavity + noise, upwind, LSERK(5,4) step", "precisions": small}
        print("bench: 64-problem batch", file=sys.stderr, flush=True)
        line["batch"] = batch_modes(torch, dg, args.steps, args.warmup)
        print("bench: run-time compiled systems", file=sys.stderr, flush=True)
        line["compiled_systems"] = {"workload": "jittered Kuhn cube 24^3x6 tets (K=82944), N=5, FP32, one RHS "
                                                "of a system compiled at run time from its flux description",
                                    "systems": systems_rhs(torch, 24, 5, "fp32", args.rhs_reps)}
    if not args.no_cpu_baseline:
        print("bench: cpu baseline", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(24 if k >= 24 else k, N, 12 if k >= 24 else max(2, k // 2))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
