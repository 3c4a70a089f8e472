"""Benchmark of the space-time BEM hot path on one MI355X.

One step = the forward path of the method on one synthetic workload, in
two phases that keep the resident matrices within the GPU's memory:
  1. assemble V_h, K_h, D_h and M_h^0 in FP64 in one call (V_h's and K_h's
     separated blocks come from D_h's far tiles), form the right-hand side of
     eq.(4), release K_h and M_h^0, solve with D_h-preconditioned GMRES,
     release V_h and D_h;
  2. assemble V_h and D_h into FP32 storage (V_h as an FP32 hi + lo pair
     computed in FP64, D_h in FP32 arithmetic on separated time blocks; no
     FP64 copy), solve by FP64 iterative refinement around FP32 inner GMRES.
Inputs are resident in HBM before the timed region.  Prints one JSON line.

Default workload (the precision configuration, the largest that fits one
GPU): unit square, 512 boundary segments, 256 uniform time steps
(N = 131072), alpha = 1, Omega_h 128^2 grid (32768 triangles),
manufactured u = exp(k.x + |k|^2 t/alpha), k = (0.7, -0.7).  Beside the
step it times the adjoint gradient on the differentiation workload and the
D_h assembly on the paper's Table 2 mesh.
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

METRIC = "entries/s (V_h,K_h,D_h) + precond. GMRES solve s to 1e-10, FP64 vs FP32-refined"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3

# HBM bytes per work unit of a kernel (units as reported by the library's
# launch timing), from rocprofv3 counters: 2 x FETCH_SIZE + WRITE_SIZE
# (KiB x 1024) per dispatch over the units of the dispatch; the factor 2 on
# FETCH_SIZE comes from a 1 GiB device copy read by the same counters.  A
# kernel changed after its counters were taken has no entry here.
HBM_BYTES_PER_UNIT = {
    # precision workload, profiles/dfar_q3_precision_counters.md: FETCH_SIZE
    # 165,364 KiB (x 2) and WRITE_SIZE 196,418,614 KiB per dispatch of
    # 8.2248e9 D entries (the D, V and K entries written, FP64)
    "k_assemble_dfar<3, true, true>": 24.50,
}
# bytes streamed per stored entry by the matrix-vector kernels
GEMV_BYTES = {"k_gemv_n_vec<double>": 8, "k_gemv_t_vec<double>": 8, "k_gemv_n_vec<float hi+lo>": 8,
              "k_gemv_t_vec<float hi+lo>": 8, "k_gemv_n_vec<float>": 4, "k_gemv_t_vec<float>": 4}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="precision")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-paper-mesh", action="store_true", help="skip the D_h assembly on the paper's Table 2 mesh")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint gradient on the differentiation workload")
    ap.add_argument("--no-accuracy", action="store_true", help="skip the untimed reference solve after the steps")
    ap.add_argument("--cpu-sample", type=int, default=0, help="entries per operator for the oracle timing")
    # tolerances chosen so that both solutions are within 1e-10 (relative l2)
    # of an FP64 solve to 1e-15 (tests/test_gpu_workloads.py checks them on
    # the precision workload): plain GMRES stops on the preconditioned
    # residual, the refinement on the FP64 residual of V_h
    ap.add_argument("--tol", type=float, default=3e-11, help="FP64 GMRES: preconditioned relative residual")
    ap.add_argument("--ir-tol", type=float, default=1e-12, help="FP32 refinement: FP64 relative residual")
    ap.add_argument("--inner-tol", type=float, default=1e-6, help="FP32 refinement: inner GMRES tolerance")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 1 GiB device-to-device copy (scale for the HBM byte counters)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); sharding over several GPUs "
              "is not implemented", file=sys.stderr)
        sys.exit(2)
    import torch
    import workloads as W
    import paper_1811_05224_amd as P
    from paper_1811_05224_amd import _lib as L

    wl = W.make(args.workload)
    dev = torch.device("cuda:0")
    if args.copy_calibration:
        src = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    ctx = P.Context.from_workload(wl, device=dev)
    g = torch.as_tensor(wl.g, device=dev)
    u0 = torch.as_tensor(wl.u0, device=dev)
    stream = torch.cuda.current_stream()
    ev = lambda: torch.cuda.Event(enable_timing=True)
    phases = ("V+K+D+M0 fp64", "rhs", "solve fp64", "V+D fp32", "solve fp32-refined")

    def step(record):
        e = [ev() for _ in range(len(phases) + 1)]
        e[0].record(stream)
        # V_h's and K_h's separated blocks come from D_h's far tiles (one call)
        ctx.assemble(L.V | L.K | L.D | L.M0)
        e[1].record(stream)
        f = ctx.rhs(g, u0)
        e[2].record(stream)
        ctx.release(L.K | L.M0)
        w64, i64 = ctx.solve(f, tol=args.tol, max_it=400)
        e[3].record(stream)
        ctx.release(L.V | L.D)
        ctx.assemble(L.V | L.D, precision=L.FP32_IR)
        e[4].record(stream)
        w32, i32 = ctx.solve(f, tol=args.ir_tol, max_it=400, mode=L.FP32_IR, inner_tol=args.inner_tol, max_outer=12,
                             ir_tol=args.ir_tol)
        e[5].record(stream)
        torch.cuda.synchronize()
        ctx.release(L.V | L.D)
        if record is not None:
            r = {ph: e[q].elapsed_time(e[q + 1]) for q, ph in enumerate(phases)}
            r.update(i64=i64, i32=i32)
            record.append(r)
        return f, w64, w32

    for _ in range(args.warmup):
        step(None)
    torch.cuda.synchronize()
    rec = []
    ctx.set_timing(True)      # HIP events around every assembly and GEMV launch, on its stream
    t0 = time.perf_counter()
    for _ in range(args.steps):
        f, w64, w32 = step(rec)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = 1e3 * wall / args.steps
    ktimes = ctx.kernel_times()
    ctx.set_timing(False)

    entries = ctx.packed_entries            # per causal matrix
    avg = {ph: float(np.mean([r[ph] for r in rec])) for ph in phases}
    value = 3 * entries / (ms_per_step * 1e-3)
    last64, last32 = rec[-1]["i64"], rec[-1]["i32"]

    out = {
        "metric": METRIC, "value": value, "unit": "entries/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{args.workload}: N_Gamma={ctx.ng}, N_I={ctx.nt}, N={ctx.n}, M_Omega={ctx.nv}, "
                               f"alpha={wl.alpha}, entries per causal matrix={entries}"},
        "phase_ms": avg,
        "assembly_entries_per_s": {"V+K+D fp64 (M0 in the same call)": 3 * entries / (avg["V+K+D+M0 fp64"] * 1e-3),
                                   "V+D fp32 storage": 2 * entries / (avg["V+D fp32"] * 1e-3)},
        "solve_s_fp64": avg["solve fp64"] * 1e-3, "solve_s_fp32_refined": avg["solve fp32-refined"] * 1e-3,
        "solve_speedup_fp32_refined": avg["solve fp64"] / avg["solve fp32-refined"],
        "gmres_iters_fp64": last64.iters, "gmres_iters_fp32_inner_total": last32.iters,
        "ir_outer_steps": last32.outer,
        "true_relres_fp64": last64.true_relres, "true_relres_fp32_refined": last32.true_relres,
        "solve_tol": {"fp64_precond_relres": args.tol, "fp32_refined_fp64_relres": args.ir_tol,
                      "fp32_inner": args.inner_tol},
        "storage_GB": {"V+K+D fp64": 3 * entries * 8 / 1e9, "M0 fp64": ctx.n * ctx.nv * 8 / 1e9,
                       "V+D fp32 (V hi+lo, D fp32)": entries * 12 / 1e9},
    }
    out["gemv"] = gemv_rates(ktimes)
    out["roofline"] = roofline(ktimes)
    out["kernel_ms_per_step"] = {k: round(v[1] / args.steps, 3) for k, v in sorted(ktimes.items(), key=lambda kv: -kv[1][1])}
    out["kernel_tflops"] = {k: v[3] / (v[1] * 1e-3) / 1e12 for k, v in ktimes.items() if v[3] > 0}
    out["kernel_units_per_launch"] = {k: v[2] / v[0] for k, v in ktimes.items()}

    if not args.no_accuracy:
        # untimed: both timed solutions against an FP64 solve to 1e-15, the
        # FP32-refined one against the FP64 one, and against the exact flux
        ctx.assemble(L.V | L.D)
        wref, _ = ctx.solve(f, tol=1e-15, max_it=800)
        w64n, w32n, wrn = w64.cpu().numpy(), w32.cpu().numpy(), wref.cpu().numpy()
        out["solution_err_vs_fp64_1e-15_solve"] = {"fp64": float(np.linalg.norm(w64n - wrn) / np.linalg.norm(wrn)),
                                                   "fp32_refined": float(np.linalg.norm(w32n - wrn) / np.linalg.norm(wrn))}
        out["fp32_refined_vs_fp64_rel_err"] = float(np.linalg.norm(w32n - w64n) / np.linalg.norm(w64n))
        out["discretisation_err_vs_exact_flux"] = float(np.linalg.norm(w64n - wl.w_ref) / np.linalg.norm(wl.w_ref))
    ctx.close()
    del ctx
    torch.cuda.empty_cache()
    if not args.no_adjoint:
        out["adjoint_diff_workload"] = adjoint_gradient(dev)
    if not args.no_paper_mesh:
        out["paper_table2"] = paper_table2(dev)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_sample)
    print(json.dumps(out), flush=True)


def gemv_rates(ktimes):
    """Matrix-vector kernels: average launch time and stream rate (bytes of
    the stored entries read once per product) from the timed steps."""
    res = {}
    for name, per in GEMV_BYTES.items():
        if name in ktimes:
            launches, ms, units = ktimes[name][:3]
            gbs = per * units / (ms * 1e-3) / 1e9
            res[name] = {"launch_ms": ms / launches, "GB/s": gbs, "frac_hbm": gbs / HBM_PEAK_GBS}
    return res


def roofline(ktimes):
    """Roofline of the kernel with the largest event time in the timed steps:
    algorithmic work per launch (the library's operation count, or bytes for
    a matrix-vector kernel) over the average launch duration from the HIP
    events."""
    name, (launches, ms, units, flops) = max(ktimes.items(), key=lambda kv: kv[1][1])
    per_launch_s = ms * 1e-3 / launches
    per_launch_units = units / launches
    traffic = HBM_BYTES_PER_UNIT.get(name)
    traffic = traffic * per_launch_units if traffic is not None else None
    base = {"kernel": name, "launch_ms": per_launch_s * 1e3, "units_per_launch": per_launch_units, "traffic": traffic}
    if name in GEMV_BYTES:
        achieved = GEMV_BYTES[name] * per_launch_units / per_launch_s / 1e9
        return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, **base}
    peak = FP64_PEAK_TFLOPS             # every assembly kernel computes in FP64 (f32-store only stores FP32)
    achieved = flops / launches / per_launch_s / 1e12 if flops > 0 else None
    return {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
            "frac": achieved / peak if achieved is not None else None,
            "flop_per_unit": flops / units if flops > 0 else None, **base}


def adjoint_gradient(dev):
    """The adjoint of the differentiation workload (128 segments x 128 steps,
    N = 16384): gradient of J = 1/2 ||w_h - w_obs||^2 in g and alpha at
    alpha = 1 (data from alpha* = 1.5 plus seeded noise): forward solve,
    transposed solve, (1/2 M_h + K_h)^T lam and lam^T (dK g - dM0 u0 - dV w),
    with the alpha-derivative matrices assembled; FP64, timed with HIP
    events after one untimed pass."""
    import torch
    import workloads as W
    import paper_1811_05224_amd as P
    from paper_1811_05224_amd import _lib as L
    wl = W.make("diff")
    c = P.Context.from_workload(wl, device=dev)
    g = torch.as_tensor(wl.g, device=dev)
    u0 = torch.as_tensor(wl.u0, device=dev)
    w_obs = torch.as_tensor(wl.w_ref + wl.extra["sigma"] * wl.extra["noise"], device=dev)
    stream = torch.cuda.current_stream()
    names = ("assemble V,K,D,M0", "assemble dV,dK,dM0", "forward solve", "adjoint solve", "grad g", "grad alpha")
    res = None
    for rep in range(2):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(len(names) + 1)]
        e[0].record(stream)
        c.assemble(L.V | L.K | L.D | L.M0)
        e[1].record(stream)
        c.assemble(L.DV | L.DK | L.DM0)
        e[2].record(stream)
        f = c.rhs(g, u0)
        w, i1 = c.solve(f, tol=1e-12, max_it=300)
        e[3].record(stream)
        lam, i2 = c.solve(w - w_obs, tol=1e-12, max_it=300, trans=True)
        e[4].record(stream)
        gg = c.rhs_adjoint(lam)
        e[5].record(stream)
        ga = c.grad_alpha(lam, w, g, u0)
        e[6].record(stream)
        torch.cuda.synchronize()
        res = {n: e[q].elapsed_time(e[q + 1]) for q, n in enumerate(names)}
    # dJ/dalpha with the alpha-derivative matrices recomputed block-row range
    # by range instead of stored (the path for meshes where they do not fit)
    c.release(L.DV | L.DK | L.DM0)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    ga2 = c.grad_alpha(lam, w, g, u0)
    b.record(stream)
    torch.cuda.synchronize()
    res["grad alpha, matrices recomputed (not stored)"] = a.elapsed_time(b)
    d_alpha, d_alpha2 = float(ga.cpu()[0]), float(ga2.cpu()[0])
    c.close()
    return {"workload": "diff: N_Gamma=128, N_I=128, N=16384, M_Omega=1089, alpha=1.0", "ms": res,
            "gradient_ms": sum(res[n] for n in names[1:]), "iters": {"forward": i1.iters, "adjoint": i2.iters},
            "dJ_dalpha": d_alpha, "dJ_dalpha_recomputed_rel_diff": abs(d_alpha2 - d_alpha) / abs(d_alpha),
            "norm_dJ_dg": float(gg.norm())}


def paper_table2(dev):
    """D_h assembly on the paper's 65 536-element mesh (Sec. 4 setting:
    unit square, alpha = 10, 512 segments x 128 uniform steps; 2.16e9 entries
    of the lower block triangle, 17.3 GB), timed with HIP events after one
    untimed assembly; the paper's time for it is 184.1 s on one node
    (Table 2)."""
    import torch
    import workloads as W
    import paper_1811_05224_amd as P
    from paper_1811_05224_amd import _lib as L
    wl = W.paper_level(7)
    c = P.Context.from_workload(wl, device=dev)
    c.assemble(L.D)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    stream = torch.cuda.current_stream()
    a.record(stream)
    c.assemble(L.D)
    b.record(stream)
    torch.cuda.synchronize()
    s = a.elapsed_time(b) * 1e-3
    ent = c.packed_entries
    c.close()
    return {"mesh": "65 536 space-time elements: 512 segments x 128 steps, alpha = 10", "entries": ent,
            "D_h_assembly_s": s, "entries_per_s": ent / s, "paper_s": 184.1,
            "paper_hardware": "one Salomon node: 2 x 12-core Xeon E5-2680v3 (Haswell), 2 MPI x 12 OpenMP",
            "paper_over_this": 184.1 / s}


def cpu_baseline(wl, nsamp):
    """The oracle (long-double CPU code) on a bounded sample of the same
    workload: random entries of V_h, K_h and D_h, all host cores."""
    from oracle.oracle import Oracle
    o = Oracle.from_workload(wl)
    rng = np.random.default_rng(0)
    ng, nt = wl.n_gamma, wl.n_t
    n = nsamp or 40000
    res = {}
    total_e, total_s = 0, 0.0
    for op, cnt in (("V", n), ("K", n), ("D", max(n // 8, 50))):
        k = rng.integers(0, nt, cnt)
        m = np.minimum(k, rng.integers(0, nt, cnt))
        idx = np.stack([k, m, rng.integers(0, ng, cnt), rng.integers(0, ng, cnt)], 1)
        t0 = time.perf_counter()
        o.entries(op, idx)
        dt = time.perf_counter() - t0
        res[op] = cnt / dt
        total_e += cnt
        total_s += dt
    # V, K, D weighted equally: entries of the three matrices per second
    rate = 3.0 / sum(1.0 / res[op] for op in ("V", "K", "D"))
    return {"value": rate, "unit": "entries/s", "cores": o.nthreads, "kind": "oracle",
            "sample": f"{n} random V_h, {n} K_h, {max(n // 8, 50)} D_h entries of the same workload "
                      f"({total_s:.1f} s); per-operator entries/s " + ", ".join(f"{k}={v:.0f}" for k, v in res.items())}


if __name__ == "__main__":
    main()
