"""Benchmark of the space-time BEM hot path on one MI355X.

One step = the whole path of the method on one synthetic workload:
assemble V_h, K_h, D_h and M_h^0 (FP64), form the right-hand side of eq.(4),
solve with D_h-preconditioned GMRES in FP64, then solve again with FP32
storage of V_h and D_h inside an FP64 iterative refinement.  Inputs are
resident in HBM before the timed region.  Prints one JSON line.

Default workload (the medium configuration): unit square, 256 boundary
segments, 128 uniform time steps (N = 32768), alpha = 1, Omega_h 64^2 grid
(8192 triangles), manufactured u = exp(k.x + |k|^2 t/alpha), k = (1, 0).
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

# Per work unit of each kernel on the medium workload (units as reported by
# the library's launch timing: matrix entries, or (row, triangle) pairs for
# the M_h^0 moment kernels), measured with rocprofv3 counters:
#   FP64 operations = 64 x (ADD_F64 + MUL_F64 + 2 FMA_F64 + TRANS_F64) wave
#   instructions (inactive lanes included), profiles/counters_fp64_medium.md;
#   HBM bytes = 2 x FETCH_SIZE + WRITE_SIZE (KiB x 1024), the factors from a
#   1 GiB device copy read by the same counters, profiles/counters_hbm_medium.md.
# A kernel changed after its counters were taken has no entry here.  The
# fused tiles k_assemble_dfar<q, true> and k_assemble_dnear<true> count D_h
# entries and write as many V_h entries (16 B per unit).
FLOP_PER_UNIT = {'k_assemble_dfar<3, true>': 4555.6,
    'k_assemble_dnear<true>': 31402.0,
    'k_m0_rows<false>': 16233.1,
    'k_assemble_vkfar<1, 4>': 2399.4,
    'k_assemble_dfar<4, true>': 16174.2,
    'k_assemble_knear<1>': 12373.6,
    'k_m0_tri<false, true, 1>': 58332.9,
    'k_assemble_vkfar<1, 5>': 7447.3,
    'k_m0_pow': 35571.0,
    'k_m0_tri<false, true, 2>': 4523.3,
    'k_m0_pow_gather': 6.0,
    'k_m0_pow_apply': 81.0,
    'k_m0_gather': 6.0}
HBM_BYTES_PER_UNIT = {'k_gemv_n_vec<double>': 8.035,
    'k_assemble_dfar<3, true>': 16.188,
    'k_assemble_dnear<true>': 16.088,
    'k_m0_rows<false>': 24.179,
    'k_assemble_vkfar<1, 4>': 9.805,
    'k_assemble_dfar<4, true>': 16.414,
    'k_gemv_n_vec<float>': 4.035,
    'k_assemble_knear<1>': 9.659,
    'k_m0_tri<false, true, 1>': 24.353,
    'k_assemble_vkfar<1, 5>': 10.03,
    'k_m0_pow': 888.5,
    'k_m0_tri<false, true, 2>': 0.478,
    'k_gemv_n_vec<float hi+lo>': 8.035,
    'k_m0_pow_gather': 70.042,
    'k_m0_pow_apply': 10.821,
    'k_m0_gather': 67.234}
# bytes streamed per stored entry by the matrix-vector kernels
GEMV_BYTES = {"k_gemv_n_vec<double>": 8, "k_gemv_t_vec<double>": 8, "k_gemv_n_vec<float hi+lo>": 8,
              "k_gemv_t_vec<float hi+lo>": 8, "k_gemv_n_vec<float>": 4, "k_gemv_t_vec<float>": 4}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="medium")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-paper-mesh", action="store_true", help="skip the D_h assembly on the paper's Table 2 mesh")
    ap.add_argument("--cpu-sample", type=int, default=0, help="entries per operator for the oracle timing")
    # tolerances calibrated on the medium workload so that both solutions are
    # within 1e-10 (relative l2) of a 1e-15 FP64 solve: plain GMRES stops on
    # the preconditioned residual, the refinement on the FP64 residual of V_h
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

    def step(record):
        t = {}
        e0, e1, e2, e3, e4, e5, e6, e7 = (ev() for _ in range(8))
        e0.record(stream)
        ctx.assemble(L.V | L.D)       # one call: V_h's separated blocks come from D_h's far tiles
        e1.record(stream)
        ctx.assemble(L.K)
        e2.record(stream)
        e3.record(stream)
        ctx.assemble(L.M0)
        e4.record(stream)
        f = ctx.rhs(g, u0)
        e5.record(stream)
        w64, i64 = ctx.solve(f, tol=args.tol, max_it=400)
        e6.record(stream)
        w32, i32 = ctx.solve(f, tol=args.ir_tol, max_it=400, mode=L.FP32_IR, inner_tol=args.inner_tol, max_outer=12,
                             ir_tol=args.ir_tol)
        e7.record(stream)
        torch.cuda.synchronize()
        if record is not None:
            record.append({"V+D": e0.elapsed_time(e1), "K": e1.elapsed_time(e2),
                           "M0": e3.elapsed_time(e4), "rhs": e4.elapsed_time(e5), "solve64": e5.elapsed_time(e6),
                           "solve32": e6.elapsed_time(e7), "i64": i64, "i32": i32})
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
    avg = {k: float(np.mean([r[k] for r in rec])) for k in ("V+D", "K", "M0", "rhs", "solve64", "solve32")}
    value = 3 * entries / (ms_per_step * 1e-3)

    # GEMV rate on V_h (HBM-bound), HIP events on the launch stream
    x = torch.randn(ctx.n, dtype=torch.float64, device=dev)
    y = ctx.apply(L.V, x)
    a, b = ev(), ev()
    reps = 20
    a.record(stream)
    for _ in range(reps):
        ctx.apply(L.V, x, out=y)
    b.record(stream)
    torch.cuda.synchronize()
    gemv_ms = a.elapsed_time(b) / reps
    gemv_gbs = entries * 8 / (gemv_ms * 1e-3) / 1e9

    # accuracy (untimed): both timed solutions against an FP64 solve to 1e-15,
    # the FP32-refined against the FP64 one, and both against the exact flux
    wref, _ = ctx.solve(f, tol=1e-15, max_it=800)
    w64n, w32n, wrn = w64.cpu().numpy(), w32.cpu().numpy(), wref.cpu().numpy()
    err64 = float(np.linalg.norm(w64n - wrn) / np.linalg.norm(wrn))
    err32 = float(np.linalg.norm(w32n - wrn) / np.linalg.norm(wrn))
    ir_vs_fp64 = float(np.linalg.norm(w32n - w64n) / np.linalg.norm(w64n))
    disc64 = float(np.linalg.norm(w64n - wl.w_ref) / np.linalg.norm(wl.w_ref))

    roof = roofline(ktimes)
    kernel_ms = {k: round(v[1] / args.steps, 3) for k, v in sorted(ktimes.items(), key=lambda kv: -kv[1][1])}
    kernel_units = {k: v[2] / v[0] for k, v in ktimes.items()}

    out = {
        "metric": METRIC, "value": value, "unit": "entries/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{args.workload}: N_Gamma={ctx.ng}, N_I={ctx.nt}, N={ctx.n}, M_Omega={ctx.nv}, "
                               f"alpha={wl.alpha}, entries per causal matrix={entries}"},
        "assembly_ms": {k: avg[k] for k in ("V+D", "K", "M0")},
        "assembly_entries_per_s": {"V+D": 2 * entries / (avg["V+D"] * 1e-3), "K": entries / (avg["K"] * 1e-3)},
        "rhs_ms": avg["rhs"],
        "solve_s_fp64": avg["solve64"] * 1e-3, "solve_s_fp32_refined": avg["solve32"] * 1e-3,
        "gmres_iters_fp64": rec[-1]["i64"].iters, "gmres_iters_fp32_inner_total": rec[-1]["i32"].iters,
        "ir_outer_steps": rec[-1]["i32"].outer,
        "true_relres_fp64": rec[-1]["i64"].true_relres, "true_relres_fp32_refined": rec[-1]["i32"].true_relres,
        "solve_tol": {"fp64_precond_relres": args.tol, "fp32_refined_fp64_relres": args.ir_tol,
                      "fp32_inner": args.inner_tol},
        "solution_err_vs_fp64_1e-15_solve": {"fp64": err64, "fp32_refined": err32},
        "fp32_refined_vs_fp64_rel_err": ir_vs_fp64, "discretisation_err_vs_exact_flux": disc64,
        "gemv_V": {"ms": gemv_ms, "GB/s": gemv_gbs, "frac_hbm": gemv_gbs / HBM_PEAK_GBS},
        "roofline": roof,
        "kernel_ms_per_step": kernel_ms,
        "kernel_units_per_launch": kernel_units,
    }
    if not args.no_paper_mesh:
        ctx.close()
        out["paper_table2"] = paper_table2(dev)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_sample)
    print(json.dumps(out), flush=True)


def roofline(ktimes):
    """Roofline of the kernel with the largest event time in the timed steps:
    algorithmic work per launch (per-unit figure x units per launch) over the
    average launch duration from the HIP events."""
    name, (launches, ms, units) = max(ktimes.items(), key=lambda kv: kv[1][1])
    per_launch_s = ms * 1e-3 / launches
    per_launch_units = units / launches
    traffic = HBM_BYTES_PER_UNIT.get(name)
    traffic = traffic * per_launch_units if traffic is not None else None
    if name in GEMV_BYTES:
        achieved = GEMV_BYTES[name] * per_launch_units / per_launch_s / 1e9
        return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": name,
                "launch_ms": per_launch_s * 1e3, "units_per_launch": per_launch_units}
    flop = FLOP_PER_UNIT.get(name)
    achieved = flop * per_launch_units / per_launch_s / 1e12 if flop is not None else None
    return {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / FP64_PEAK_TFLOPS if achieved is not None else None, "traffic": traffic,
            "kernel": name, "launch_ms": per_launch_s * 1e3, "units_per_launch": per_launch_units,
            "flop_per_unit": flop}


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
