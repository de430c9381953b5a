"""Benchmark: steady-state HOTRG step of the 4D Ising model on one MI355X.

Workload (the metric's configuration): Dcut = 10, h = 0, beta = 0.14968 (a
point of the 16-point scan in [0.1494, 0.1500]), bf16x3 contraction with FP64
environments / eigh / norms, impurity tensors S_m and S_e carried, so every
step contracts M = 3 * 10^4 operand rows against N = 10^4 columns over
K = 10^7 (2 M N K = 6.0e15 algorithmic flops).  Steps 1-3 (bond dims ramping
up to 10) run untimed; W warm-up steps follow; then exactly K steps are timed
with a device synchronisation on both sides.

Prints one JSON line.  --precision fp64 times the plain FP64 path instead.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_BF16 = 2.5e15     # MI355X dense bf16 MFMA, flop/s
PEAK_FP64 = 78.6e12    # MI355X FP64 matrix, flop/s

# HBM bytes per GEMM call (main + tail dispatch + fix-up) of the bf16x3 GEMM at this workload, from two
# rocprofv3 --pmc passes (FETCH_SIZE x 2.0, WRITE_SIZE x 1.0, factors from a
# plain 2 GiB copy); valid only while the kernel source is the one profiled.
GEMM_TRAFFIC_BYTES = {("z2", 10, True, True): 71635075814}
GEMM_TRAFFIC_SRC_SHA = "5564fef28b45ecad"


BF16X3_SECTION = "// ---------------------------------------------------------------- bf16x3 ---"


def gemm_source_sha():
    """sha256 prefix of the bf16x3 part of gemm.hip (from its section marker to
    the end of the file), the source the stored traffic counters belong to."""
    import hashlib
    with open(os.path.join(ROOT, "paper_1906_06060_amd", "csrc", "gemm.hip")) as f:
        text = f.read()
    return hashlib.sha256(text[text.index(BF16X3_SECTION):].encode()).hexdigest()[:16]


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=2)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--dcut", type=int, default=10)
    p.add_argument("--beta", type=float, default=0.14968)
    p.add_argument("--h", type=float, default=0.0)
    p.add_argument("--precision", choices=["bf16x3", "fp64"], default="bf16x3")
    p.add_argument("--no-impurities", action="store_true")
    p.add_argument("--dense", action="store_true",
                   help="contract densely even at h = 0 (no Z2 block form), for comparison")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-dcut", type=int, default=8)
    p.add_argument("--cpu-slices", type=int, default=2)
    p.add_argument("--no-fp64", action="store_true", help="skip the FP64 step sub-record")
    p.add_argument("--fp64-pure", action="store_true",
                   help="FP64 sub-record on a pure-T step (impurities off) instead of the bench workload")
    p.add_argument("--no-adjoint", action="store_true", help="skip the adjoint sub-record")
    p.add_argument("--adjoint", type=int, default=0, metavar="NSTEPS",
                   help="time an FP64 flow of NSTEPS steps with checkpoints plus hotrg_backward "
                        "(impurities off; Dcut from --dcut)")
    p.add_argument("--precision-study", type=int, default=0, metavar="NSTEPS",
                   help="run bf16x3 and FP64 flows of NSTEPS steps side by side for each --betas "
                        "and print the per-step differences of lnZ/N, e, m (impurity estimators)")
    p.add_argument("--betas", type=str, default="0.1490,0.1497,0.1502")
    p.add_argument("--table", type=str, default="", metavar="DCUTS",
                   help="comma-separated Dcut values: forward step and reverse pass, mixed vs FP64")
    p.add_argument("--table-precisions", type=str, default="bf16x3,fp64")
    p.add_argument("--table-parts", type=str, default="forward,adjoint")
    p.add_argument("--tc", type=str, default="", metavar="DCUTS",
                   help="comma-separated Dcut values: locate T_c(Dcut) from the settled X indicator "
                        "(scan --tc-scan for a bracket, then --tc-iterations bisection rounds)")
    p.add_argument("--tc-scan", type=str, default="0.144:0.156:0.002", metavar="LO:HI:STEP")
    p.add_argument("--tc-iterations", type=int, default=10)
    p.add_argument("--tc-steps", type=int, default=40)
    p.add_argument("--tc-precision", choices=["bf16x3", "fp64"], default="bf16x3")
    p.add_argument("--jump", type=int, default=0, metavar="DCUT",
                   help="energy and magnetisation jumps at --jump-tc from flows at T_c -/+ --jump-dt")
    p.add_argument("--jump-tc", type=float, default=0.0)
    p.add_argument("--jump-dt", type=str, default="0.004,0.008,0.012")
    p.add_argument("--jump-steps", type=int, default=40)
    p.add_argument("--jump-precision", choices=["bf16x3", "fp64"], default="bf16x3")
    p.add_argument("--copy-calibration", action="store_true",
                   help="only run a plain device copy of 2 GiB (for scaling HBM byte counters)")
    return p.parse_args()


def copy_calibration():
    """A plain device-to-device copy of exactly 2 GiB read + 2 GiB written:
    the reference for FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    x = torch.ones(1 << 28, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": x.numel() * 8, "copy_bytes_written": y.numel() * 8}), flush=True)


def cpu_baseline(dcut, nslices):
    """The CPU oracle's own contraction (oracle.hotrg.coarse_grain: NumPy with
    BLAS-backed tensordot, its own contraction order) on a bounded part of a
    steady-state step: `nslices` of the D^2 output (m1, m2) slices of one
    Dcut = `dcut` step of T (seeded Z2 input of dims D^4, seeded isometries
    D^2 x D), timed on the host.  Reported as the algorithmic rate
    2 D^15 (nslices / D^2) / t, with the projected full pure-T step time."""
    import numpy as np
    from oracle import hotrg as OH
    from tests import synth
    threads, blas = os.cpu_count(), "unknown"
    try:
        import threadpoolctl
        info = [i for i in threadpoolctl.threadpool_info() if i.get("user_api") == "blas"]
        if info:
            threads = max(i.get("num_threads", 1) for i in info)
            blas = ",".join(sorted({f"{i.get('internal_api')} {i.get('version')}" for i in info}))
    except Exception:
        pass
    D = dcut
    T = synth.z2_tensor((D, D, D, D), seed=5)
    Us = {q: synth.isometry(D * D, D, seed=50 + q) for q in range(3)}
    pairs = [(i // D, i % D) for i in range(nslices)]
    t0 = time.perf_counter()
    out = OH.coarse_grain(T, T, Us, 3, slices=pairs)
    dt = time.perf_counter() - t0
    assert np.isfinite(out).all()
    flops = 2.0 * D ** 15 * nslices / D ** 2
    return {
        "value": flops / dt / 1e12,
        "unit": "TFLOP/s",
        "cores": threads,
        "kind": "oracle",
        "blas": blas,
        "host_cpus": os.cpu_count(),
        "sample": f"oracle.hotrg.coarse_grain of one steady-state Dcut={D} step of T (dims {D}^4, "
                  f"2 D^15 = {2.0 * D ** 15:.3g} flop), {nslices} of its {D * D} output (m1, m2) slices "
                  f"in {dt:.1f} s on {threads} BLAS threads; projected full pure-T step "
                  f"{dt * D * D / nslices:.1f} s",
    }


def precision_study(a):
    """bf16x3 contraction vs the FP64 path on the same flows (Dcut from --dcut,
    impurities on): per step the relative difference of lnZ/N and the absolute
    differences of the impurity energy and magnetisation."""
    from paper_1906_06060_amd import hotrg as H
    out = []
    for beta in [float(b) for b in a.betas.split(",")]:
        runs = {}
        for name, prec in (("fp64", H.FP64), ("bf16x3", H.BF16X3)):
            t0 = time.perf_counter()
            runs[name] = H.flow(beta, a.h, a.dcut, a.precision_study, precision=prec)
            runs[name + "_s"] = time.perf_counter() - t0
            print(f"[precision-study] beta={beta} {name}: {a.precision_study} steps in "
                  f"{runs[name + '_s']:.1f} s", file=sys.stderr, flush=True)
        rows = []
        for f, m in zip(runs["fp64"], runs["bf16x3"]):
            rows.append({"n": f["n"], "lnz_fp64": f["lnz_per_site"],
                         "d_lnz_rel": abs(m["lnz_per_site"] - f["lnz_per_site"]) / abs(f["lnz_per_site"]),
                         "e_fp64": f["e_imp"], "d_e": abs(m["e_imp"] - f["e_imp"]),
                         "m_fp64": f["m_imp"], "d_m": abs(m["m_imp"] - f["m_imp"]),
                         "X_fp64": f["X"], "d_X": abs(m["X"] - f["X"])})
        out.append({"beta": beta, "h": a.h, "dcut": a.dcut, "fp64_s": round(runs["fp64_s"], 2),
                    "bf16x3_s": round(runs["bf16x3_s"], 2), "steps": rows,
                    "max_d_lnz_rel": max(r["d_lnz_rel"] for r in rows),
                    "max_d_e": max(r["d_e"] for r in rows), "max_d_m": max(r["d_m"] for r in rows)})
        print(json.dumps(out[-1]), flush=True)


def adjoint_run(a):
    """Forward flow with per-step checkpoints, then the reverse pass: the
    energy and magnetisation of the flow's last step by differentiation."""
    import torch
    from paper_1906_06060_amd import hotrg as H
    ctx = H.Context(a.beta, a.h, a.dcut, precision=H.FP64, impurities=False, keep_checkpoints=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for n in range(a.adjoint):
        ctx.step(n % 4)
    lnz = ctx.lnz()
    t1 = time.perf_counter()
    db, dh = ctx.backward()
    t2 = time.perf_counter()
    ob = ctx.observables()
    ctx.close()
    print(json.dumps({
        "metric": "HOTRG forward + reverse-mode adjoint time",
        "value": round(t2 - t0, 3), "unit": "s", "higher_is_better": False,
        "config": {"workload": f"4D Ising HOTRG, Dcut={a.dcut}, {a.adjoint} steps, FP64, checkpoints, pure T",
                   "beta": a.beta, "h": a.h, "dims": list(ob["dims"])},
        "forward_s": round(t1 - t0, 3), "backward_s": round(t2 - t1, 3),
        "lnz_per_site": lnz, "dlnz_dbeta": db, "dlnz_dh": dh,
        "energy_per_site": -db, "magnetisation": dh / a.beta if a.beta else None,
    }), flush=True)


def tc_run(a):
    """T_c(Dcut) from X^(n) (Sec. 3): per Dcut, pure-T flows at h = 0 over a
    beta grid until the settled X changes from 1 to 2, then bisection."""
    from paper_1906_06060_amd import hotrg as H
    from paper_1906_06060_amd import tc
    prec = H.BF16X3 if a.tc_precision == "bf16x3" else H.FP64
    lo, hi, st = (float(v) for v in a.tc_scan.split(":"))
    grid = [round(lo + i * st, 10) for i in range(int(round((hi - lo) / st)) + 1)]
    for dcut in [int(v) for v in a.tc.split(",")]:
        cache, times = {}, []

        def x_of(beta):
            if beta not in cache:
                t0 = time.perf_counter()
                cache[beta] = tc.x_history(beta, dcut, a.tc_steps, prec)[-1]
                times.append(time.perf_counter() - t0)
                print(f"[tc] Dcut={dcut} beta={beta:.9f} X={cache[beta]:.6f} ({times[-1]:.2f} s)",
                      file=sys.stderr, flush=True)
            return cache[beta]

        t0 = time.perf_counter()
        pair, scan = tc.bracket_by_scan(x_of, grid)
        line = {"metric": "T_c(Dcut) from the settled X indicator", "unit": "T (J = k_B = 1)",
                "higher_is_better": None,
                "config": {"workload": f"4D Ising HOTRG, pure T, h = 0, Dcut={dcut}, {a.tc_steps} steps "
                                       f"(lattice {2 ** (a.tc_steps // 4)}^4), {a.tc_precision}",
                           "scan": a.tc_scan, "iterations": a.tc_iterations},
                "scan": [{"beta": p["beta"], "X": p["X"]} for p in scan]}
        if pair is None:
            line.update(value=None, error="no disordered-to-ordered change on the scan grid")
        else:
            r = tc.bisect_transition(x_of, pair[0], pair[1], a.tc_iterations)
            line.update(value=r["T_c"], T_c_halfwidth=r["T_c_halfwidth"], beta_c=r["beta_c"],
                        beta_bracket=[r["beta_lo"], r["beta_hi"]], unsettled_points=r["unsettled"],
                        bisection=[{"beta": p["beta"], "X": p["X"]} for p in r["points"][2:]])
        line.update(flows=len(times), seconds_per_flow=round(sum(times) / max(len(times), 1), 3),
                    total_s=round(time.perf_counter() - t0, 2))
        print(json.dumps(line), flush=True)


def jump_run(a):
    """Delta E and Delta m at T_c(Dcut) (Sec. 3): per temperature one flow at
    h = 0 (energy) and two at h = 1e-9, 2e-9 (magnetisation, continued to
    h -> 0); straight lines from both sides evaluated at T_c."""
    from paper_1906_06060_amd import hotrg as H
    from paper_1906_06060_amd import jump
    prec = H.BF16X3 if a.jump_precision == "bf16x3" else H.FP64
    dts = [float(v) for v in a.jump_dt.split(",")]
    temps = sorted([a.jump_tc - d for d in dts] + [a.jump_tc + d for d in dts])
    pts = []
    t0 = time.perf_counter()
    for T in temps:
        t1 = time.perf_counter()
        pts.append(jump.point(1.0 / T, a.jump, a.jump_steps, 1e-9, 2e-9, prec))
        print(f"[jump] Dcut={a.jump} T={T:.6f} e={pts[-1]['e']:.9f} m={pts[-1]['m']:.9f} "
              f"X={pts[-1]['X']:.4f} ({time.perf_counter() - t1:.1f} s)", file=sys.stderr, flush=True)
    r = jump.jumps_from_points(pts, a.jump_tc)
    print(json.dumps({"metric": "first-order jumps at T_c(Dcut)", "unit": "per site", "higher_is_better": None,
                      "config": {"workload": f"4D Ising HOTRG with impurities, Dcut={a.jump}, {a.jump_steps} steps "
                                             f"(lattice {2 ** (a.jump_steps // 4)}^4), {a.jump_precision}, "
                                             f"h = 0 / 1e-9 / 2e-9", "T_c": a.jump_tc, "dT": dts},
                      **r, "points": pts, "flows": 3 * len(temps),
                      "total_s": round(time.perf_counter() - t0, 2)}), flush=True)


def table_run(a):
    """Per Dcut and precision: one steady-state forward step with impurities
    (after the three ramp-up steps), and the reverse pass of a checkpointed
    pure-T flow of four steps (three ramp-up + one steady-state step).  One
    JSON line per measurement."""
    import torch
    from paper_1906_06060_amd import hotrg as H
    for D in [int(x) for x in a.table.split(",")]:
        for pname in a.table_precisions.split(","):
            prec = H.BF16X3 if pname == "bf16x3" else H.FP64
            peak = PEAK_BF16 if prec == H.BF16X3 else PEAK_FP64
            issue = 3.0 if prec == H.BF16X3 else 1.0
            parts = a.table_parts.split(",")
            if "forward" in parts:
                ctx = H.Context(a.beta, a.h, D, precision=prec, impurities=True)
                for n in range(3):
                    ctx.step(n % 4)
                    print(f"[table] Dcut={D} {pname} forward ramp step {n + 1} done", file=sys.stderr, flush=True)
                dims_in, _ = ctx.dims()
                ctx.reset_stats()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                ctx.step(3)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                ob = ctx.observables()
                st = ctx.gemm_stats()
                ctx.close()
                flops = st["flops"]  # 2 M N K summed over the step's contraction GEMMs
                print(json.dumps({"table": "forward", "dcut": D, "precision": pname, "step_s": round(dt, 3),
                                  "step_flops": flops, "dims_in": list(dims_in),
                                  "tflops_alg": round(flops / dt / 1e12, 2),
                                  "pct_peak_issued": round(100 * issue * flops / dt / peak, 2),
                                  "gemm_s": round(st["ms"] / 1e3, 3),
                                  "device_gb": round(ob["device_bytes"] / 1e9, 2),
                                  "lnz_per_site": ob["lnz_per_site"], "dims": list(ob["dims"])}), flush=True)
            if "adjoint" in parts:
                ctx = H.Context(a.beta, a.h, D, precision=prec, impurities=False, keep_checkpoints=True)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for n in range(4):
                    ctx.step(n % 4)
                    print(f"[table] Dcut={D} {pname} checkpointed step {n + 1} done", file=sys.stderr, flush=True)
                lnz = ctx.lnz()
                t1 = time.perf_counter()
                db, dh = ctx.backward()
                t2 = time.perf_counter()
                ob = ctx.observables()
                ctx.close()
                print(json.dumps({"table": "adjoint", "dcut": D, "precision": pname, "steps": 4,
                                  "forward_s": round(t1 - t0, 3), "backward_s": round(t2 - t1, 3),
                                  "backward_over_forward": round((t2 - t1) / (t1 - t0), 2),
                                  "device_gb": round(ob["device_bytes"] / 1e9, 2),
                                  "lnz_per_site": lnz, "dlnz_dbeta": db, "dlnz_dh": dh}), flush=True)


def fp64_step(a, D, imp):
    """The plain FP64 path on the same flow: the three ramp-up steps, then one
    timed steady-state step (FP64 environments, eigh and contraction)."""
    import torch
    from paper_1906_06060_amd import hotrg as H
    ctx = H.Context(a.beta, a.h, D, precision=H.FP64, impurities=imp, dense_only=a.dense)
    for n in range(3):
        ctx.step(n)
    ctx.reset_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(3)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = ctx.gemm_stats()
    ob = ctx.observables()
    ctx.close()
    dense = 2.0 * (3 if imp else 1) * D ** 15
    gemm_s = st["ms"] / 1e3
    print(f"[bench] fp64 step {dt:.2f} s", file=sys.stderr, flush=True)
    return {
        "step_s": round(dt, 3),
        "rows": "T+S_m+S_e" if imp else "T",
        "dense_flops": dense,
        "tflops_dense": round(dense / dt / 1e12, 3),
        "executed_flops": st["flops"],
        "gemm_s": round(gemm_s, 3),
        "gemm_tflops_executed": round(st["flops"] / gemm_s / 1e12, 3) if gemm_s > 0 else None,
        "gemm_frac_of_fp64_peak": round(st["flops"] / gemm_s / PEAK_FP64, 4) if gemm_s > 0 else None,
        "lnz_per_site": ob["lnz_per_site"],
    }


def adjoint_step(a, D, nsteps=4):
    """Forward flow of `nsteps` pure-T steps with per-step checkpoints (three
    ramp-up steps and one steady-state step, bf16x3 from step 4) and the
    reverse pass hotrg_backward: E = -dlnZ/dbeta, M = dlnZ/dh."""
    import torch
    from paper_1906_06060_amd import hotrg as H
    ctx = H.Context(a.beta, a.h, D, precision=H.BF16X3, impurities=False, keep_checkpoints=True,
                    dense_only=a.dense)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for n in range(nsteps):
        ctx.step(n % 4)
    lnz = ctx.lnz()
    t1 = time.perf_counter()
    db, dh = ctx.backward()
    t2 = time.perf_counter()
    ob = ctx.observables()
    ctx.close()
    print(f"[bench] adjoint: forward {t1 - t0:.2f} s, reverse {t2 - t1:.2f} s", file=sys.stderr, flush=True)
    return {"steps": nsteps, "forward_s": round(t1 - t0, 3), "backward_s": round(t2 - t1, 3),
            "device_gb": round(ob["device_bytes"] / 1e9, 2), "lnz_per_site": lnz,
            "energy_per_site": -db, "dlnz_dh": dh}


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1",
                          "n_gpus": a.gpus}))
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    if a.copy_calibration:
        copy_calibration()
        return
    if a.adjoint:
        adjoint_run(a)
        return
    if a.precision_study:
        precision_study(a)
        return
    if a.table:
        table_run(a)
        return
    if a.tc:
        tc_run(a)
        return
    if a.jump:
        jump_run(a)
        return
    from paper_1906_06060_amd import hotrg as H
    prec = H.BF16X3 if a.precision == "bf16x3" else H.FP64
    imp = not a.no_impurities
    D = a.dcut
    ctx = H.Context(a.beta, a.h, D, precision=prec, impurities=imp, dense_only=a.dense)
    axis = 0
    t_setup = time.perf_counter()
    for _ in range(3):                      # ramp-up steps (dims grow to Dcut)
        ctx.step(axis % 4)
        axis += 1
    for _ in range(a.warmup):
        ctx.step(axis % 4)
        axis += 1
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t_setup
    dims, _ = ctx.dims()
    ctx.reset_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        ctx.step(axis % 4)
        axis += 1
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ob = ctx.observables()
    st = ctx.gemm_stats()
    ph = ctx.phase_stats()
    ctx.close()

    rows = (3 if imp else 1) * D ** 4
    # the method's count of the step (dense O(D^15) contraction, Sec. 2 cost
    # paragraph); the Z2 block form at h = 0 executes about a quarter of it
    step_flops = 2.0 * rows * D ** 4 * D ** 7
    sec = elapsed / a.steps
    tflops = step_flops / sec / 1e12
    exec_flops = st["flops"] / a.steps      # GEMM flops the engine launched per step
    block = bool(ob["block_sparse"])
    peak = PEAK_BF16 if prec == H.BF16X3 else PEAK_FP64
    issue = 3.0 if prec == H.BF16X3 else 1.0
    gemm_s = st["ms"] / 1e3
    achieved = st["flops"] / gemm_s if gemm_s > 0 else float("nan")
    traffic_key = ("z2" if block else "dense", D, imp, prec == H.BF16X3)
    line = {
        "metric": "HOTRG step time & TFLOP/s (% MFMA peak) at Dcut=10, mixed vs FP64",
        "value": round(tflops, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(sec * 1e3, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16x3" if prec == H.BF16X3 else "f64",
        "data": "synthetic",
        "config": {
            "workload": f"4D Ising HOTRG steady-state step, Dcut={D}, "
                        f"{'bf16x3' if prec == H.BF16X3 else 'fp64'} contraction, "
                        f"{'T+S_m+S_e rows' if imp else 'T rows'} (M={rows}, N={D ** 4}, K={D ** 7})",
            "beta": a.beta, "h": a.h, "dcut": D, "dims": list(dims),
            "contraction": ("Z2 block form (h = 0: two parity-class GEMMs per K slice)" if block else "dense"),
            "step_flops": step_flops,
            "flop_count": "value = step_flops / step time, step_flops = 2 M N K of the dense contraction "
                          "(the method's O(D^15) count); executed_flops_per_step = what the GEMMs ran",
            "executed_flops_per_step": exec_flops,
            "tflops_executed": round(exec_flops / sec / 1e12, 3),
            "pct_mfma_peak_issued": round(100 * issue * exec_flops / sec / peak, 2),
            "setup_s": round(setup_s, 2),
            "lnz_per_site": ob["lnz_per_site"], "nn_imp": ob["nn_imp"], "m_imp": ob["m_imp"], "X": ob["X"],
        },
        "roofline": {
            "bound": "mfma" if prec == H.BF16X3 else "alu",
            "kernel": "gemm_bf16x3_kernel" if prec == H.BF16X3 else "gemm_f64_kernel",
            "achieved": round(achieved / 1e12, 3),
            "peak": peak / 1e12,
            "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4),
            "issued_frac": round(issue * achieved / peak, 4),
            "traffic": (GEMM_TRAFFIC_BYTES.get(traffic_key) if gemm_source_sha() == GEMM_TRAFFIC_SRC_SHA
                        else None),
            "traffic_unit": "bytes per GEMM call (HBM, rocprofv3 FETCH_SIZE + WRITE_SIZE)",
            "launches": st["launches"],
            "avg_launch_ms": round(st["ms"] / max(st["launches"], 1), 3),
            "launch": (("one GEMM call per K slice covering both parity classes' products as one tile list: "
                        if block else "one GEMM call per K slice: ") +
                       "a main dispatch over whole rounds of tiles, a tail dispatch running the last partial "
                       "round as k-halves, and gemm_tail_fixup_kernel"
                       if prec == H.BF16X3 else
                       ("two gemm_f64_kernel dispatches per K slice (one per parity class)" if block
                        else "one gemm_f64_kernel dispatch per K slice")),
        },
    }
    n_ph = max(ph["steps"], 1)
    line["phases_ms_per_step"] = {
        "isometries": round(ph["isometries_ms"] / n_ph, 2),
        "contraction": round(ph["contraction_ms"] / n_ph, 2),
        "of_which_gemm": round(ph["gemm_ms"] / n_ph, 2),
        "operand_products": round((ph["contraction_ms"] - ph["gemm_ms"]) / n_ph, 2),
        "normalise_permute": round(ph["normalise_ms"] / n_ph, 2),
    }
    if prec == H.BF16X3 and not a.no_fp64:
        line["fp64"] = fp64_step(a, D, imp and not a.fp64_pure)
    if prec == H.BF16X3 and not a.no_adjoint:
        line["adjoint"] = adjoint_step(a, D)
    if not a.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(a.cpu_dcut, a.cpu_slices)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
