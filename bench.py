"""Benchmark: principal square roots per second of a real SPD matrix, n=4096,
kappa=1e4, with the mixed-precision method (float32 spectral decomposition +
float64 approximate-Newton refinement, Alg. 3) beside the plain float64 Schur
method on the same GPU.  Every timed call is a complete msqrt_sqrtm (factor,
X_0, refinement, final residual check to 1e-13) with A already in HBM.

Prints one JSON line (see the measurement section of the design doc).
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

PEAK = {"gemm_f32": (157.3, "TFLOP/s"), "gemm_f64": (78.6, "TFLOP/s")}
HBM_PEAK_GBS = 8000.0


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--workload", default="spd",
                   choices=["spd", "nonsym", "complex_square", "table1"],
                   help="spd (default, the benchmark line); nonsym = real nonsymmetric "
                        "A = 2I + G/sqrt(n) (n=2048, seed 5); complex_square = complex A = B^2 "
                        "(seed 6): general path, mixed vs FP64 factor, no roofline; table1 = the "
                        "paper's test sets I-VII (Table 1): relative time of the mixed solve to "
                        "the FP64 Schur solve, nullified-stop accuracy traces, Hilbert threshold")
    p.add_argument("--sets", default="I,II,III,IV,V,VI,VII", help="table1: sets to run")
    p.add_argument("--trace", type=int, default=8, help="table1: corrections traced per set")
    p.add_argument("--steps", type=int, default=None)
    p.add_argument("--warmup", type=int, default=None)
    p.add_argument("--n", type=int, default=None)
    p.add_argument("--kappa", type=float, default=1e4)
    p.add_argument("--seed", type=int, default=3)
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--no-fp64", action="store_true", help="skip the fixed-FP64 comparator")
    p.add_argument("--cpu-n", type=int, default=None,
                   help="order of the CPU oracle sample (default: the benchmark's n)")
    p.add_argument("--copy-probe", action="store_true",
                   help="run one 512 MiB device copy first (reference kernel for HBM counters)")
    args = p.parse_args()
    spd = args.workload == "spd"
    if args.steps is None:
        args.steps = 10 if spd else (3 if args.workload == "table1" else 2)
    if args.warmup is None:
        args.warmup = 3 if spd else 1
    if args.n is None:
        args.n = {"spd": 4096, "nonsym": 2048, "complex_square": 4096, "table1": 0}[args.workload]
    return args


def time_solves(msq, torch, a, prec, steps, warmup):
    x = torch.empty_like(a)
    info = None
    for _ in range(warmup):
        _, info = msq.sqrtm(a, prec=prec, tol=1e-13, fallback=False, out=x)
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for _ in range(steps):
        _, info = msq.sqrtm(a, prec=prec, tol=1e-13, fallback=False, out=x)
        infos.append(info)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return (t1 - t0), x, infos


def time_solves_opts(msq, torch, a, prec, steps, warmup):
    """Like time_solves, with the library's precision escalation on."""
    x = torch.empty_like(a)
    for _ in range(warmup):
        msq.sqrtm(a, prec=prec, tol=1e-13, out=x)
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for _ in range(steps):
        _, info = msq.sqrtm(a, prec=prec, tol=1e-13, out=x)
        infos.append(info)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, x, infos


def recorded_traffic(kernel_class, workload):
    """HBM bytes per launch from a committed counter summary under profiles/,
    valid only while the kernel's source file is unchanged (sha256)."""
    import glob
    import hashlib
    for path in glob.glob(os.path.join(ROOT, "profiles", "*.md")):
        for line in open(path):
            if not line.startswith("traffic-record:"):
                continue
            rec = json.loads(line.split(":", 1)[1])
            if rec.get("kernel") != kernel_class or rec.get("workload") != workload:
                continue
            src = os.path.join(ROOT, rec["source"])
            if not os.path.exists(src):
                return None
            if hashlib.sha256(open(src, "rb").read()).hexdigest() != rec["source_sha256"]:
                return None
            return rec["traffic_bytes_per_launch"]
    return None


def gpu_relres(torch, x, a):
    r = torch.linalg.matrix_norm(x @ x - a) / torch.linalg.matrix_norm(a)
    return float(r)


def host_cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(n_cpu, n, kappa, seed):
    """The float64 oracle (Alg. 3 route: Householder tridiagonalisation +
    implicit QL, X = Q diag(lam^1/2) Q^T) on all host cores, one solve of the
    benchmark's own matrix (n_cpu = n) or of a same-law matrix of order
    n_cpu scaled by (n / n_cpu)^3."""
    import oracle
    import workloads as W
    a, _, _ = W.spd(n_cpu, kappa, seed)
    threads = oracle.lib().orc_get_threads()
    t0 = time.perf_counter()
    oracle.sqrtm_spd(a)
    dt = time.perf_counter() - t0
    scale = (n / n_cpu) ** 3
    what = (f"one solve of the benchmark matrix (n={n}, kappa={kappa:g}, seed {seed}), {dt:.2f} s"
            if n_cpu == n else
            f"one solve at n={n_cpu}, kappa={kappa:g}, {dt:.2f} s, scaled by (n/{n_cpu})^3 to n={n}")
    return {
        "value": 1.0 / (dt * scale),
        "unit": "solves/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"oracle float64 SPD route (Householder tridiagonalisation + implicit QL, "
                   f"X = Q diag(lam^1/2) Q^T, OpenMP), {what}; host: {host_cpu_model()}, "
                   f"{os.cpu_count()} logical CPUs visible"),
    }


def spd_flops(n, sweeps):
    """Algorithmic flops of one mixed SPD solve with `sweeps` corrections
    (symmetry exploited): float32 factorisation 4/3 n^3 (tridiagonalisation)
    + 4/3 n^3 (eigensolver merges, upper bound) + 2 n^3 (back-transform),
    X_0 n^3, per correction 6 n^3 (W = R Q, Q^T W upper half, V = Q Y,
    V Q^T upper half); float64 residuals n^3 each, sweeps + 1 of them."""
    n3 = float(n) ** 3
    return {"fp32": (17.0 / 3.0 + 6.0 * sweeps) * n3, "fp64": (sweeps + 1.0) * n3}


def run_general(args):
    """General path (Alg. 2): mixed (FP32 / complex64 Schur factor) against the
    FP64 factor on the same GPU, both refined to relres <= 1e-13."""
    import numpy as np
    import torch

    import paper_2607_12430_amd as msq
    import workloads as W

    n = args.n
    if args.workload == "nonsym":
        a_h = W.nonsym_shifted(n, 5)
        workload = f"nonsym_shifted_n{n}"
    else:
        a_h, _ = W.complex_square(n, 6)
        workload = f"complex_square_n{n}"
    a = torch.from_numpy(np.ascontiguousarray(a_h)).cuda()
    del a_h
    torch.cuda.synchronize()
    dt, x, infos = time_solves(msq, torch, a, "fp32", args.steps, args.warmup)
    rr = gpu_relres(torch, x, a)
    res = {"solves_per_s": args.steps / dt, "ms_per_solve": 1e3 * dt / args.steps}
    fp64 = None
    if not args.no_fp64:
        dt64, x64, infos64 = time_solves(msq, torch, a, "fp64", args.steps, args.warmup)
        fp64 = {"solves_per_s": args.steps / dt64, "ms_per_solve": 1e3 * dt64 / args.steps,
                "relres": gpu_relres(torch, x64, a), "steps": infos64[-1]["steps"],
                "phases_ms": {k: round(v, 3) for k, v in infos64[-1]["t_ms"].items()}}
    out = {
        "metric": "sqrtm solves/s, general path, mixed vs FP64 Schur, relres<=1e-13",
        "value": round(res["solves_per_s"], 5),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(res["ms_per_solve"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "complex64 factor+transforms, complex128 residual+update",
        "data": "synthetic",
        "config": {"workload": workload, "n": n, "tol": 1e-13},
        "relres": rr,
        "refinement_steps": infos[-1]["steps"],
        "phases_ms": {k: round(v, 3) for k, v in infos[-1]["t_ms"].items()},
        "fp64_schur": fp64,
        "speedup_vs_fp64": (round(res["solves_per_s"] / fp64["solves_per_s"], 4) if fp64 else None),
        "roofline": None,
        "dominant_phase": "eig (multishift QR: serial bulge chains, latency-bound)",
        "cpu_baseline": None,
    }
    print(json.dumps(out))


def run_table1(args):
    """The paper's Table 1 test sets on one GPU (Sec. 5): for each set the
    mixed-precision solve (FP32 factor) and the fixed FP64 Schur solve on the
    same GPU (median of `steps` timed solves each, relative execution time as
    in Sec. 5.2), and the accuracy trace of Sec. 5.1: the stopping test
    nullified, relative residual and relative error after every correction,
    the FP64 solve's output taken as the ground truth (as the paper does).
    Then the Hilbert threshold: H_1024 + tau I with the FP32 factor and no
    escalation, over a range of tau."""
    import numpy as np
    import torch

    import paper_2607_12430_amd as msq
    import workloads as W

    def med_time(a, prec):
        ts = []
        x = None
        for i in range(args.warmup + args.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x, info = msq.sqrtm(a, prec=prec, tol=1e-13, fallback=False)
            torch.cuda.synchronize()
            if i >= args.warmup:
                ts.append(time.perf_counter() - t0)
        return float(np.median(ts)), x, info

    def rel(u, v):
        return float(torch.linalg.matrix_norm(u - v) / torch.linalg.matrix_norm(v))

    sets = []
    for sid in [x for x in args.sets.split(",") if x]:
        a_h, shift = W.table1(sid, 1000 + len(sets))
        a = torch.from_numpy(np.ascontiguousarray(a_h)).cuda()
        n = a_h.shape[0]
        del a_h
        t32, x32, i32 = med_time(a, "fp32")
        t64, x64, i64 = med_time(a, "fp64")
        # nullified-stop trace with the FP32 factor
        f = msq.factor(a, prec="fp32")
        x = torch.zeros_like(a)
        info = msq.refine(f, a, x, init_from_factor=True, maxit=0, tol=-1.0)
        trace = [{"k": 0, "relres": info["relres"], "relerr": rel(x, x64)}]
        for k in range(1, args.trace + (8 if sid == "VII" else 0) + 1):
            info = msq.refine(f, a, x, init_from_factor=False, maxit=1, tol=-1.0)
            trace.append({"k": k, "relres": info["relres"], "relerr": rel(x, x64)})
        f.close()
        rec = {"set": sid, "n": n, "shift": round(shift, 6), "struct": i32["struct_used"],
               "mixed_ms": round(1e3 * t32, 2), "fp64_ms": round(1e3 * t64, 2),
               "relative_time": round(t32 / t64, 4), "speedup": round(t64 / t32, 3),
               "mixed_steps": i32["steps"], "mixed_relres": i32["relres"],
               "fp64_relres": i64["relres"], "mixed_relerr_vs_fp64": rel(x32, x64),
               "mixed_phases_ms": {k: round(v, 2) for k, v in i32["t_ms"].items()},
               "trace": trace}
        print(json.dumps({"table1_set": rec}), flush=True)
        sets.append(rec)
        del a, x, x32, x64
        torch.cuda.empty_cache()
    hil = []
    for tau in (1e-6, 6e-7, 4e-7, 3e-7, 2.8e-7, 2.5e-7, 2e-7, 1.5e-7, 1e-7, 1e-8):
        a = torch.from_numpy(np.ascontiguousarray(W.hilbert(1024, tau))).cuda()
        _, info = msq.sqrtm(a, prec="fp32", tol=1e-12, fallback=False, allow_fail=True)
        hil.append({"tau": tau, "status": info["status"], "corrections": info["steps"],
                    "relres": info["relres"]})
    out = {"metric": "relative execution time mixed / FP64 Schur, Table 1 sets (Sec. 5)",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "data": "synthetic",
           "config": {"workload": "table1", "sets": [r["set"] for r in sets]},
           "sets": [{k: v for k, v in r.items() if k != "trace"} for r in sets],
           "hilbert_threshold_fp32_tol1e-12": hil}
    print(json.dumps(out))


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "single-GPU benchmark: --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.workload == "table1":
        run_table1(args)
        return
    if args.workload != "spd":
        run_general(args)
        return
    import numpy as np
    import torch

    import paper_2607_12430_amd as msq
    from paper_2607_12430_amd import _lib
    import workloads as W

    n, kappa = args.n, args.kappa
    a_h, _, _ = W.spd(n, kappa, args.seed)
    a = torch.from_numpy(np.ascontiguousarray(a_h)).cuda()
    torch.cuda.synchronize()

    if args.copy_probe:
        src = torch.empty(64 * 1024 * 1024, dtype=torch.float64, device="cuda")
        src.fill_(1.0)
        dst = src.clone()
        torch.cuda.synchronize()
        del src, dst

    # ---- mixed precision: timed region without per-launch instrumentation
    for _ in range(args.warmup):
        msq.sqrtm(a, prec="fp32", tol=1e-13, fallback=False)
    torch.cuda.synchronize()
    dt_mixed, x, infos = time_solves(msq, torch, a, "fp32", args.steps, 0)
    rr_mixed = gpu_relres(torch, x, a)
    steps_mixed = infos[-1]["steps"]
    phases = infos[-1]["t_ms"]

    # ---- the same solves again with HIP events around every kernel launch
    # (on the launch stream): per-class time, flops and bytes
    _lib.profile_enable(True)
    dt_instr, _, _ = time_solves(msq, torch, a, "fp32", args.steps, 0)
    stats = _lib.profile_stats()
    _lib.profile_enable(False)

    # ---- fixed FP64 Schur method on the same GPU
    fp64 = None
    if not args.no_fp64:
        dt64, x64, infos64 = time_solves(msq, torch, a, "fp64", args.steps, args.warmup)
        fp64 = {"solves_per_s": args.steps / dt64, "ms_per_solve": 1e3 * dt64 / args.steps,
                "relres": gpu_relres(torch, x64, a), "steps": infos64[-1]["steps"],
                "phases_ms": {k: round(v, 3) for k, v in infos64[-1]["t_ms"].items()}}

    # ---- the BF16-split transforms (same float factor; the Schur-basis
    # products as three bf16 products with float accumulation)
    dts, xs, infs = time_solves(msq, torch, a, "bf16split", args.steps, args.warmup)
    bf16split = {"solves_per_s": args.steps / dts, "ms_per_solve": 1e3 * dts / args.steps,
                 "relres": gpu_relres(torch, xs, a), "steps": infs[-1]["steps"],
                 "phases_ms": {k: round(v, 3) for k, v in infs[-1]["t_ms"].items()}}

    # ---- learned precision selector (AUTO, fallback on)
    dta, xa, infa = time_solves_opts(msq, torch, a, "auto", args.steps, args.warmup)
    auto = {"solves_per_s": args.steps / dta, "ms_per_solve": 1e3 * dta / args.steps,
            "relres": gpu_relres(torch, xa, a), "prec_used": infa[-1]["prec_used"],
            "steps": infa[-1]["steps"], "fallbacks": infa[-1]["fallbacks"],
            "predicted_steps": [round(v, 2) for v in infa[-1]["predicted_steps"]]}

    # ---- roofline of the dominant kernel class
    classes = {}
    for k, v in stats.items():
        base = k.split(":")[0]
        c = classes.setdefault(base, {"launches": 0, "ms": 0.0, "flops": 0.0, "bytes": 0.0})
        for f in c:
            c[f] += v[f]
    cls, st = max(classes.items(), key=lambda kv: kv[1]["ms"])
    if cls.startswith("gemm"):
        peak, unit = PEAK[cls]
        achieved = st["flops"] / (st["ms"] * 1e-3) / 1e12
        bound = "mfma"
    else:
        peak, unit = HBM_PEAK_GBS, "GB/s"
        achieved = st["bytes"] / (st["ms"] * 1e-3) / 1e9
        bound = "hbm"
    workload = f"spd_n{n}_kappa{kappa:g}"
    roof = {"bound": bound, "kernel": cls, "achieved": round(achieved, 3), "peak": peak,
            "unit": unit, "frac": round(achieved / peak, 4),
            "traffic": recorded_traffic(cls, workload),
            "launches_per_solve": st["launches"] / args.steps,
            "avg_launch_ms": round(st["ms"] / st["launches"], 5),
            "timing": "HIP events around each launch on its stream, in a repeat of the timed solves"}
    kernel_ms = {k: round(v["ms"] / args.steps, 3) for k, v in classes.items()}
    gemm_tflops = {k: {"tflops": round(v["flops"] / (v["ms"] * 1e-3) / 1e12, 2),
                       "frac_peak": round(v["flops"] / (v["ms"] * 1e-3) / 1e12 /
                                          PEAK[k.split(":")[0]][0], 4),
                       "us_per_launch": round(1e3 * v["ms"] / v["launches"], 1)}
                   for k, v in sorted(stats.items()) if k.split(":")[0] in PEAK}

    # ---- the refinement GEMMs together: per correction W = R Q and V = Q Y
    # (2 n^3 each) and the two symmetric-output products Q^T W and V Q^T
    # (n^2 (n + 1) each), over the transform and update phases of the last
    # timed solve (launch gaps included)
    rg_flops = float(steps_mixed) * (4.0 * n ** 3 + 2.0 * n * n * (n + 1.0))
    rg_ms = phases.get("transform", 0.0) + phases.get("update", 0.0)
    refinement_gemms = None
    if rg_flops > 0 and rg_ms > 0:
        rg_tf = rg_flops / (rg_ms * 1e-3) / 1e12
        refinement_gemms = {"tflops": round(rg_tf, 2), "frac_peak": round(rg_tf / PEAK["gemm_f32"][0], 4),
                            "ms": round(rg_ms, 3), "flops": rg_flops, "corrections": steps_mixed}

    # ---- whole solve against the FP32 / FP64 matrix peaks
    fl = spd_flops(n, steps_mixed)
    t = dt_mixed / args.steps
    solve_rate = {
        "fp32_tflops": round(fl["fp32"] / t / 1e12, 2),
        "fp64_tflops": round(fl["fp64"] / t / 1e12, 2),
        # time the algorithmic flops would take at the two matrix peaks,
        # as a fraction of the measured time
        "matrix_peak_frac": round((fl["fp32"] / (PEAK["gemm_f32"][0] * 1e12) +
                                   fl["fp64"] / (PEAK["gemm_f64"][0] * 1e12)) / t, 4),
        "flops": fl,
    }

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(args.cpu_n or n, n, kappa, args.seed)

    value = args.steps / dt_mixed
    out = {
        "metric": "sqrtm solves/s at n=4096, mixed vs FP64 Schur, relres<=1e-13; % matrix peak",
        "value": round(value, 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * dt_mixed / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 factor+transforms, f64 residual+update",
        "data": "synthetic",
        "config": {"workload": workload, "n": n, "kappa": kappa,
                   "seed": args.seed, "tol": 1e-13, "eigs": "log-uniform, endpoints pinned"},
        "relres": rr_mixed,
        "refinement_steps": steps_mixed,
        "phases_ms": {k: round(v, 3) for k, v in phases.items()},
        "solve_rate": solve_rate,
        "kernel_ms_per_solve": kernel_ms,
        "instrumented_ms_per_step": round(1e3 * dt_instr / args.steps, 3),
        "gemm_tflops": gemm_tflops,
        "refinement_gemms": refinement_gemms,
        "fp64_schur": fp64,
        "speedup_vs_fp64": (round(value / fp64["solves_per_s"], 4) if fp64 else None),
        "bf16split": bf16split,
        "auto": auto,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
