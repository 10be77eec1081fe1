"""Learned precision selector: training driver and installation.

The selector predicts, from 16 O(n^2) features of A, the number of
corrections the refinement needs with a BF16SPLIT, FP32 and FP64 factor
(label = corrections if the run converges, maxit + 10 otherwise; the network
output is log(1 + label)) and the
runtime picks the precision with the smallest predicted cost
fac_p + (y_p + 1) res + y_p sweep_p (cost model fitted to measured phase
times).  Labels come from the method itself: every training matrix is
solved with each precision, fallback off.  The network is trained on the GPU
by the library's own kernels (msqrt_mlp_grad, msqrt_mlp_adam).

    python -m paper_2607_12430_amd.selector --out selector.bin
"""

from __future__ import annotations

import argparse
import ctypes
import gzip
import json
import os
import struct
import time

import numpy as np
import torch

from . import _lib
from ._lib import check, lib

PRECS = ("bf16split", "fp32", "fp64")
NFEAT, NPARAM, NCOST = 16, 5443, 42
HID = 64
DEFAULT_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "selector.bin")
PHASES_FAC = ("validate", "select", "reduce", "eig", "back", "x0")
PHASES_SWEEP = ("transform", "solve", "update")


def _vp(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def features(a: torch.Tensor) -> torch.Tensor:
    """16 features of a device matrix (float64 or complex128) as a float tensor."""
    a = a.contiguous()
    f = torch.empty(NFEAT, dtype=torch.float32, device=a.device)
    dt = _lib.COMPLEX128 if a.is_complex() else _lib.REAL64
    n = a.shape[-1]
    check(lib().msqrt_features(dt, n, _vp(a), n, _vp(f), _stream()), "msqrt_features")
    return f


def mlp_forward(x: torch.Tensor, p: torch.Tensor) -> torch.Tensor:
    out = torch.empty((x.shape[0], 3), dtype=torch.float32, device=x.device)
    check(lib().msqrt_mlp_forward(x.shape[0], _vp(x), _vp(p), _vp(out), _stream()),
          "msqrt_mlp_forward")
    return out


def mlp_grad(x: torch.Tensor, y: torch.Tensor, p: torch.Tensor):
    g = torch.empty(NPARAM, dtype=torch.float32, device=x.device)
    loss = torch.empty(1, dtype=torch.float32, device=x.device)
    check(lib().msqrt_mlp_grad(x.shape[0], _vp(x), _vp(y), _vp(p), _vp(g), _vp(loss), _stream()),
          "msqrt_mlp_grad")
    return g, loss


def mlp_adam(g, p, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    check(lib().msqrt_mlp_adam(_vp(g), _vp(p), _vp(m), _vp(v), int(step), float(lr), float(beta1),
                               float(beta2), float(eps), _stream()), "msqrt_mlp_adam")


def init_params(seed: int = 0) -> np.ndarray:
    """He-normal weights, zero biases."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = [rng.standard_normal((HID, NFEAT)) * np.sqrt(2.0 / NFEAT), np.zeros(HID),
             rng.standard_normal((HID, HID)) * np.sqrt(2.0 / HID), np.zeros(HID),
             rng.standard_normal((3, HID)) * np.sqrt(1.0 / HID), np.zeros(3)]
    return np.concatenate([x.ravel() for x in parts]).astype(np.float32)


def train(x: np.ndarray, y: np.ndarray, epochs=400, lr=2e-3, batch=256, seed=0, log=None):
    """Adam on the mean squared error, minibatches drawn with a seeded shuffle.
    x is already normalised.  Returns (params, loss history per epoch)."""
    dev = torch.device("cuda")
    xd = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(dev)
    yd = torch.from_numpy(np.ascontiguousarray(y, dtype=np.float32)).to(dev)
    p = torch.from_numpy(init_params(seed)).to(dev)
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    hist = []
    step = 0
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(len(x))).to(dev)
        tot = 0.0
        for s in range(0, len(x), batch):
            idx = perm[s:s + batch]
            xb = xd.index_select(0, idx).contiguous()
            yb = yd.index_select(0, idx).contiguous()
            g, loss = mlp_grad(xb, yb, p)
            step += 1
            mlp_adam(g, p, m, v, step, lr)
            tot += float(loss) * len(idx)
        hist.append(tot / len(x))
        if log and (ep % 50 == 0 or ep == epochs - 1):
            log(f"epoch {ep} loss {hist[-1]:.4f}")
    return p.cpu().numpy(), hist


def save(path, params, mean, scale, cost):
    with open(path, "wb") as fh:
        fh.write(b"MSQSEL01")
        fh.write(struct.pack("<3i", NPARAM, NFEAT, NCOST))
        fh.write(np.asarray(params, "<f4").tobytes())
        fh.write(np.asarray(mean, "<f4").tobytes())
        fh.write(np.asarray(scale, "<f4").tobytes())
        fh.write(np.asarray(cost, "<f8").tobytes())


def read(path):
    raw = open(path, "rb").read()
    assert raw[:8] == b"MSQSEL01"
    np_, nf, nc = struct.unpack("<3i", raw[8:20])
    o = 20
    params = np.frombuffer(raw, "<f4", np_, o); o += 4 * np_
    mean = np.frombuffer(raw, "<f4", nf, o); o += 4 * nf
    scale = np.frombuffer(raw, "<f4", nf, o); o += 4 * nf
    cost = np.frombuffer(raw, "<f8", nc, o)
    return params, mean, scale, cost


def install(path: str = DEFAULT_FILE) -> bool:
    """Installs a selector file for MSQRT_PREC_AUTO; False if there is none."""
    if not os.path.exists(path):
        return False
    check(lib().msqrt_selector_load(path.encode()), "msqrt_selector_load")
    return True


def label(a: torch.Tensor, maxit=30, tol=1e-13):
    """Runs every precision with fallback off: corrections (or maxit + 10 on
    failure), status and phase times."""
    from . import sqrtm
    out = {}
    for p in PRECS:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info = sqrtm(a, prec=p, fallback=False, allow_fail=True, maxit=maxit, tol=tol)
        torch.cuda.synchronize()
        wall = 1e3 * (time.perf_counter() - t0)
        ok = info["status"] == "ok"
        out[p] = {"y": info["steps"] if ok else maxit + 10, "ok": ok, "steps": info["steps"],
                  "wall_ms": wall, "t_ms": info["t_ms"], "struct": info["struct_used"]}
    return out


def fit_cost(records):
    """Least-squares fit of ms = c3 n^3 + c2 n^2 + c0 for every structure and
    quantity (factorisation per precision, one correction per precision, one
    residual) from the phase timers of the labelling runs.  BF16SPLIT keeps
    the float factorisation, so its factorisation cost is fitted together
    with FP32's (one set of coefficients for both)."""
    cost = np.zeros(NCOST)
    for s, sname in enumerate(("hpd", "general")):
        for q in range(7):
            rows, rhs = [], []
            for r in records:
                n = r["n"]
                for p_i, p in enumerate(PRECS):
                    lab = r["labels"][p]
                    if lab["struct"] != sname:
                        continue
                    t = lab["t_ms"]
                    steps = lab["steps"]
                    if (q < 2 and p_i < 2) or (q == 2 and p_i == 2):
                        val = sum(t.get(k, 0.0) for k in PHASES_FAC)
                    elif 3 <= q < 6 and p_i == q - 3 and steps > 0:
                        val = sum(t.get(k, 0.0) for k in PHASES_SWEEP) / steps
                    elif q == 6 and p_i == 1:
                        val = t.get("residual", 0.0) / (steps + 1)
                    else:
                        continue
                    rows.append([n ** 3, n ** 2, 1.0])
                    rhs.append(val)
            if len(rows) >= 3:
                A = np.array(rows)
                sc = A.max(axis=0)
                c, *_ = np.linalg.lstsq(A / sc, np.array(rhs), rcond=None)
                cost[(7 * s + q) * 3:(7 * s + q) * 3 + 3] = c / sc
    return cost


def fit(records, epochs=400, oversample=10, seed=0, log=None):
    """Trains the network on labelled records: inputs are the normalised
    features, targets log(1 + y); records where some precision failed are
    repeated `oversample` times in the training split (failures are rare in
    the training law but decide the choice).  Returns (params, mean, scale,
    report) with the validation error on the held-out fifth."""
    dev = torch.device("cuda")
    x = np.array([r["features"] for r in records], dtype=np.float64)
    y = np.array([[r["labels"][p]["y"] for p in PRECS] for r in records], dtype=np.float64)
    failed = np.array([not all(r["labels"][p]["ok"] for p in PRECS) for r in records])
    mean = x.mean(axis=0)
    scale = x.std(axis=0)
    scale[scale < 1e-6] = 1.0
    xn = (x - mean) / scale
    rng = np.random.Generator(np.random.PCG64(5))
    perm = rng.permutation(len(x))
    nval = max(1, len(x) // 5)
    val, tr = perm[:nval], perm[nval:]
    tr_os = np.concatenate([tr] + [tr[failed[tr]]] * (oversample - 1))
    params, hist = train(xn[tr_os], np.log1p(y[tr_os]), epochs=epochs, seed=seed, log=log)
    pd = torch.from_numpy(params).to(dev)
    pred = np.expm1(mlp_forward(torch.from_numpy(xn[val].astype(np.float32)).to(dev),
                                pd).cpu().numpy())
    fail32 = y[val, 1] > 30
    caught = int(np.sum(fail32 & (pred[:, 1] > 20)))
    return params, mean, scale, {
        "train_loss_log1p": hist[-1], "val_mse_steps": float(np.mean((pred - y[val]) ** 2)),
        "n_train": int(len(tr)), "n_train_oversampled": int(len(tr_os)), "n_val": int(nval),
        "val_fp32_failures": int(fail32.sum()), "val_fp32_failures_predicted": caught}


def boundary_params(index: int):
    """Extra labelling law near the float factor's failure boundary at the
    evaluation sizes: (kind, n, kappa, seed).  Two thirds SPD with n
    log-uniform in [2048, 4096] and kappa = 10^U(6, 9); one third
    nonsymmetric (Q (L + N) Q^T) with n log-uniform in [512, 1024] and
    kappa = 10^U(3, 9)."""
    rng = np.random.Generator(np.random.PCG64(7_000_003 * (index + 1)))
    seed = int(rng.integers(1, 2 ** 31))
    if rng.uniform() < 2.0 / 3.0:
        n = int(round(np.exp(rng.uniform(np.log(2048.0), np.log(4096.0)))))
        return "spd", n, float(10.0 ** rng.uniform(6.0, 9.0)), seed
    n = int(round(np.exp(rng.uniform(np.log(512.0), np.log(1024.0)))))
    return "kappa", n, float(10.0 ** rng.uniform(3.0, 9.0)), seed


def evaluate(path, count=64, first=50_000, n=4096, kinds=("spd", "nonsym"), maxit=30,
             device_inputs=False, n_nonsym=None, log=True):
    """Selector gain on fresh matrices of the selector law (kind, kappa and
    seed of matrix `first + k`; SPD at order n, nonsymmetric at n_nonsym,
    default n; with kinds = ("spd",) every matrix is SPD): time of AUTO
    (selector + fallback) against always-BF16SPLIT / FP32 / FP64 (with
    fallback) and the per-matrix best; every AUTO answer is checked against
    the float64 residual bound."""
    import workloads as W
    from . import sqrtm
    install(path)
    dev = torch.device("cuda")
    # warm every code path once (allocations, first launches) before timing
    if device_inputs:
        import workloads.device as WD
        a0d = WD.spd(n, 1e3, 7, dev)
        a1d = WD.nonsym_shifted(n_nonsym or n, 7, dev)
    else:
        a0, _, _ = W.spd(n, 1e3, 7)
        a0d = torch.from_numpy(np.ascontiguousarray(a0)).to(dev)
        a1d = torch.from_numpy(np.ascontiguousarray(W.nonsym_shifted(n_nonsym or n, 7))).to(dev)
    for p in ("auto",) + PRECS:
        sqrtm(a0d, prec=p, fallback=True, allow_fail=True, maxit=maxit)
    if "nonsym" in kinds:
        for p in ("auto",) + PRECS:
            sqrtm(a1d, prec=p, fallback=True, allow_fail=True, maxit=maxit)
    torch.cuda.synchronize()
    rows = []
    for k in range(count):
        kind, _, kappa, seed = W.selector_params(first + k)
        if kind != "spd" and "nonsym" not in kinds:
            kind = "spd"
        elif kind == "spd" and "spd" not in kinds:
            kind = "kappa"
        nk = n if kind == "spd" or not n_nonsym else n_nonsym
        if device_inputs:
            import workloads.device as WD
            ad = {"spd": lambda: WD.spd(nk, kappa, seed, dev),
                  "shifted": lambda: WD.nonsym_shifted(nk, seed, dev),
                  "kappa": lambda: WD.nonsym_kappa(nk, kappa, seed, dev)}[kind]()
        else:
            if kind == "spd":
                a, _, _ = W.spd(nk, kappa, seed)
            elif kind == "shifted":
                a = W.nonsym_shifted(nk, seed)
            else:
                a = W.nonsym_kappa(nk, kappa, seed)
            ad = torch.from_numpy(np.ascontiguousarray(a)).to(dev)
        row = {"kappa": kappa, "kind": kind, "n": nk}
        for p in ("auto",) + PRECS:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x, info = sqrtm(ad, prec=p, fallback=True, allow_fail=True, maxit=maxit)
            torch.cuda.synchronize()
            row[p] = 1e3 * (time.perf_counter() - t0)
            row[p + "_escalations"] = info["fallbacks"]
            if p == "auto":
                rr = float(torch.linalg.matrix_norm(x @ x - ad) / torch.linalg.matrix_norm(ad))
                row["auto_ok"] = info["status"] == "ok" and rr <= 1e-13
                row["auto_prec"] = info["prec_used"]
                row["predicted"] = info["predicted_steps"]
        rows.append(row)
        if log:
            print(f"[selector-eval] {k + 1}/{count} {kind} n={nk} kappa={kappa:.1e} "
                  f"auto={row['auto_prec']} t_auto={row['auto']:.1f} t_fp32={row['fp32']:.1f} "
                  f"t_fp64={row['fp64']:.1f}", flush=True)
    out = {"count": count, "n": n, "n_nonsym": n_nonsym, "kinds": list(kinds),
           "auto_all_ok": all(r["auto_ok"] for r in rows), "rows": rows}
    groups = {"spd": ("spd",), "nonsym": ("shifted", "kappa"), "all": ("spd", "shifted", "kappa")}
    for g, members in groups.items():
        rs = [r for r in rows if r["kind"] in members]
        if not rs:
            continue
        out[g] = {
            "count": len(rs),
            "total_ms": {p: sum(r[p] for r in rs) for p in ("auto",) + PRECS},
            "per_matrix_best_ms": sum(min(r[p] for p in PRECS) for r in rs),
            "auto_choices": {p: sum(r["auto_prec"] == p for r in rs) for p in PRECS},
            "escalations": {p: sum(r[p + "_escalations"] for r in rs) for p in ("auto",) + PRECS}}
    return out


def main(argv=None):
    import workloads as W

    ap = argparse.ArgumentParser()
    ap.add_argument("--evaluate", action="store_true", help="measure the gain of --out instead")
    ap.add_argument("--eval-n", type=int, default=4096)
    ap.add_argument("--eval-kinds", default="spd,nonsym")
    ap.add_argument("--eval-n-nonsym", type=int, default=None,
                    help="order of the nonsymmetric evaluation matrices (default: --eval-n)")
    ap.add_argument("--only-kinds", default=None,
                    help="label only the indices of these kinds of the selector law "
                         "(comma-separated: spd, shifted, kappa)")
    ap.add_argument("--boundary", action="store_true",
                    help="label matrices of the boundary law (boundary_params) instead of the "
                         "selector law")
    ap.add_argument("--eval-first", type=int, default=50_000,
                    help="first evaluation index (disjoint from the training indices)")
    ap.add_argument("--count", type=int, default=1200, help="training (or evaluation) matrices")
    ap.add_argument("--first", type=int, default=10_000, help="first dataset index")
    ap.add_argument("--n-max-nonsym", type=int, default=320)
    ap.add_argument("--epochs", type=int, default=400)
    ap.add_argument("--out", default=DEFAULT_FILE)
    ap.add_argument("--records", default=None, help="write the labelled records (JSON)")
    ap.add_argument("--from-records", default=None,
                    help="train from previously labelled records (comma-separated files) "
                         "instead of labelling")
    ap.add_argument("--device-inputs", action="store_true",
                    help="generate the matrices on the device (same laws, torch generator)")
    ap.add_argument("--label-only", action="store_true",
                    help="label and write --records without training")
    ap.add_argument("--refit-cost", default=None, metavar="SELECTOR",
                    help="keep the network of this selector file and refit only its cost "
                         "model from --count freshly timed matrices (after kernel changes)")
    args = ap.parse_args(argv)
    if args.evaluate:
        res = evaluate(args.out, count=args.count, n=args.eval_n,
                       kinds=tuple(args.eval_kinds.split(",")), first=args.eval_first,
                       device_inputs=args.device_inputs, n_nonsym=args.eval_n_nonsym)
        if args.records:
            with open(args.records, "w") as fh:
                json.dump(res, fh)
        print(json.dumps({k: v for k, v in res.items() if k != "rows"}), flush=True)
        return
    dev = torch.device("cuda")
    records = []
    feats = []
    t0 = time.time()
    if args.from_records:
        # a later file replaces the records of the same index (relabelling)
        byidx = {}
        for fname in args.from_records.split(","):
            with (gzip.open(fname, "rt") if fname.endswith(".gz") else open(fname)) as fh:
                for r in json.load(fh):
                    byidx[(r.get("law", "selector"), r["index"])] = r
        records = list(byidx.values())
    only = set(args.only_kinds.split(",")) if args.only_kinds else None
    for k in range(0 if args.from_records else args.count):
        if only is not None and W.selector_params(args.first + k, args.n_max_nonsym)[0] not in only:
            continue
        if args.boundary:
            import workloads.device as WD
            kind, n, kappa, seed = boundary_params(args.first + k)
            ad = (WD.spd(n, kappa, seed, dev) if kind == "spd"
                  else WD.nonsym_kappa(n, kappa, seed, dev))
        elif args.device_inputs:
            import workloads.device as WD
            ad, kind, n, kappa = WD.selector_matrix(args.first + k, args.n_max_nonsym, dev)
        else:
            a, kind, n, kappa = W.selector_matrix(args.first + k, args.n_max_nonsym)
            ad = torch.from_numpy(np.ascontiguousarray(a)).to(dev)
        f = features(ad).cpu().numpy()
        labs = label(ad)
        records.append({"index": args.first + k, "law": "boundary" if args.boundary else "selector",
                        "kind": kind, "n": n, "kappa": kappa, "features": f.tolist(),
                        "labels": labs})
        feats.append(f)
        if k % 50 == 0:
            print(f"[selector] labelled {k + 1}/{args.count} ({time.time() - t0:.0f} s)", flush=True)
    if args.refit_cost:
        params, mean, scale, _ = read(args.refit_cost)
        # the first solves of a process include one-time module loading
        cost = fit_cost(records[20:] if len(records) > 40 else records)
        save(args.out, params, mean, scale, cost)
        print(json.dumps({"refit_cost_from": len(records), "out": args.out}), flush=True)
        return
    if args.label_only:
        with (gzip.open(args.records, "wt") if args.records.endswith(".gz")
              else open(args.records, "w")) as fh:
            json.dump(records, fh)
        print(json.dumps({"labelled": len(records), "records": args.records}), flush=True)
        return
    params, mean, scale, report = fit(records, epochs=args.epochs,
                                      log=lambda s: print("[selector] " + s, flush=True))
    cost = fit_cost(records)
    save(args.out, params, mean.astype(np.float32), scale.astype(np.float32), cost)
    report["out"] = args.out
    print(json.dumps(report), flush=True)
    if args.records:
        with open(args.records, "w") as fh:
            json.dump(records, fh)


if __name__ == "__main__":
    main()
