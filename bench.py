"""Benchmark: end-to-end EDA solves on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-extra]

Workload (the largest configuration that fits one GPU): d = 65536 (256 x 256
images), k = 100 classes x n_j = 20 samples (n = 2000), t = 99 dominant
eigenpairs, block width 8, tol 1e-6 (per-pair floors u lam_1 / lam_i),
float64 throughout.  Synthetic samples (unit-norm columns, 512-dim class
signal, 5% noise) stand in for face images, which are not available.

One step = the whole hot path on one batch of samples already resident in
HBM: scatter factors -> factor ingest + Gram + small eigensolves + cores ->
block Lanczos with Rayleigh-Ritz -> back-transform + orthonormalisation.
`value` is solves per second over the timed steps.

`roofline` covers the exp-op, the block product e^{-s} M V (b = 8) with two
streaming passes over P = [H_W H_B] (d x 2100 float64, 1.1 GB, far larger
than the 256 MB Infinity Cache): its algorithmic bytes 2 d N 8 + 3 d b 8 per
product divided by its average duration, measured with HIP events on the
library's stream around every product inside the timed solves (P^T V on the
matrix cores, the chunk sum, the core product and its column-group sum,
alpha V + P Z).  Peak: MI355X HBM3E, 8 TB/s.  `traffic` is the
counter-measured HBM bytes per product from the committed rocprofv3 summary
(while the streaming kernels are unchanged since it was taken).

`cpu_baseline` times the FP64 CPU oracle (exact (n+k)-dimensional reduction
of the pencil, NumPy/SciPy) on one full solve of the same workload with all
host threads; `cpu_baseline_1thread` the same with one thread.

Extras (--no-extra skips them): the C5 step with FP8 storage + float32 basis
+ float64 refinement against the float64 step (preparation included); the
d = 32256 workload in float64, bfloat16 and FP8 storage; the ORL-shaped
d = 10304 workload (its 19.8 MB factor sits in the Infinity Cache, so its
"HBM" bandwidth is effective cache bandwidth); the Lanczos form, Arnoldi
form and direct solve side by side; the Section 3.3 tolerance sweep; the
64-problem batch against the float64 and float32 one-by-one loops.

`--profile-op K [--workload C5|C2]`: only K exponential products (b = 8)
plus one 1 GiB copy, for hardware-counter runs.
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

METRIC = "exp(S)·V HBM GB/s vs peak; EDA solves/s mixed vs FP64 at residual 1e-6"
HBM_PEAK_GBPS = 8000.0


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(p, threads=None) -> dict:
    """One full solve by the oracle's exact reduction (scatter factors,
    Householder QR of [H_W H_B], dense pencil eigenproblem) with `threads`
    BLAS threads (None: all the host offers)."""
    import oracle
    from threadpoolctl import threadpool_info, threadpool_limits
    with threadpool_limits(threads):
        used = max((i.get("num_threads", 1) for i in threadpool_info()), default=1)
        t0 = time.perf_counter()
        H_W, H_B = oracle.scatter_factors(p.X, p.counts)
        oracle.eda_reduced(H_W, H_B, p.t)
        el = time.perf_counter() - t0
    return {"value": 1.0 / el, "unit": "solves/s", "cores": int(used), "kind": "oracle",
            "sample": f"1 full solve of the same workload by the oracle's exact (n+k)-dim "
                      f"reduction (scatter factors, Householder QR of [H_W H_B], dense pencil "
                      f"eig), {el:.1f} s",
            "cpu_model": _cpu_model(), "host_cpus": os.cpu_count()}


def counter_traffic():
    """HBM bytes per product from the committed counter summary, or None when
    the streaming kernels have changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "exp_op_c5_counters.md")
    src = os.path.join(ROOT, "paper_1512_06500_amd", "csrc", "k_tsmm.hip")
    try:
        fields = dict(line.split(": ", 1) for line in open(path).read().splitlines()
                      if line.startswith(("traffic_bytes_per_op: ", "kernel_source_sha256: ")))
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    if fields.get("kernel_source_sha256", "").strip() != sha:
        return None
    return float(fields["traffic_bytes_per_op"])


def profile_op(torch, eda, h, Xd, counts, reps):
    """K products e^{-s} M V (b = 8) and one 1 GiB device copy."""
    H_W, H_B = h.scatter_factors(Xd, counts)
    h.prepare(H_W, H_B)
    V = torch.randn(8, Xd.shape[0], dtype=torch.float64, device="cuda").t()
    out = torch.empty_like(V.t()).t()
    for _ in range(reps):
        h.opmv("M", V, out=out)
    src = torch.ones(128 << 20, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"profile_op": reps, "copy_bytes": 2 * src.numel() * 8}), flush=True)


def _upload(torch, X):
    return torch.from_numpy(np.ascontiguousarray(X.T)).cuda().t()


def mixed_vs_f64(torch, eda, reps: int = 3) -> dict:
    import datagen
    from tests.golden.reader import read as read_golden
    p = datagen.config("C3")
    g = read_golden("C3")
    Xd = _upload(torch, p.X)
    h = eda.Handle()
    H_W, H_B = h.scatter_factors(Xd, p.counts.tolist())
    out = {"workload": f"d={p.d}, k={p.k} x n_j={p.n // p.k} (n={p.n}), t={p.t}, "
                       f"block 8, tol {p.tol:g}"}
    for tag, storage, basis in (("f64", "f64", "f64"), ("mixed", "bf16", "f32"),
                                ("fp8", "fp8", "f32")):
        def one():
            h.prepare(H_W, H_B, storage=storage)
            return h.solve(p.t, p.tol, block=8, seed=p.seed, krylov_dtype=basis)
        one()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            r = one()
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / reps
        lam_err = np.abs(np.array(r.ritz) - g["lam"]) / g["lam"]
        out[tag] = {"solves_per_s": 1.0 / el, "ms": 1e3 * el, "status": r.status,
                    "storage": storage, "basis": basis, "iters": r.info["iters"],
                    "refine_passes": r.info["refine_passes"],
                    "krylov_ms": r.info["t_krylov_ms"], "refine_ms": r.info["t_refine_ms"],
                    "resid_max": max(r.resid),
                    "lam_rel_err_top": float(lam_err[0]),
                    "lam_rel_err_max_over_floor": float(np.max(lam_err / np.maximum(
                        1e-6, g["pair_floor"])))}
    out["ratio_mixed_over_f64"] = out["mixed"]["solves_per_s"] / out["f64"]["solves_per_s"]
    out["ratio_fp8_over_f64"] = out["fp8"]["solves_per_s"] / out["f64"]["solves_per_s"]
    h.close()
    return out


def large_fp8_vs_f64(torch, eda, p, Xd, reps: int = 3) -> dict:
    """The headline step (scatter -> prepare -> solve at d = 65536, n = 2000,
    k = 100, t = 99, tol 1e-6) with FP8 E4M3 storage, a float32 Krylov basis
    and float64 refinement, against the float64 step; preparation included.
    Also the exponential product's bandwidth for each storage type (its
    algorithmic bytes over the event-timed products inside the solves)."""
    from tests.golden.reader import read as read_golden
    g = read_golden("C5")
    h = eda.Handle()
    counts = p.counts.tolist()
    out = {"workload": f"d={p.d}, k={p.k} x n_j={p.n // p.k} (n={p.n}), t={p.t}, block 8, "
                       f"tol {p.tol:g}, prepare + solve"}
    for tag, storage, basis in (("f64", "f64", "f64"), ("fp8", "fp8", "f32")):
        def one():
            H_W, H_B = h.scatter_factors(Xd, counts)
            h.prepare(H_W, H_B, storage=storage)
            return h.solve(p.t, p.tol, block=8, seed=p.seed, krylov_dtype=basis)
        one()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = []
        for _ in range(reps):
            r = one()
            infos.append(r.info)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / reps
        lam_err = np.abs(np.array(r.ritz) - g["lam"]) / np.array(g["lam"])
        op_calls = sum(i["op_calls"] for i in infos)
        op_s = sum(i["t_op_ms"] for i in infos) / max(op_calls, 1) / 1e3
        op_bytes = infos[-1]["op_bytes"]
        out[tag] = {"solves_per_s": 1.0 / el, "ms": 1e3 * el, "status": r.status,
                    "storage": storage, "basis": basis, "iters": r.info["iters"],
                    "refine_passes": r.info["refine_passes"],
                    "prepare_ms": r.info["t_prepare_ms"],
                    "krylov_ms": r.info["t_krylov_ms"], "refine_ms": r.info["t_refine_ms"],
                    "resid_max": max(r.resid),
                    "lam_rel_err_max_over_floor": float(np.max(lam_err / np.maximum(
                        1e-6, g["pair_floor"]))),
                    "exp_op": {"us": op_s * 1e6, "algorithmic_bytes": op_bytes,
                               "GB_per_s": op_bytes / op_s / 1e9 if op_calls else None,
                               "frac_of_hbm_peak": op_bytes / op_s / 1e9 / HBM_PEAK_GBPS
                               if op_calls else None, "products": op_calls}}
    out["ratio_fp8_over_f64"] = out["fp8"]["solves_per_s"] / out["f64"]["solves_per_s"]
    h.close()
    return out


def orl_mall_resident(torch, eda, reps: int = 20) -> dict:
    """The ORL-shaped workload (d = 10304, n = 200, k = 40, t = 39, tol 1e-8,
    float64): prepare + solve per second and its product bandwidth.  Its
    19.8 MB factor stays in the 256 MB Infinity Cache between products, so
    the bandwidth is effective cache bandwidth, not an HBM fraction."""
    import datagen
    p = datagen.config("C2")
    h = eda.Handle()
    Xd = _upload(torch, p.X)
    counts = p.counts.tolist()

    def one():
        H_W, H_B = h.scatter_factors(Xd, counts)
        h.prepare(H_W, H_B)
        return h.solve(p.t, p.tol, block=8, seed=p.seed)
    for _ in range(3):
        one()
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for _ in range(reps):
        r = one()
        infos.append(r.info)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / reps
    op_calls = sum(i["op_calls"] for i in infos)
    op_s = sum(i["t_op_ms"] for i in infos) / op_calls / 1e3
    h.close()
    return {"workload": f"d={p.d}, k={p.k} x n_j=5 (n={p.n}), t={p.t}, block 8, tol {p.tol:g}, "
                        "float64, prepare + solve",
            "solves_per_s": 1.0 / el, "ms": 1e3 * el, "status": r.status,
            "iters": r.info["iters"],
            "exp_op": {"us": op_s * 1e6, "effective_GB_per_s": infos[-1]["op_bytes"] / op_s / 1e9,
                       "note": "Infinity-Cache resident factor: effective, not HBM, bandwidth"}}


def solve_variants(torch, eda, reps: int = 5) -> dict:
    """Lanczos-form Krylov solve, Arnoldi-form Krylov solve and reduced
    direct solve, solve phase only (the preparation is shared), at C1 and C2."""
    import datagen
    out = {}
    for name in ("C1", "C2"):
        p = datagen.config(name)
        h = eda.Handle()
        HW, HB = h.scatter_factors(_upload(torch, p.X), p.counts.tolist())
        h.prepare(HW, HB)
        row = {"workload": f"d={p.d}, n={p.n}, k={p.k}, t={p.t}, tol={p.tol:g}"}
        for tag, fn in (("lanczos", lambda: h.solve(p.t, p.tol, block=8, seed=p.seed)),
                        ("arnoldi", lambda: h.solve(p.t, p.tol, block=8, seed=p.seed, form="A")),
                        ("jacobi_davidson", lambda: h.solve(p.t, p.tol, block=8, seed=p.seed,
                                                            form="JD")),
                        ("direct", lambda: h.solve_direct(p.t))):
            r = fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                r = fn()
            torch.cuda.synchronize()
            el = (time.perf_counter() - t0) / reps
            row[tag] = {"solves_per_s": 1.0 / el, "ms": 1e3 * el, "status": r.status,
                        "iters": r.info["iters"], "resid_max": max(r.resid), "lam": r.ritz}
        lk = np.array(row["lanczos"].pop("lam"))
        for tag in ("arnoldi", "jacobi_davidson", "direct"):
            lv = np.array(row[tag].pop("lam"))
            row[f"lam_max_rel_diff_{tag}"] = float(np.max(np.abs(lk - lv) / lv))
            row[f"ratio_{tag}_over_lanczos"] = (row[tag]["solves_per_s"]
                                                / row["lanczos"]["solves_per_s"])
        out[name] = row
        h.close()
    return out


def nn_tol_sweep(torch, eda, reps: int = 20) -> dict:
    """Section 3.3 on the headline-shaped split (d = 10304, 200 training
    samples of 40 classes, 5 testing samples per class from the same class
    model): solve to each tolerance, classify the testing samples by 1-NN in
    the solution's subspace, and compare with the tightest solution: the
    accuracy, sin of the angle, the largest change of a nearest distance and
    whether Theorem 3.7's bounds hold.  Also the classification call itself
    (projections of all samples + distances): time and the bytes of the
    samples it streams."""
    import datagen
    p = datagen.config("C2", with_data=False)
    Xtr, Xte, lte = datagen.make_split(p.d, p.counts, np.full(p.k, 5), p.r, p.seed)
    h = eda.Handle()
    tr, te = _upload(torch, Xtr), _upload(torch, Xte)
    labels = torch.as_tensor(p.labels()).cuda()
    HW, HB = h.scatter_factors(tr, p.counts.tolist())
    h.prepare(HW, HB)
    sols = {}
    for tol in (1e-2, 1e-4, 1e-6, 1e-8, 1e-10):
        r = h.solve(p.t, tol, block=8, seed=p.seed)
        pred, idx, dist = h.nn_classify(r.X, tr, labels, te)
        torch.cuda.synchronize()
        sols[tol] = (r, r.X.cpu().numpy(), pred.cpu().numpy(), dist.cpu().numpy())
    Vref = sols[1e-10][1]
    dref = sols[1e-10][3]
    rows = []
    for tol, (r, X, pred, dist) in sols.items():
        # sin = ||(I - Vref Vref^T) X||_2, cos = ||Vref^T X||_2 (Theorem 3.7)
        sin = float(np.linalg.norm(X - Vref @ (Vref.T @ X), 2))
        cos = float(np.linalg.norm(Vref.T @ X, 2))
        lo, hi = (dist - 2 * sin) / cos, dist * cos + 2 * sin
        rows.append({"tol": tol, "status": r.status, "iters": r.info["iters"],
                     "accuracy": float(np.mean(pred == lte)), "sin_angle_vs_1e-10": sin,
                     "max_nn_dist_change": float(np.max(np.abs(dist - dref))),
                     "thm37_holds": bool(np.all(lo <= dref + 1e-12) and np.all(dref <= hi + 1e-12))})
    X = sols[1e-8][0].X
    for _ in range(3):
        h.nn_classify(X, tr, labels, te)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        h.nn_classify(X, tr, labels, te)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / reps
    nbytes = 8.0 * p.d * (Xtr.shape[1] + Xte.shape[1] + p.t)
    h.close()
    return {"workload": f"d={p.d}, {Xtr.shape[1]} training / {Xte.shape[1]} testing samples, "
                        f"k={p.k}, t={p.t}",
            "sweep": rows,
            "classify": {"us": 1e6 * el, "sample_bytes": nbytes, "GB_per_s": nbytes / el / 1e9,
                         "testing_samples_per_s": Xte.shape[1] / el}}


def batched(torch, eda, count: int = 64, reps: int = 2) -> dict:
    import datagen
    ps = datagen.batched_configs(count)
    h = eda.Handle()
    probs = []
    for p in ps:
        HW, HB = h.scatter_factors(_upload(torch, p.X), p.counts.tolist())
        probs.append((HW, HB, p.t, p.tol))
    out = {"workload": f"{count} problems, d in {{1024, 4096, 10304}}, k in [10, 68], "
                       f"n_j in [2, 20], t = k-1, tol 1e-6",
           "P_bytes_f32_total": int(sum(p.d * (p.n + p.k) * 4 for p in ps))}
    for tag, storage, basis in (("f32", "f32", "f32"), ("f64", "f64", "f64")):
        h.solve_batched(probs, storage=storage, krylov_dtype=basis, seed=4000)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            res, st = h.solve_batched(probs, storage=storage, krylov_dtype=basis, seed=4000)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / reps
        out[tag] = {"problems_per_s": count / el, "ms_per_batch": 1e3 * el, "status": int(st),
                    "ok": int(sum(r.status == 0 for r in res)),
                    "max_iters": int(max(r.info["iters"] for r in res)),
                    "max_refine_passes": int(max(r.info["refine_passes"] for r in res)),
                    "float64_continuations": int(sum(bool(r.info["flags"] & eda.EDA_WARN_FALLBACK)
                                                     for r in res))}
    # the same problems one after another: float64 (the plain single-problem
    # solve) and float32 factors with a float32 basis
    hs = eda.Handle()
    for tag, storage, basis in (("f64", "f64", "f64"), ("f32", "f32", "f32")):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i, (HW, HB, t, tol) in enumerate(probs):
            hs.prepare(HW, HB, storage=storage)
            hs.solve(t, tol, block=8, seed=4000 + i, krylov_dtype=basis)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out[f"one_by_one_{tag}"] = {"problems_per_s": count / el, "ms": 1e3 * el}
    out["speedup_batched_f64_over_one_by_one_f64"] = (out["f64"]["problems_per_s"]
                                                      / out["one_by_one_f64"]["problems_per_s"])
    out["speedup_batched_f32_over_one_by_one_f64"] = (out["f32"]["problems_per_s"]
                                                      / out["one_by_one_f64"]["problems_per_s"])
    hs.close()
    h.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the measurements beside the headline step")
    ap.add_argument("--profile-op", type=int, default=0)
    ap.add_argument("--workload", default="C5", choices=["C5", "C2"],
                    help="workload of --profile-op")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the row-sharded design is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch
    import datagen
    import paper_1512_06500_amd as eda

    torch.cuda.set_device(0)
    p = datagen.config(args.workload if args.profile_op > 0 else "C5")
    b, tol = 8, p.tol
    Xd = _upload(torch, p.X)
    counts = p.counts.tolist()
    h = eda.Handle()

    if args.profile_op > 0:
        profile_op(torch, eda, h, Xd, counts, args.profile_op)
        return

    def step():
        H_W, H_B = h.scatter_factors(Xd, counts)
        h.prepare(H_W, H_B)
        return h.solve(p.t, tol, block=b, seed=p.seed)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = step()
        infos.append(res.info)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    assert res.status == eda.EDA_OK, res.message

    op_calls = sum(i["op_calls"] for i in infos)
    op_ms = sum(i["t_op_ms"] for i in infos)
    op_bytes = infos[-1]["op_bytes"]
    avg_op_s = op_ms / op_calls / 1e3
    achieved = op_bytes / avg_op_s / 1e9
    # sanity against the stored oracle values (text file, no oracle import)
    from tests.golden.reader import read as read_golden
    g = read_golden("C5")
    lam_err = np.abs(np.array(res.ritz) - g["lam"]) / g["lam"]

    out = {
        "metric": METRIC,
        "value": args.steps / el,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * el / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "large EDA solve: d=65536 (256x256), k=100 x n_j=20 (n=2000), "
                               "t=99, block 8, tol 1e-6 (per-pair floors), float64, "
                               "scatter -> prepare -> solve",
                   "d": p.d, "n": p.n, "k": p.k, "t": p.t, "block": b, "tol": tol,
                   "storage": "f64"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBPS,
                     "traffic": counter_traffic(),
                     "kernel": "exp-op e^{-s} M V (b=8) over the 1.1 GB factor: tn_lds + reduce "
                               "+ split core product + reduce + nn_stream",
                     "bytes_per_launch": op_bytes, "avg_launch_us": avg_op_s * 1e6,
                     "launches": op_calls},
        "breakdown_ms": {
            "prepare": float(np.mean([i["t_prepare_ms"] for i in infos])),
            "krylov": float(np.mean([i["t_krylov_ms"] for i in infos])),
            "refine_and_final": float(np.mean([i["t_refine_ms"] for i in infos])),
            "op_total": op_ms / args.steps,
        },
        "solve": {"iters": res.info["iters"], "restarts": res.info["restarts"],
                  "resid_max": max(res.resid),
                  "lam_max_rel_err_vs_stored_oracle": float(lam_err.max()),
                  "lam_rel_err_max_over_pair_floor": float(np.max(
                      lam_err / np.maximum(1e-6, g["pair_floor"])))},
    }
    h.close()
    if not args.no_extra:
        out["large_fp8_vs_f64"] = large_fp8_vs_f64(torch, eda, p, Xd)
        out["orl_mall_resident"] = orl_mall_resident(torch, eda)
        out["mixed_vs_f64"] = mixed_vs_f64(torch, eda)
        out["solve_variants"] = solve_variants(torch, eda)
        out["nn_tol_sweep"] = nn_tol_sweep(torch, eda)
        out["batched"] = batched(torch, eda)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p)
        out["cpu_baseline_1thread"] = cpu_baseline(p, threads=1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
