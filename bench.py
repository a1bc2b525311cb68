"""Benchmark: end-to-end EDA solves on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Workload (the configuration the metric is quoted on): d = 10304 (112 x 92
images), k = 40 classes x n_j = 5 samples (n = 200), t = 39 dominant
eigenpairs, block width 8, tol 1e-8, float64 throughout.  Synthetic samples
(unit-norm columns, 128-dim class signal, 5% noise) stand in for the ORL
face images, which are not available.

One step = the whole hot path on one batch of samples already resident in
HBM: scatter factors -> factor ingest + Gram + small eigensolves + cores ->
block Lanczos with Rayleigh-Ritz -> back-transform + orthonormalisation.
`value` is solves per second over the timed steps.

`roofline` covers the exp-op, the block product e^{-s} M V (b = 8) with two
streaming passes over P = [H_W H_B] (d x 240 float64): its algorithmic
bytes 2 d N 8 + 3 d b 8 per product divided by its average duration,
measured with HIP events on the library's stream around every product
inside the timed solves (four launches: P^T V on the matrix cores, the
chunk sum, the core product, alpha V + P Z).  Peak: MI355X HBM3E, 8 TB/s.

`cpu_baseline` times the FP64 CPU oracle (exact (n+k)-dimensional reduction
of the pencil, NumPy/SciPy on the host's cores) on the same workload.

`mixed_vs_f64` (second half of the metric): solves/s of the d = 32256,
k = 38, n = 1216, t = 37 workload at tol 1e-6, float64 end to end against
bfloat16 factors + float32 basis + float64 refinement (prepare + solve each).

`nn_tol_sweep`: Section 3.3 on a split of the headline workload (200
training, 200 testing samples): 1-NN accuracy, angle to the tol-1e-10
subspace and the Theorem 3.7 check for tol 1e-2 ... 1e-10, and the time of
one eda_nn_classify call.

`batched`: 64 independent problems of uneven shape (d in {1024, 4096,
10304}, k in [10, 68], n_j in [2, 20], float32 factors, tol 1e-6) solved by
one eda_solve_batched call, problems/s, against the same problems solved one
after another.

`--profile-op K`: only K exponential products (b = 8) on the headline
workload plus one 256 MiB copy, for hardware-counter runs.
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


def cpu_baseline(p, budget_s: float = 15.0) -> dict:
    import oracle
    try:
        from threadpoolctl import threadpool_info
        threads = max((i.get("num_threads", 1) for i in threadpool_info()), default=1)
    except Exception:  # pragma: no cover
        threads = os.cpu_count() or 1
    reps, t0 = 0, time.perf_counter()
    while True:
        H_W, H_B = oracle.scatter_factors(p.X, p.counts)
        oracle.eda_reduced(H_W, H_B, p.t)
        reps += 1
        if time.perf_counter() - t0 > budget_s or reps >= 50:
            break
    el = time.perf_counter() - t0
    return {"value": reps / el, "unit": "solves/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{reps} full solves of the same workload by the oracle's exact "
                      f"(n+k)-dim reduction (scatter factors, Householder QR of [H_W H_B], "
                      f"dense pencil eig), {el:.1f} s"}


def counter_traffic():
    """HBM bytes per product from the committed counter summary, or None when
    the streaming kernels have changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "exp_op_c2_counters.md")
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
    """K products e^{-s} M V (b = 8) and one 256 MiB device copy."""
    H_W, H_B = h.scatter_factors(Xd, counts)
    h.prepare(H_W, H_B)
    V = torch.randn(8, Xd.shape[0], dtype=torch.float64, device="cuda").t()
    out = torch.empty_like(V.t()).t()
    for _ in range(reps):
        h.opmv("M", V, out=out)
    src = torch.ones(32 << 20, dtype=torch.float64, device="cuda")
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


def large_fp8_vs_f64(torch, eda, reps: int = 3) -> dict:
    """The large FP8 workload (d = 65536, n = 2000, k = 100, t = 99, tol
    1e-6): float64 solve against FP8 E4M3 storage with a float32 basis and
    float64 refinement (solve phase only, preparation shared per storage),
    with the exponential product's bandwidth for each storage type."""
    import datagen
    from tests.golden.reader import read as read_golden
    p = datagen.config("C5")
    g = read_golden("C5")
    h = eda.Handle()
    H_W, H_B = h.scatter_factors(_upload(torch, p.X), p.counts.tolist())
    N = p.n + p.k
    out = {"workload": f"d={p.d}, k={p.k} x n_j={p.n // p.k} (n={p.n}), t={p.t}, block 8, "
                       f"tol {p.tol:g}"}
    for tag, storage, basis in (("f64", "f64", "f64"), ("fp8", "fp8", "f32")):
        h.prepare(H_W, H_B, storage=storage)
        V = torch.randn(8, p.d, dtype=torch.float64, device="cuda").t()
        o = torch.empty_like(V.t()).t()
        for _ in range(3):
            h.opmv("M", V, out=o)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(10):
            h.opmv("M", V, out=o)
        torch.cuda.synchronize()
        op_s = (time.perf_counter() - t0) / 10
        sp = {"f64": 8, "fp8": 1}[storage]
        op_bytes = 2.0 * p.d * N * sp + 3.0 * p.d * 8 * 8
        r = h.solve(p.t, p.tol, block=8, seed=p.seed, krylov_dtype=basis)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            r = h.solve(p.t, p.tol, block=8, seed=p.seed, krylov_dtype=basis)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / reps
        lam_err = np.abs(np.array(r.ritz) - g["lam"]) / np.array(g["lam"])
        out[tag] = {"solves_per_s": 1.0 / el, "ms": 1e3 * el, "status": r.status,
                    "storage": storage, "basis": basis, "iters": r.info["iters"],
                    "refine_passes": r.info["refine_passes"],
                    "krylov_ms": r.info["t_krylov_ms"], "refine_ms": r.info["t_refine_ms"],
                    "resid_max": max(r.resid),
                    "lam_rel_err_max_over_floor": float(np.max(lam_err / np.maximum(
                        1e-6, g["pair_floor"]))),
                    "exp_op": {"us": op_s * 1e6, "algorithmic_bytes": op_bytes,
                               "GB_per_s": op_bytes / op_s / 1e9,
                               "frac_of_hbm_peak": op_bytes / op_s / 1e9 / HBM_PEAK_GBPS}}
    out["ratio_fp8_over_f64"] = out["fp8"]["solves_per_s"] / out["f64"]["solves_per_s"]
    h.close()
    return out


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
        for tag in ("arnoldi", "direct"):
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
                    "max_refine_passes": int(max(r.info["refine_passes"] for r in res))}
    # the same problems one after another (float32 factors, float32 basis)
    hs = eda.Handle()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i, (HW, HB, t, tol) in enumerate(probs):
        hs.prepare(HW, HB, storage="f32")
        hs.solve(t, tol, block=8, seed=4000 + i, krylov_dtype="f32")
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    out["one_by_one_f32"] = {"problems_per_s": count / el, "ms": 1e3 * el}
    out["speedup_batched_over_one_by_one"] = out["f32"]["problems_per_s"] / (count / el)
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
                    help="skip the mixed-precision and batched measurements")
    ap.add_argument("--profile-op", type=int, default=0)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the row-sharded design is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch
    import datagen
    import paper_1512_06500_amd as eda

    torch.cuda.set_device(0)
    p = datagen.config("C2")
    b, tol = 8, p.tol
    Xd = torch.from_numpy(np.ascontiguousarray(p.X.T)).cuda().t()
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
    g = read_golden("C2")
    lam_err = float(np.max(np.abs(np.array(res.ritz) - g["lam"]) / g["lam"]))

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
        "config": {"workload": "ORL-shaped EDA solve: d=10304, k=40 x n_j=5 (n=200), "
                               "t=39, block 8, tol 1e-8, float64",
                   "d": p.d, "n": p.n, "k": p.k, "t": p.t, "block": b, "tol": tol,
                   "storage": "f64"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBPS,
                     "traffic": counter_traffic(),
                     "kernel": "exp-op e^{-s} M V (b=8): tn_mfma + reduce + core nn + nn",
                     "bytes_per_launch": op_bytes, "avg_launch_us": avg_op_s * 1e6,
                     "launches": op_calls},
        "breakdown_ms": {
            "prepare": float(np.mean([i["t_prepare_ms"] for i in infos])),
            "krylov": float(np.mean([i["t_krylov_ms"] for i in infos])),
            "op_total": op_ms / args.steps,
        },
        "solve": {"iters": res.info["iters"], "restarts": res.info["restarts"],
                  "resid_max": max(res.resid), "lam_max_rel_err_vs_stored_oracle": lam_err},
    }
    h.close()
    if not args.no_extra:
        out["mixed_vs_f64"] = mixed_vs_f64(torch, eda)
        out["solve_variants"] = solve_variants(torch, eda)
        out["nn_tol_sweep"] = nn_tol_sweep(torch, eda)
        out["large_fp8_vs_f64"] = large_fp8_vs_f64(torch, eda)
        out["batched"] = batched(torch, eda)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
