"""Throughput benchmark of the FAST-HALS sweep on one MI355X.

Workloads (``--config``):
  c4  (default) large bag-of-words matrix, V = 100,000 terms x D = 300,000
      documents CSR, about 0.1% dense (30,006,921 nnz), Zipf(1.05) term
      popularity, tf-idf with unit-norm documents; K = 400; FP32 path (or
      ``--precision bf16`` for the BF16 products)
  c1  the bag-of-words stand-in for 20 Newsgroups, V = 26,000 x D = 11,000
      CSR (about 0.3% dense); K = 200 by default (``--K``)
  c2  dense image-shaped matrix, 10,000 x 10,000, planted rank 300; K = 240

A "step" is one full sweep of Alg. 1 (H half, then W half) with all inputs
resident in HBM.  Prints one JSON line:
  value        sweeps per second, event-timed over --steps sweeps
  roofline     the dominant kernel's algorithmic work per launch divided by its
               event-timed duration (HIP events recorded on the plan's stream
               around every launch), against MI355X's published peak
  cpu_baseline the FP64 oracle (untiled Alg. 1, NumPy/SciPy) timed on this
               host's cores on a bounded sample of the same workload
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "HALS sweeps/s + % HBM/MFMA roofline; time-to-rel-objective 1e-4 vs plain FP32"
PEAK = {"fp32_tflops": 157.3, "bf16_tflops": 2500.0, "hbm_gbs": 8000.0}
COUNTERS = os.path.join(ROOT, "profiles", "counters.json")
CSRC = os.path.join(ROOT, "paper_1904_07935_amd", "csrc")
DEFAULT_K = {"c1": 200, "c2": 240, "c4": 400}


def parse(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="c4", choices=["c1", "c2", "c4"])
    ap.add_argument("--K", type=int, default=0, help="rank (default: the workload's own)")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16"])
    ap.add_argument("--profile-sweeps", type=int, default=5)
    ap.add_argument("--repeats", type=int, default=3,
                    help="further timed runs of --steps sweeps (their median is reported)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tsync", action="store_true")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="afterwards, copy this many bytes device-to-device three times "
                         "(a kernel of known traffic for scaling HBM counters)")
    return ap.parse_args(argv)


# ------------------------------------------------------------ workloads ----

def load_workload(name, K, precision):
    """Inputs of a named workload: (A as datagen.Csr or dense ndarray, W0, H0, config)."""
    import datagen

    K = K or DEFAULT_K[name]
    if name == "c2":
        A = datagen.c2()
        V, D = A.shape
        W0, H0 = datagen.uniform_init(V, D, K, seed=1)
        cfg = {"V": V, "D": D, "nnz": V * D, "format": "dense",
               "init": "U[0,1) W and H (seed 1)"}
        tag = f"c2_dense_{V}x{D}_k{K}_{precision}"
    else:
        corpus = datagen.c4() if name == "c4" else datagen.c1()
        A = corpus.A
        V, D = A.rows, A.cols
        W0, H0 = datagen.uniform_init_matched(V, D, K, datagen.mean_value(A), seed=1)
        cfg = {"V": V, "D": D, "nnz": int(A.nnz), "format": "csr",
               "init": "U[0,1) W, H scaled to the data mean (seed 1)"}
        tag = f"{name}_bow_{V}x{D}_k{K}_{precision}"
    cfg.update({"workload": tag, "K": K, "precision": precision, "eps": 1e-16})
    return A, W0, H0, cfg


# ------------------------------------------------------------- roofline ----

def step_work(step, V, D, K, nnz, dense=False, precision="fp32"):
    """Algorithmic work of one launch of a step: (amount, unit, bound, peak).

    Column updates and Grams: 2 rows K^2 flop on the FP32 matrix cores.
    Dense products: 2 V D K flop on the matrix cores of their input type.
    Sparse products: compulsory bytes -- the CSR (index and value per nonzero,
    row pointers), the gathered factor read once and the output written once."""
    if step == "update_W":
        return 2.0 * V * K * K, "flop", "mfma", PEAK["fp32_tflops"]
    if step == "update_H":
        return 2.0 * D * K * K, "flop", "mfma", PEAK["fp32_tflops"]
    if step in ("gram_S", "gram_Q"):
        rows = V if step == "gram_S" else D
        return 2.0 * rows * K * K, "flop", "mfma", PEAK["fp32_tflops"]
    if dense:
        peak = PEAK["bf16_tflops"] if precision == "bf16" else PEAK["fp32_tflops"]
        return 2.0 * V * D * K, "flop", "mfma", peak
    rows_out, rows_x = (D, V) if step == "product_R" else (V, D)
    vbytes = 6.0 if precision == "bf16" else 8.0
    xbytes = 2.0 if precision == "bf16" else 4.0
    b = vbytes * nnz + 4.0 * (rows_out + 1) + xbytes * K * rows_x + 4.0 * K * rows_out
    return b, "byte", "hbm", PEAK["hbm_gbs"]


def bound_seconds(step, V, D, K, nnz, dense, precision):
    """Time of one launch at its roofline (work / peak)."""
    amount, unit, _, peak = step_work(step, V, D, K, nnz, dense, precision)
    return amount / (peak * (1e12 if unit == "flop" else 1e9))


def source_digest():
    """Digest of the code (comments and blank lines left out) of every library
    source; the stored HBM counters are reported only if it matches."""
    h = hashlib.sha256()
    for f in sorted(os.listdir(CSRC)):
        if not f.endswith((".hip", ".cpp", ".hpp", ".h")):
            continue
        with open(os.path.join(CSRC, f)) as fh:
            txt = fh.read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        txt = re.sub(r"//[^\n]*", "", txt)
        h.update(f.encode())
        h.update("\n".join(l.rstrip() for l in txt.splitlines() if l.strip()).encode())
    return h.hexdigest()[:16]


def traffic_for(step, workload):
    """HBM bytes per launch from the committed PMC counters (FETCH_SIZE +
    WRITE_SIZE, scaled by a copy of known size), if they were taken on the
    current sources; else None."""
    if not os.path.exists(COUNTERS):
        return None
    try:
        with open(COUNTERS) as fh:
            c = json.load(fh)
    except ValueError:
        return None
    ent = c.get("entries", {}).get(f"{workload}:{step}")
    if not ent or c.get("source_digest") != source_digest():
        return None
    return ent["hbm_bytes_per_launch"]


# --------------------------------------------------------- CPU baseline ----

def host_cpu():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _threads():
    try:
        from threadpoolctl import threadpool_info
        return int(max([i.get("num_threads", 1) for i in threadpool_info()] or [os.cpu_count()]))
    except Exception:
        return int(os.cpu_count() or 1)


def cpu_baseline(A, W0, H0, min_seconds, sample_div=0):
    """The FP64 oracle on this host.  sample_div = 0: whole sweeps, repeated for
    at least min_seconds.  sample_div = s > 0: one sweep's oracle halves on
    slices -- the H half on the first D/s and D/(2s) documents, the W half on
    the first V/s and V/(2s) terms -- each half's time fitted as a + b n over
    its slice size n (the intercept holds the Gram matrix of the full other
    factor) and evaluated at the full size."""
    import numpy as np
    import scipy.sparse as sp

    import datagen
    from oracle import hals

    eps = 1e-16
    if isinstance(A, datagen.Csr):
        Ao = sp.csr_matrix((A.val.astype(np.float64), A.col, A.rowptr), shape=(A.rows, A.cols))
    else:
        Ao = np.asarray(A, dtype=np.float64)
    W = hals.normalize_columns(W0)
    H = H0.astype(np.float64)
    out = {"unit": "sweeps/s", "cores": _threads(), "kind": "oracle", "host_cpu": host_cpu()}
    if sample_div <= 0:
        t0 = time.perf_counter()
        done = 0
        while done < 1 or (time.perf_counter() - t0 < min_seconds and done < 500):
            W, H = hals.sweep(Ao, W, H, eps)
            done += 1
        dt = time.perf_counter() - t0
        out.update(value=done / dt,
                   sample=f"{done} full sweeps of the same workload (FP64 oracle, untiled "
                          f"Alg. 1, NumPy/SciPy), {dt:.1f} s")
        return out
    V, D = Ao.shape
    AoT = Ao.T.tocsr()
    s = sample_div
    t_total = 0.0
    th, tw = [], []
    for n in (D // (2 * s), D // s):
        An = AoT[:n].T  # the first n documents (columns of A)
        t0 = time.perf_counter()
        hals.h_half(An, W, H[:, :n], eps)
        th.append((n, time.perf_counter() - t0))
    for m in (V // (2 * s), V // s):
        Am = Ao[:m]
        t0 = time.perf_counter()
        hals.w_half(Am, W[:m], H, eps)
        tw.append((m, time.perf_counter() - t0))

    def at_full(pts, full):
        (n1, t1), (n2, t2) = pts
        b = (t2 - t1) / (n2 - n1)
        return max(t1 - b * n1, 0.0) + b * full

    est = at_full(th, D) + at_full(tw, V)
    t_total = sum(t for _, t in th + tw)
    out.update(value=1.0 / est,
               sample=f"one sweep extrapolated from the oracle's halves on slices (H half on "
                      f"{th[0][0]} and {th[1][0]} of {D} documents, W half on {tw[0][0]} and "
                      f"{tw[1][0]} of {V} terms; linear in slice size), {t_total:.1f} s of "
                      f"CPU work, estimated {est:.1f} s per sweep")
    return out


# --------------------------------------------------------------- t_sync ----

def measure_t_sync(groups, K, dev):
    """The W update's per-column latency floor: the W update on a problem of
    64 rows per column group (the same number of groups as the workload), where
    each column's arithmetic is negligible next to its norm exchange; microseconds
    per column."""
    import numpy as np

    import datagen
    from paper_1904_07935_amd.api import Matrix, Plan

    V = max(64 * groups, K)
    corpus = datagen.bag_of_words(V, max(2 * K, 1024), 1.1, 40.0, 11)
    W0, H0 = datagen.uniform_init_matched(V, corpus.A.cols, K, datagen.mean_value(corpus.A), 1)
    old = os.environ.get("NMF_W_COLUMN_GROUPS")
    os.environ["NMF_W_COLUMN_GROUPS"] = str(groups)
    try:
        import torch
        W = torch.tensor(W0, device=dev)
        Ht = torch.tensor(np.ascontiguousarray(H0.T), device=dev)
        plan = Plan(Matrix.from_csr(corpus.A, dev), W, Ht, eps=1e-16)
    finally:
        if old is None:
            del os.environ["NMF_W_COLUMN_GROUPS"]
        else:
            os.environ["NMF_W_COLUMN_GROUPS"] = old
    got = plan.info()["w_groups"]
    plan.sweep(2)
    plan.profile(True)
    plan.sweep(5)
    plan.profile(False)
    ms, n = plan.profile_read()["update_W"]
    plan.close()
    return {"us_per_column": round(1000.0 * ms / max(n, 1) / K, 3), "w_groups": got,
            "probe": f"W update of a {V} x {corpus.A.cols} CSR problem at K = {K} with {got} "
                     f"column groups, per column"}


# ----------------------------------------------------------------- main ----

def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}, WORLD_SIZE {world}); "
              "the FAST-HALS library here runs on a single GPU", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import datagen
    from paper_1904_07935_amd.api import Matrix, Plan

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    t_gen = time.perf_counter()
    A, W0, H0, cfg = load_workload(args.config, args.K, args.precision)
    t_gen = time.perf_counter() - t_gen
    print(f"[bench] {cfg['workload']}: inputs drawn in {t_gen:.1f} s", file=sys.stderr, flush=True)
    dense = cfg["format"] == "dense"
    V, D, K, nnz = cfg["V"], cfg["D"], cfg["K"], cfg["nnz"]
    W = torch.tensor(W0, device=dev)
    Ht = torch.tensor(np.ascontiguousarray(H0.T), device=dev)
    M = Matrix.from_dense(A, dev) if dense else Matrix.from_csr(A, dev)
    plan = Plan(M, W, Ht, eps=1e-16, precision=args.precision)
    info = plan.info()

    def timed(n):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        plan.sweep(n)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n

    plan.sweep(args.warmup)
    torch.cuda.synchronize()
    ms = timed(args.steps)
    print(f"[bench] timed {args.steps} sweeps: {ms:.4f} ms per sweep", file=sys.stderr, flush=True)
    repeats = [timed(args.steps) for _ in range(args.repeats)]

    # per-step event timing (separate pass; events on the plan's stream)
    plan.profile(True)
    plan.sweep(max(args.profile_sweeps, 1))
    plan.profile(False)
    prof = plan.profile_read()
    per_step_us = {k: 1000.0 * v[0] / max(v[1], 1) for k, v in prof.items() if v[1] > 0}
    dominant = max(per_step_us, key=per_step_us.get)
    amount, unit, bound, peak = step_work(dominant, V, D, K, nnz, dense, args.precision)
    t = per_step_us[dominant] * 1e-6
    if unit == "flop":
        achieved, runit = amount / t / 1e12, "TFLOP/s"
    else:
        achieved, runit = amount / t / 1e9, "GB/s"
    bound_us = {k: 1e6 * bound_seconds(k, V, D, K, nnz, dense, args.precision)
                for k in per_step_us}
    per_kernel_frac = {k: round(bound_us[k] / per_step_us[k], 4) for k in per_step_us}
    _, rel = plan.objective()
    plan.close()
    del plan, W, Ht, M
    torch.cuda.empty_cache()

    out = {
        "metric": METRIC,
        "value": round(1000.0 / ms, 3),
        "unit": "sweeps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "bf16-products/f32",
        "data": "synthetic",
        "config": cfg,
        "roofline": {"kernel": dominant, "bound": bound, "achieved": round(achieved, 3),
                     "peak": peak, "unit": runit, "frac": round(achieved / peak, 5),
                     "traffic": traffic_for(dominant, cfg["workload"]),
                     "work_per_launch": amount, "work_unit": unit},
        "repeat_ms_per_step": [round(r, 4) for r in repeats],
        "median_ms_per_step": round(float(np.median([ms] + repeats)), 4),
        "per_step_us": {k: round(v, 2) for k, v in per_step_us.items()},
        "per_step_roofline_frac": per_kernel_frac,
        "sweep_roofline_frac": round(sum(bound_us.values()) / (1000.0 * ms), 4),
        "w_groups": info["w_groups"],
        "rel_objective": rel,
    }
    if not args.no_tsync:
        ts = measure_t_sync(info["w_groups"], K, dev)
        out["t_sync_us_per_column"] = ts["us_per_column"]
        out["t_sync"] = ts
        out["k_t_sync_us"] = round(K * ts["us_per_column"], 1)
    if args.copy_bytes > 0:
        src = torch.ones(args.copy_bytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_bytes"] = args.copy_bytes
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(A, W0, H0, args.cpu_seconds,
                                           sample_div=3 if args.config == "c4" else 0)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
