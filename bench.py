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
    ap.add_argument("--config", default="c4", choices=["c1", "c2", "c3", "c4"])
    ap.add_argument("--K", type=int, default=0, help="rank (default: the workload's own)")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16"])
    ap.add_argument("--profile-sweeps", type=int, default=5)
    ap.add_argument("--repeats", type=int, default=3,
                    help="further timed runs of --steps sweeps (their median is reported)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tsync", action="store_true")
    ap.add_argument("--tto", action="store_true",
                    help="time-to-objective instead of throughput: FAST-HALS FP32 against "
                         "its BF16-product form and the MU baseline (--config c1/c2/c4), "
                         "or cold/WTA/network-warm fold-in (--config c3)")
    ap.add_argument("--tto-sweeps", type=int, default=0)
    ap.add_argument("--tile-study", action="store_true",
                    help="time the H update for tile widths 16/32/64 at K = 80/160/240/400 "
                         "(rows-in-registers kernel) beside the LDS/VGPR capacity model")
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


def plnmf_cpu_baseline(A, W0, H0, min_seconds):
    """PL-NMF-cpu (the paper's tiled Alg. 2 in FP64 with OpenMP, libplnmf_cpu.so)
    on all host threads: one warm-up sweep, then whole sweeps for at least
    min_seconds (at least one)."""
    from paper_1904_07935_amd import cpu

    p = cpu.CpuPlan(A, W0, H0)
    p.sweep(1)
    t0 = time.perf_counter()
    done = 0
    while done < 1 or (time.perf_counter() - t0 < min_seconds and done < 500):
        p.sweep(1)
        done += 1
    dt = time.perf_counter() - t0
    info = p.info()
    p.close()
    return {"value": done / dt, "unit": "sweeps/s", "cores": info["threads"], "tile": info["tile"],
            "kind": "plnmf_cpu", "host_cpu": host_cpu(),
            "sample": f"{done} full sweeps of the same workload after one warm-up, {dt:.1f} s"}


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


# ------------------------------------------------------ time to objective ----

TTO_SWEEPS = {"c1": 100, "c2": 100, "c4": 50}


def _first(trace, pred):
    for i, (t, f) in enumerate(trace):
        if pred(i, f):
            return i, t
    return None, None


def tto_full(args, dev):
    """FAST-HALS FP32 (the reference), FAST-HALS with BF16 products and the MU
    baseline from the same init: per sweep the event-timed sweep time
    (objective off the clock) and the relative objective.  Target: the FP32
    run's objective after the workload's sweep count plus 1e-4 (absolute, in
    relative-objective units); also the alternative reading, the first sweep
    whose relative decrease is below 1e-4."""
    import numpy as np
    import torch

    from paper_1904_07935_amd.api import Matrix, Plan

    n = args.tto_sweeps or TTO_SWEEPS[args.config]
    A, W0, H0, cfg = load_workload(args.config, args.K, "fp32")
    dense = cfg["format"] == "dense"
    M = Matrix.from_dense(A, dev) if dense else Matrix.from_csr(A, dev)
    runs = {}
    for name, prec, algo in (("hals_fp32", "fp32", "hals"), ("hals_bf16", "bf16", "hals"),
                             ("mu_fp32", "fp32", "mu")):
        W = torch.tensor(W0, device=dev)
        Ht = torch.tensor(np.ascontiguousarray(H0.T), device=dev)
        plan = Plan(M, W, Ht, eps=1e-16, precision=prec)
        step = plan.sweep if algo == "hals" else plan.mu_sweep
        step(1)  # warm-up of the code paths, then back to the init
        W.copy_(torch.tensor(W0, device=dev))
        Ht.copy_(torch.tensor(np.ascontiguousarray(H0.T), device=dev))
        plan.close()
        plan = Plan(M, W, Ht, eps=1e-16, precision=prec)
        step = plan.sweep if algo == "hals" else plan.mu_sweep
        trace, tot = [], 0.0
        for _ in range(n):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record()
            step(1)
            e1.record()
            torch.cuda.synchronize()
            tot += e0.elapsed_time(e1) / 1000.0
            trace.append((tot, plan.objective()[1]))
        plan.close()
        del W, Ht
        runs[name] = trace
        print(f"[tto] {name}: {n} sweeps in {tot:.3f} s, final {trace[-1][1]:.6f}", file=sys.stderr,
              flush=True)
    f_ref = runs["hals_fp32"][-1][1]
    target = f_ref + 1e-4
    out = {"mode": "time_to_objective", "config": cfg, "sweeps": n, "f_ref": f_ref,
           "target": target, "runs": {}}
    for name, tr in runs.items():
        i, t = _first(tr, lambda i, f: f <= target)
        j, tj = _first(tr, lambda i, f: i > 0 and (tr[i - 1][1] - f) / tr[i - 1][1] < 1e-4)
        out["runs"][name] = {"sweeps_to_target": None if i is None else i + 1,
                             "seconds_to_target": t,
                             "sweeps_to_rel_change_1e-4": None if j is None else j + 1,
                             "seconds_to_rel_change_1e-4": tj,
                             "final": tr[-1][1], "ms_per_sweep": 1000.0 * tr[-1][0] / n}
    # time for each run to first reach a relative objective e, for a grid of e
    # from the slowest run's final value up to the largest first-sweep value
    hi = max(tr[0][1] for tr in runs.values())
    lo = max(tr[-1][1] for tr in runs.values())
    grid = [lo + (hi - lo) * x for x in (0.0, 0.01, 0.03, 0.1, 0.3, 0.6)]
    out["time_to_reach"] = [
        {"rel_objective": e, **{name: _first(tr, lambda i, f: f <= e)[1] for name, tr in runs.items()}}
        for e in grid]
    for name, tr in runs.items():
        out["runs"][name]["trace"] = [round(f, 8) for _, f in tr]
        out["runs"][name]["seconds"] = [round(t, 6) for t, _ in tr]
    hb, hf = runs["hals_bf16"], runs["hals_fp32"]
    out["bf16_vs_fp32_max_rel_diff"] = max(abs(b[1] - f[1]) / f[1] for b, f in zip(hb, hf))
    # the MU run's final objective: when FAST-HALS FP32 first reached it
    fm = runs["mu_fp32"][-1][1]
    i, t = _first(hf, lambda i, f: f <= fm)
    out["hals_time_to_mu_final"] = {"mu_final": fm, "hals_sweeps": None if i is None else i + 1,
                                    "hals_seconds": t, "mu_seconds": runs["mu_fp32"][-1][0]}
    print(json.dumps(out), flush=True)


def _csr_rows(c, r0, r1):
    import numpy as np

    import datagen
    a, b = int(c.rowptr[r0]), int(c.rowptr[r1])
    return datagen.Csr(r1 - r0, c.cols, (c.rowptr[r0:r1 + 1] - a).astype(np.int32),
                       c.col[a:b].copy(), c.val[a:b].copy())


def tto_foldin(args, dev):
    """Fold-in of new documents with W fixed: W from 100 FP32 sweeps of the
    C1 corpus at K = 200; 200,000 new documents drawn like C1 (its term
    permutation and idf, seed 3), the first 100,000 for training the network
    on HALS-converged solutions, the rest for evaluation.  Target: the
    cold-start fold-in's converged relative objective (decrease below 1e-9, at
    most 500 sweeps) plus 1e-4.  Time to target for cold (U[0,1), seed 4),
    WTA (max(eps, A^T W)) and network-warm starts, each a whole fold-in call
    (product, Gram, initialisation -- the network's inference included -- and
    the sweeps), event-timed."""
    import numpy as np
    import torch

    import datagen
    from paper_1904_07935_amd.api import Matrix, Mlp, Plan

    K, hidden = 200, 512
    corpus = datagen.c1()
    V = corpus.A.rows
    W0, H0 = datagen.uniform_init_matched(V, corpus.A.cols, K, datagen.mean_value(corpus.A), 1)
    W = torch.tensor(W0, device=dev)
    Ht = torch.tensor(np.ascontiguousarray(H0.T), device=dev)
    plan = Plan(Matrix.from_csr(corpus.A, dev), W, Ht, eps=1e-16)
    plan.sweep(100)
    t0 = time.perf_counter()
    docs = datagen.c3_docs(corpus, 200000, seed=3)
    half = docs.rows // 2
    train, evald = _csr_rows(docs, 0, half), _csr_rows(docs, half, docs.rows)
    print(f"[tto] documents drawn in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    Mtr, Mev = Matrix.from_csr(train, dev), Matrix.from_csr(evald, dev)

    def cold(c):
        _, h = datagen.uniform_init_matched(V, c.rows, K, datagen.mean_value(c), seed=4)
        return torch.tensor(np.ascontiguousarray(h.T), device=dev)

    def timed_foldin(M, H, init, net, sweeps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        plan.foldin(M, H, init=init, mlp=net, n_sweeps=sweeps, trace=False)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1000.0

    # training pairs: converged cold-start fold-in of the training documents
    Hs = cold(train)
    trs = plan.foldin(Mtr, Hs, init="given", n_sweeps=500, tol=1e-9)
    R = torch.zeros(train.rows, K, device=dev)
    plan.foldin(Mtr, R, init="wta", n_sweeps=0, trace=False)
    nrm = R.norm(dim=1, keepdim=True).clamp_min(1e-30)
    X, Y = (R / nrm).contiguous(), (Hs / nrm).contiguous()
    net = Mlp(K, hidden, device=dev, seed=11)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    losses = net.train(X, Y, epochs=args.tto_sweeps or 200, batch=1024, lr=1e-3, seed=3)
    e1.record()
    torch.cuda.synchronize()
    t_train = e0.elapsed_time(e1) / 1000.0
    print(f"[tto] network trained in {t_train:.2f} s, loss {losses[0]:.3e} -> {losses[-1]:.3e}",
          file=sys.stderr, flush=True)

    ref = plan.foldin(Mev, cold(evald), init="given", n_sweeps=500, tol=1e-12)
    target = ref[-1] + 1e-4
    gaps = (1e-4, 1e-5, 1e-6, 1e-7, 1e-8)
    out = {"mode": "time_to_objective", "config": {"workload": "c3_foldin_c1w_k200",
           "V": V, "K": K, "train_docs": train.rows, "eval_docs": evald.rows,
           "eval_nnz": int(evald.nnz), "hidden": hidden},
           "f_ref": ref[-1], "ref_sweeps": len(ref) - 1, "target": target,
           "train": {"pairs_sweeps": len(trs) - 1, "epochs": len(losses), "seconds": t_train,
                     "loss_first": losses[0], "loss_last": losses[-1]},
           "runs": {}}
    for init in ("given", "wta", "mlp"):
        H0e = cold(evald) if init == "given" else torch.zeros(evald.rows, K, device=dev)
        tr = plan.foldin(Mev, H0e.clone(), init=init, mlp=net if init == "mlp" else None,
                         n_sweeps=300)
        hit = [i for i, f in enumerate(tr) if f <= target]
        ns = hit[0] if hit else None
        t_setup = timed_foldin(Mev, H0e.clone(), init, net if init == "mlp" else None, 0)
        t_total = timed_foldin(Mev, H0e.clone(), init, net if init == "mlp" else None, ns) \
            if ns is not None else None
        name = {"given": "cold", "wta": "wta", "mlp": "mlp"}[init]
        per_gap = {}
        for g in gaps:
            h = [i for i, f in enumerate(tr) if f <= ref[-1] + g]
            per_gap[f"{g:g}"] = h[0] if h else None
        t_sweep = (timed_foldin(Mev, H0e.clone(), init, net if init == "mlp" else None, 50)
                   - t_setup) / 50.0
        out["runs"][name] = {"rel_after_init": tr[0], "sweeps_to_target": ns,
                             "seconds_to_target": t_total, "seconds_setup_and_init": t_setup,
                             "seconds_per_sweep": t_sweep, "sweeps_to_within": per_gap,
                             "trace_first_12": tr[:12]}
        print(f"[tto] {name}: init {tr[0]:.6f}, sweeps to target {ns}", file=sys.stderr,
              flush=True)
    plan.close()
    print(json.dumps(out), flush=True)


# ----------------------------------------------------------- tile study ----

LDS_BYTES = 160 * 1024
MFMA_CYCLES = 64  # one 32x32x2 FP32 matrix-core product per SIMD


def tile_model(K, T):
    """Capacity and cost model of the rows-in-registers H update at tile width
    T (the analogue of Sec. 5's model for this kernel).  Capacity: the
    workgroup's LDS holds two panels of NB = max(1, T/32) x 32 ceil(K/32) rows
    of 32 floats, two T x T G blocks and four 32 x max(T+1, 33) transposes; a
    lane's VGPRs hold the 16 ceil(K/32) row values, NB accumulators and the
    phase-2 columns (about 1.5 T / 2).  Cost per wave and tile: the product
    takes 16 ceil(K/32) NB matrix-core steps of 64 cycles (a 16-wide tile
    still runs a 32-wide product); phase 2 takes T column steps whose work
    grows with the T/2 columns a lane updates.  Returns the LDS bytes, a VGPR
    estimate, whether it fits, and the product and phase-2 cycles per sweep
    of one wave (phase-2 step cost 40 + 4 T/2 cycles, an estimate)."""
    nt = (K + 31) // 32
    nb = max(1, T // 32)
    lds = 4 * (2 * nb * nt * 1024 + 2 * T * T + 4 * 32 * max(T + 1, 33))
    vgpr = 16 * nt + 32 * nb + 3 * T // 2 + 64
    tiles = (K + T - 1) // T
    prod = tiles * 16 * nt * nb * MFMA_CYCLES
    ph2 = tiles * T * (40 + 4 * (T // 2))
    return {"lds_bytes": lds, "vgpr_est": vgpr, "fits": lds <= LDS_BYTES and (T != 64 or nt <= 6),
            "product_cycles": prod, "phase2_cycles": ph2, "model_cycles": prod + ph2}


def tile_study(args, dev):
    import numpy as np
    import torch

    import datagen
    from paper_1904_07935_amd.api import Matrix, Plan

    corpus = datagen.c4() if args.config == "c4" else datagen.c1()
    A = corpus.A
    M = Matrix.from_csr(A, dev)
    rows = []
    os.environ["NMF_H_KERNEL"] = "rows"
    for K in (80, 160, 240, 400):
        W0, H0 = datagen.uniform_init_matched(A.rows, A.cols, K, datagen.mean_value(A), 1)
        for T in (16, 32, 64):
            os.environ["NMF_TILE_T"] = str(T)
            mod = tile_model(K, T)
            W = torch.tensor(W0, device=dev)
            Ht = torch.tensor(np.ascontiguousarray(H0.T), device=dev)
            plan = Plan(M, W, Ht, eps=1e-16)
            got = plan.info()["tile"]
            us = None
            if got == T:
                plan.sweep(2)
                plan.profile(True)
                plan.sweep(5)
                plan.profile(False)
                ms, n = plan.profile_read()["update_H"]
                us = 1000.0 * ms / max(n, 1)
            plan.close()
            rows.append({"K": K, "T": T, "update_H_us": None if us is None else round(us, 1),
                         **mod})
            print(f"[tile] K={K} T={T}: {us} us (fits {mod['fits']})", file=sys.stderr, flush=True)
    del os.environ["NMF_TILE_T"], os.environ["NMF_H_KERNEL"]
    print(json.dumps({"mode": "tile_study", "config": {"workload": args.config, "V": A.rows,
                      "D": A.cols, "nnz": int(A.nnz)}, "rows": rows}), flush=True)


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
    if args.tile_study:
        tile_study(args, dev)
        return
    if args.tto or args.config == "c3":
        if args.config == "c3":
            tto_foldin(args, dev)
        else:
            tto_full(args, dev)
        return
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
        out["cpu_plnmf"] = plnmf_cpu_baseline(A, W0, H0, min(args.cpu_seconds, 5.0))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
