#!/usr/bin/env python3
"""Benchmark of the GAP SAFE screened coordinate-descent library on one MI355X.

A step is one whole Lasso path of the 72 x 7129 FP32 workload (AR(1)
correlation 0.5, standardized columns, 20-sparse truth, SNR 3), 100 lambdas
from lambda_max to lambda_max/1000, screening every 10 epochs, each lambda
solved to gap <= 1e-8 ||y||^2, X already resident in device memory.  The
value is seconds per path (lower is better).

The same run also reports, each with its own workload description:
  * the X^T rho sweep (the HBM-bound step of every screening pass) on the
    1000 x 100000 FP32 design (400 MB, rotated between two copies so the
    256 MB last-level cache cannot serve it), timed with HIP events recorded
    by the library on the launch stream, against the 8 TB/s HBM peak;
  * the 256-path stability-selection batch (one captured graph) and the
    512-problem uneven batch (autotuned tiles, p50/p99 latency), each beside
    a pool of CPU threads running the oracle on a bounded sample;
  * the whole 100-lambda path of the 1000 x 100000 design (plain warm
    starts) and the learned warm start against it on the first lambdas;
  * the oracle (plain FP64 C, one thread) on the whole 72 x 7129 path.

Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM bytes per launch of the sweep kernel from the FETCH_SIZE and WRITE_SIZE
# counter runs in profiles/k_wide_sweep_c4_hbm_counters.md (scaled by a plain
# copy of known size), valid while the source text of the kernel and of the
# device helpers it uses hashes to SWEEP_SRC_SHA1.
GS_MLP_B3 = 4608  # offset of the network's output bias in the parameter array
SWEEP_TRAFFIC_BYTES = 406.84e6
SWEEP_SRC_SHA1 = "bf45d5958163a52b"
# (file, first marker, end marker): the hashed slices
SWEEP_SRCS = (
    ("paper_1505_03410_amd/csrc/gs_wide.hpp", "// ---- the sweep:", "// ---- gap, stop test"),
    ("paper_1505_03410_amd/csrc/gs_device.hpp", "// ---- cross-lane reductions",
     "// ---- GAP SAFE sphere"),
)


def sweep_src_hash():
    import hashlib
    h = hashlib.sha1()
    for f, a, b in SWEEP_SRCS:
        with open(os.path.join(ROOT, f), encoding="utf-8") as fh:
            t = fh.read()
        i = t.index(a)
        h.update(t[i:t.index(b, i)].encode())
    return h.hexdigest()[:16]


def sweep_traffic():
    return SWEEP_TRAFFIC_BYTES if sweep_src_hash() == SWEEP_SRC_SHA1 else None


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def bench_path(gs, torch, synth, steps, warmup):
    d = synth.c1()
    X, y = d["X"], d["y"]
    Xd = gs.colmajor_to_device(X)
    yd = torch.from_numpy(y).cuda()
    ws = None
    for _ in range(warmup):
        r = gs.lasso_path(Xd, yd, T=100, lambda_min_ratio=1e-3, workspace=ws)
        ws = r["workspace"]
    stats = torch.zeros(len(gs.STAT_NAMES), dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    gs.timing_reset()
    t0 = time.perf_counter()
    for _ in range(steps):
        r = gs.lasso_path(Xd, yd, T=100, lambda_min_ratio=1e-3, workspace=ws, stats=stats)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    path_ms, path_n = gs.timing_query("path")
    st = r["status"].cpu().numpy()
    gap = r["gap"].cpu().numpy()
    yy = float((y.astype("float64") ** 2).sum())
    ok = bool((st == 0).all() and (gap <= 1e-8 * yy).all())
    epochs = int(r["epochs"].sum())
    st = {k: int(v) // steps for k, v in zip(gs.STAT_NAMES, stats.cpu().tolist())}
    return dict(seconds=el / steps, ok=ok, epochs=epochs, path_ms=path_ms / max(path_n, 1),
                path_launches=path_n, n=X.shape[0], p=X.shape[1], stats=st)


def bench_path_learned(gs, torch, synth, params_file, steps):
    """The same c1 path (T = 100, every lambda to gap <= 1e-8 ||y||^2) through
    the learned driver: with the trained network, with the no-entrant network
    (the ablation) and with no network (plain starts, one lambda at a time)."""
    import numpy as np
    d = synth.c1()
    Xd = gs.colmajor_to_device(d["X"])
    yd = torch.from_numpy(d["y"]).cuda()
    yy = float((d["y"].astype(np.float64) ** 2).sum())
    P = torch.from_numpy(np.load(params_file).astype(np.float32)).cuda()
    out = {}
    for name, prm in (("learned", P), ("no_entrant_network", _no_entrant_params(torch, P)),
                      ("plain_starts", None)):
        ws = None
        r = gs.lasso_path_learned(Xd, yd, prm, T=100, lambda_min_ratio=1e-3)
        ws = r["workspace"]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            r = gs.lasso_path_learned(Xd, yd, prm, T=100, lambda_min_ratio=1e-3, workspace=ws)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / steps
        st, gap = r["status"].cpu().numpy(), r["gap"].cpu().numpy()
        out[name] = dict(seconds=round(el, 4), epochs=int(r["epochs"].sum()),
                         certified=bool((st == 0).all() and (gap <= 1e-8 * yy).all()),
                         network_start_lambdas=int(r["learned"].sum()))
    return out


def bench_sweep(gs, torch, d, reps):
    import numpy as np
    X, y = d["X"], d["y"]
    n, p = X.shape
    copies = [gs.colmajor_to_device(X) for _ in range(2)]
    yd = torch.from_numpy(y).cuda()
    beta = torch.zeros(p, dtype=torch.float64, device="cuda")
    lam = 0.5 * float(np.abs(X.astype(np.float64).T @ y.astype(np.float64)).max())
    ws = None
    for i in range(2):
        out = gs.screen(copies[i], yd, beta, lam, workspace=ws)
        ws = out["workspace"]
    torch.cuda.synchronize()
    gs.timing_reset()
    for i in range(reps):
        gs.screen(copies[i % 2], yd, beta, lam, workspace=ws)
    torch.cuda.synchronize()
    ms, cnt = gs.timing_query("sweep")
    avg_s = ms / cnt / 1e3
    # algorithmic bytes of one full sweep: X (4np), beta read and c, ||x_j||^2
    # written (8p each)
    nbytes = 4.0 * n * p + 24.0 * p
    gbs = nbytes / avg_s / 1e9
    return dict(avg_us=avg_s * 1e6, launches=cnt, bytes=nbytes, gbs=gbs, n=n, p=p)


def _latency(gs, ts):
    """Per-problem latency from device wall-clock timestamps (start, end):
    completion minus the earliest start, in ms, as p50 / p99 / max."""
    import numpy as np
    t = ts.cpu().numpy().reshape(-1, 2).astype(np.float64)
    hz = gs.wallclock_hz()
    lat = (t[:, 1] - t[:, 0].min()) / hz * 1e3
    return dict(p50_ms=round(float(np.percentile(lat, 50)), 3),
                p99_ms=round(float(np.percentile(lat, 99)), 3),
                max_ms=round(float(lat.max()), 3))


def bench_c2(gs, torch, synth, reps, cpu_threads=0):
    """256 row subsamples (36 rows) of the c1 design, 100 lambdas each, as one
    graph-captured batch; selection counts on the device."""
    d = synth.c2()
    X, y, rows = d["X"], d["y"], d["rows"]
    Xd = gs.colmajor_to_device(X)
    yd = torch.from_numpy(y).cuda()
    B, T = rows.shape[0], 100
    probs = [dict(X=Xd, y=yd, rows=torch.from_numpy(rows[b]).cuda(), T=T, lambda_min_ratio=1e-2)
             for b in range(B)]
    counts = torch.zeros((T, X.shape[1]), dtype=torch.int32, device="cuda")
    ts = torch.zeros(2 * B, dtype=torch.int64, device="cuda")
    plan = gs.BatchPlan(probs, select_counts=counts, timestamps=ts)
    plan.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        plan.run()
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / reps
    ok = all(bool((o["status"] == 0).all()) for o in plan.outputs)
    lat = _latency(gs, ts)
    plan.close()
    out = dict(seconds=round(el, 4), paths_per_s=round(B / el, 1), certified=ok, **lat,
               workload="c2: 256 row subsamples (36 rows) of 72x7129, T=100, ratio 1e-2, "
                        "one graph-captured batch")
    if cpu_threads:
        import numpy as np
        import oracle
        o = oracle.oracle()
        sample = 32

        def one(b):
            r = o.lasso_path(X[rows[b]], y[rows[b]], T=T, delta=2.0)
            return int(r["status"].max())

        wall, res, _ = _pool(one, range(sample), cpu_threads, None)
        out["cpu"] = dict(value=round(len(res) / wall, 2), unit="paths/s", cores=cpu_threads,
                          kind="oracle", seconds=round(wall, 3), certified=max(res) == 0,
                          sample=f"the first {sample} of the 256 paths on a pool of "
                                 f"{cpu_threads} threads (one path per thread at a time), "
                                 "FP64 C oracle")
    return out


def _cpu_threads():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _pool(fn, items, threads, budget_s):
    """Runs fn over items on a thread pool (the oracle's C calls release the
    GIL).  With budget_s, no new item starts after that many seconds.
    Returns (wall seconds, results, per-item completion times)."""
    import concurrent.futures as cf
    import threading
    t0 = time.perf_counter()
    lock = threading.Lock()
    done = []
    it = iter(items)

    def worker():
        out = []
        while True:
            with lock:
                if budget_s is not None and time.perf_counter() - t0 > budget_s:
                    return out
                try:
                    x = next(it)
                except StopIteration:
                    return out
            r = fn(x)
            out.append((r, time.perf_counter() - t0))

    with cf.ThreadPoolExecutor(threads) as ex:
        futs = [ex.submit(worker) for _ in range(threads)]
        for f in futs:
            done.extend(f.result())
    wall = time.perf_counter() - t0
    return wall, [r for r, _ in done], [t for _, t in done]


def bench_c3(gs, torch, synth, tune, cpu_threads=0, cpu_budget=20.0, max_epochs=1000000):
    """512 independent problems of uneven n, p (one lambda each, cold start).
    The epoch budget is raised above the default 100000: one problem of the
    set (n = 88, p = 9918, lambda = 0.0103 lambda_max) needs 146,700 epochs
    from its cold start, in the oracle as on the device."""
    import concurrent.futures as cf

    import numpy as np
    params = synth.c3_params()
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max(1, cpu_threads or 8)) as ex:
        host = list(ex.map(lambda pr: synth.c3_problem(pr), params))
    _log(f"c3: {len(host)} problems drawn in {time.perf_counter() - t0:.1f} s")
    probs, keep = [], []
    for d in host:
        Xd = gs.colmajor_to_device(d["X"])
        yd = torch.from_numpy(d["y"]).cuda()
        keep.append((Xd, yd))
        probs.append(dict(X=Xd, y=yd, T=1, lambdas=[d["lambda_ratio"]], relative=True))
    _log(f"c3: {len(probs)} problems uploaded")
    tiles = None
    if tune:
        t0 = time.perf_counter()
        # candidates are timed on at most 2000 epochs of each sampled problem:
        # enough to rank the layouts, without solving the slowest problems
        ch = gs.autotune(probs, max_lambdas=1, sample=2, max_epochs=2000)
        tiles = sorted(set(ch))
        _log(f"c3: autotuned in {time.perf_counter() - t0:.1f} s: {len(tiles)} tile choices")
    B = len(probs)
    ts = torch.zeros(2 * B, dtype=torch.int64, device="cuda")
    t0 = time.perf_counter()
    gs.lasso_solve_batch(probs, timestamps=ts, max_epochs=max_epochs)
    torch.cuda.synchronize()
    _log(f"c3: warm-up batch solved in {time.perf_counter() - t0:.1f} s")
    t0 = time.perf_counter()
    outs = gs.lasso_solve_batch(probs, timestamps=ts, max_epochs=max_epochs)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    st = np.array([int(o["status"][0]) for o in outs])
    ep = np.array([int(o["epochs"][0]) for o in outs])
    ok = bool((st == 0).all())
    bad = [dict(n=params[b]["n"], p=params[b]["p"], rho=round(params[b]["rho"], 3),
                lambda_ratio=round(params[b]["lambda_ratio"], 4), status=int(st[b]),
                epochs=int(ep[b])) for b in np.flatnonzero(st != 0)[:8]]
    out = dict(seconds=round(el, 4), problems_per_s=round(B / el, 2), certified=ok, tiles=tiles,
               **_latency(gs, ts),
               status_counts={str(k): int((st == k).sum()) for k in np.unique(st)},
               epochs_median=int(np.median(ep)), epochs_max=int(ep.max()), not_certified=bad,
               max_epochs=max_epochs,
               workload="c3: 512 problems, n log-U[50,2000], p log-U[1000,50000], "
                        "lambda/lambda_max U[0.01,0.5], one lambda each from a cold start, "
                        "autotuned tiles, one batched launch per tile class")
    if cpu_threads:
        import oracle
        o = oracle.oracle()
        order = np.random.default_rng(3).permutation(B)

        def one(b):
            d = host[b]
            t = time.perf_counter()
            r = o.lasso_path(d["X"], d["y"], lambdas=[d["lambda_ratio"]], relative=True,
                             K=max_epochs)
            return int(r["status"][0]), time.perf_counter() - t

        wall, res, fin = _pool(one, order, cpu_threads, cpu_budget)
        solve = np.array([t for _, t in res])
        out["cpu"] = dict(value=round(len(res) / wall, 2), unit="problems/s", cores=cpu_threads,
                          kind="oracle", problems=len(res), seconds=round(wall, 3),
                          certified=all(s_ == 0 for s_, _ in res),
                          solve_p50_ms=round(float(np.percentile(solve, 50)) * 1e3, 3),
                          solve_p99_ms=round(float(np.percentile(solve, 99)) * 1e3, 3),
                          sample=f"a pool of {cpu_threads} threads over the 512 problems in a "
                                 f"seeded random order, no new problem started after "
                                 f"{cpu_budget:g} s: {len(res)} problems solved, FP64 C oracle")
    return out


def _no_entrant_params(torch, P):
    """The trained parameters with the support logit's bias at -1e6: the
    network then predicts no entrant, so the learned driver's working set is
    the previous support grown by the rounds' violators alone (the ablation
    of the network)."""
    Q = P.clone()
    Q[GS_MLP_B3 + 1] = -1e6
    return Q


def bench_c4(gs, torch, d, params_file, piece, nl_plain, nl_learned, seed=4, ablation=True,
             plain=True):
    """The C4 workload (1000 x 100000 FP32, blocks of 50 columns with
    correlation 0.7, the grid of 100 lambdas down to lambda_max/1000, every
    lambda to gap <= 1e-8 ||y||^2): the plain path over the first `nl_plain`
    lambdas (the whole grid by default), the learned warm start over the
    first `nl_learned`, and the learned driver with a network that predicts
    no entrant (the ablation), compared on those.  All run in pieces of
    `piece` lambdas (each warm-started from the previous piece's last
    solution) so that progress shows; the learned time includes the block
    correlations, features, inference, the restricted solves and the extra
    gap checks."""
    import numpy as np
    Xd = gs.colmajor_to_device(d["X"])
    yd = torch.from_numpy(d["y"]).cuda()
    yy = float((d["y"].astype(np.float64) ** 2).sum())
    rel = 1e-3 ** (np.arange(100) / 99)
    P = None
    if params_file:
        P = torch.from_numpy(np.load(params_file).astype(np.float32)).cuda()
    stats = torch.zeros(len(gs.STAT_NAMES), dtype=torch.int64, device="cuda")

    def run(name, learned, nl, params=None):
        prev, ws, res, marks = None, None, [], []
        torch.cuda.synchronize()
        stats.zero_()
        gs.timing_reset()
        t0 = time.perf_counter()
        for k in range(0, nl, piece):
            sub = rel[k:min(k + piece, nl)]
            if learned:
                r = gs.lasso_path_learned(Xd, yd, params, lambdas=sub, relative=True,
                                          beta_init=prev, workspace=ws)
            else:
                r = gs.lasso_path(Xd, yd, lambdas=sub, relative=True, beta_init=prev,
                                  workspace=ws, stats=stats)
            ws = r["workspace"]
            prev = r["beta"][-1].contiguous()
            ep = r["epochs"].cpu().numpy()
            res.append(r)
            marks.append(time.perf_counter() - t0)
            _log(f"c4 {name}: lambdas {k}..{k + len(sub) - 1} epochs {int(ep.sum())} "
                 f"at {marks[-1]:.1f} s")
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        cat = lambda key: np.concatenate([x[key].cpu().numpy() for x in res])
        st, gap, ep = cat("status"), cat("gap"), cat("epochs")
        out = dict(seconds=round(el, 3), epochs=int(ep.sum()),
                   certified=bool((st == 0).all() and (gap <= 1e-8 * yy).all()),
                   epochs_per_lambda=[int(e) for e in ep],
                   seconds_at_piece_end=[round(m, 3) for m in marks])
        if learned:
            fl = cat("learned")
            out["network_start_fraction"] = round(float(fl[1:].mean()), 3)
            out["network_start_lambdas"] = int(fl.sum())
        else:
            sv = dict(zip(gs.STAT_NAMES, stats.cpu().tolist()))
            cd_ms, cd_n = gs.timing_query("cd")
            out["cd"] = dict(kernel="k_wide_walk", bound="latency", passes=sv["passes"],
                             exact_visits=sv["wide_visits"], rounds=sv["wide_rounds"],
                             reanchors=sv["wide_stops"], walk_ms=round(cd_ms, 1),
                             us_per_visit=round(cd_ms * 1e3 / max(sv["wide_visits"], 1), 4))
        return out

    plain = run("plain", False, nl_plain) if plain and nl_plain > 0 else None
    res = {"workload": "c4: n=1000 p=100000 FP32, 2000 blocks of 50 columns with "
                       "correlation 0.7, 50-sparse truth, SNR 5, seed %d; lambdas of the "
                       "T=100 grid lambda_max..lambda_max/1000, eps=1e-8||y||^2; plain path "
                       "over lambdas 0..%d, learned start over lambdas 0..%d" %
                       (seed, nl_plain - 1, nl_learned - 1),
           "piece": piece, "plain_lambdas": nl_plain, "learned_lambdas": nl_learned,
           "plain": plain}
    if P is not None and nl_learned > 0:
        lr = run("learned", True, nl_learned, P)
        res["learned"] = lr
        res["params"] = os.path.relpath(params_file, ROOT)
        if ablation:
            res["no_entrant_network"] = run("no-entrant network", True, nl_learned,
                                            _no_entrant_params(torch, P))
        # the plain path's time and epochs over the same lambdas
        npc = (nl_learned + piece - 1) // piece
        if plain is not None and nl_learned % piece == 0 and \
                npc <= len(plain["seconds_at_piece_end"]):
            ps = plain["seconds_at_piece_end"][npc - 1]
            res["plain_same_lambdas"] = dict(
                seconds=ps, epochs=int(sum(plain["epochs_per_lambda"][:nl_learned])))
            res["speedup_learned_vs_plain"] = round(ps / max(lr["seconds"], 1e-9), 2)
    return res


def bench_learned_eval(gs, torch, synth, params_file, seeds, nl_plain, piece=10):
    """Held-out evaluation of the learned start at the full C4 size: for each
    seed, the learned path over the whole 100-lambda grid and the plain path
    over its first `nl_plain` lambdas, every lambda certified; reported per
    seed with the learned time at `nl_plain` lambdas beside the plain one."""
    rows = []
    for sd in seeds:
        d = synth.c4(seed=sd)
        _log(f"learned eval: seed {sd}")
        r = bench_c4(gs, torch, d, params_file, piece, nl_plain, 100, seed=sd, ablation=False)
        lr, pl = r["learned"], r["plain"]
        k = nl_plain // piece
        rows.append(dict(seed=sd, learned_seconds=lr["seconds"], learned_epochs=lr["epochs"],
                         learned_certified=lr["certified"],
                         network_start_lambdas=lr["network_start_lambdas"],
                         learned_seconds_first=lr["seconds_at_piece_end"][k - 1],
                         learned_epochs_first=int(sum(lr["epochs_per_lambda"][:nl_plain])),
                         plain_seconds_first=pl["seconds"], plain_epochs_first=pl["epochs"],
                         plain_certified=pl["certified"]))
        del d
    return dict(workload="c4 1000x100000 FP32 held-out seeds; learned: all 100 lambdas; "
                         "plain and learned compared on the first %d" % nl_plain,
                seeds=list(seeds), rows=rows)


def bench_screening(gs, torch, synth, Ks=(10, 50, 200)):
    """The proportion of active variables against lambda and the epoch budget
    K (the paper's Fig. 3, on the 72 x 7129 workload): for every rule and K,
    a 100-lambda path (down to lambda_max/1000, warm starts) whose lambdas
    each stop after K epochs or at gap <= 1e-8 ||y||^2; reported is |A|/p at
    the exit of every lambda (wide schedule, so every rule runs the same
    kernels)."""
    import numpy as np
    d = synth.c1()
    Xd = gs.colmajor_to_device(d["X"])
    yd = torch.from_numpy(d["y"]).cuda()
    p = d["X"].shape[1]
    rules = ["sphere", "dome", "static", "dynamic_safe", "st3"]
    out = {"workload": "c1 72x7129, T=100 grid lambda_max..lambda_max/1000, warm starts, "
                       "at most K epochs per lambda; |A|/p at each lambda's exit",
           "K": list(Ks), "lambda_ratio": [round(float(1e-3 ** (t / 99)), 6) for t in range(100)],
           "proportion": {}}
    t0 = time.perf_counter()
    for rule in rules:
        out["proportion"][rule] = {}
        for K in Ks:
            r = gs.lasso_path(Xd, yd, T=100, lambda_min_ratio=1e-3, max_epochs=K, rule=rule,
                              schedule="wide")
            na = r["nactive"].cpu().numpy()
            out["proportion"][rule][str(K)] = [round(float(v) / p, 4) for v in na]
    out["seconds"] = round(time.perf_counter() - t0, 2)
    # lambdas (of 100) at which each rule keeps under half of the columns,
    # at the largest K
    kmax = str(Ks[-1])
    out["lambdas_below_half"] = {r: int((np.array(out["proportion"][r][kmax]) < 0.5).sum())
                                 for r in rules}
    return out


def copy_calibration(torch, mb, reps):
    """A plain device copy of known size, for scaling the HBM byte counters."""
    nel = int(mb * 1e6) // 4
    a = torch.ones(nel, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    _log(f"copy: {reps} x {nel * 4} bytes")


def cpu_baseline(synth, reps):
    import numpy as np
    import oracle
    d = synth.c1()
    o = oracle.oracle()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        r = o.lasso_path(d["X"], d["y"], T=100, delta=3.0, eps_rel=1e-8)
        ts.append(time.perf_counter() - t0)
    assert r["status"].max() == 0
    return dict(value=float(np.median(ts)), reps=reps)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--sweep-reps", type=int, default=20)
    ap.add_argument("--cpu-reps", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--no-path", action="store_true")
    ap.add_argument("--no-c2", action="store_true")
    ap.add_argument("--no-c3", action="store_true", help="skip the 512-problem uneven batch")
    ap.add_argument("--no-tune", action="store_true", help="no autotuning before the c3 batch")
    ap.add_argument("--no-c4", action="store_true",
                    help="skip the 1000 x 100000 path and the learned warm start")
    ap.add_argument("--c4-params", default=os.path.join(ROOT, "paper_1505_03410_amd",
                                                        "warm_mlp.npy"))
    ap.add_argument("--c4-piece", type=int, default=10)
    ap.add_argument("--c4-lambdas", type=int, default=100,
                    help="lambdas of the 100-point c4 grid solved by the plain path")
    ap.add_argument("--c4-learned-lambdas", type=int, default=100,
                    help="lambdas solved by the learned warm start (0: none)")
    ap.add_argument("--no-screening", action="store_true",
                    help="skip the screening-proportion comparison of the safe rules")
    ap.add_argument("--cpu-budget", type=float, default=20.0,
                    help="seconds of the c3 CPU pool sample")
    ap.add_argument("--copy-mb", type=float, default=0.0,
                    help="only run a plain device copy of this many MB (counter calibration)")
    ap.add_argument("--learned-eval", default="",
                    help="only evaluate the learned start on these c4 seeds (e.g. 4,20000-20009)")
    ap.add_argument("--eval-plain-lambdas", type=int, default=70,
                    help="lambdas of the plain path in the learned evaluation")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {a.gpus}); the library solves "
              "independent problems per GPU and has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1505_03410_amd as gs
    import synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if a.copy_mb > 0:
        copy_calibration(torch, a.copy_mb, 5)
        return
    gs.load_library()
    if a.learned_eval:
        seeds = []
        for part in a.learned_eval.split(","):
            lo, _, hi = part.partition("-")
            seeds += list(range(int(lo), int(hi or lo) + 1))
        ev = bench_learned_eval(gs, torch, synth, a.c4_params, seeds, a.eval_plain_lambdas)
        print(json.dumps({"learned_eval": ev}), flush=True)
        return
    gs.timing_enable(True)
    path = None
    if not a.no_path:
        _log("path: c1 72x7129, 100 lambdas")
        path = bench_path(gs, torch, synth, a.steps, a.warmup)
        _log(f"path: {path['seconds']:.4f} s/path, ok={path['ok']}")
        if a.c4_params and os.path.exists(a.c4_params):
            path["learned_driver"] = bench_path_learned(gs, torch, synth, a.c4_params, a.steps)
            _log(f"path, learned start: {path['learned_driver']['learned']['seconds']:.4f} s/path")
    roof = None
    sweep = None
    d4 = None
    if not a.no_sweep or not a.no_c4:
        d4 = synth.c4()
    if not a.no_sweep:
        _log("sweep: c4 1000x100000 FP32 (400 MB), two rotating copies")
        sweep = bench_sweep(gs, torch, d4, a.sweep_reps)
        _log(f"sweep: {sweep['avg_us']:.1f} us, {sweep['gbs']:.0f} GB/s")
        roof = {"bound": "hbm", "kernel": "k_wide_sweep<float,4,4,1>",
                "achieved": round(sweep["gbs"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(sweep["gbs"] / HBM_PEAK_GBS, 4), "traffic": sweep_traffic(),
                "bytes_per_launch": sweep["bytes"], "avg_us": round(sweep["avg_us"], 2),
                "launches": sweep["launches"], "workload": "1000x100000 FP32 full sweep"}
    threads = 0 if a.no_cpu else _cpu_threads()
    c2 = None
    if not a.no_c2:
        _log("c2: 256 row subsamples, graph-captured batch")
        c2 = bench_c2(gs, torch, synth, 3, threads)
        _log(f"c2: {c2['seconds']:.3f} s, {c2['paths_per_s']} paths/s, p99 {c2['p99_ms']} ms")
    c3 = None
    if not a.no_c3:
        _log("c3: 512 uneven problems")
        c3 = bench_c3(gs, torch, synth, not a.no_tune, threads, a.cpu_budget)
        _log(f"c3: {c3['seconds']:.3f} s, p50 {c3['p50_ms']} ms, p99 {c3['p99_ms']} ms")
    c4 = None
    if not a.no_c4:
        _log("c4: 1000x100000 path, plain and learned warm starts")
        pf = a.c4_params if a.c4_params and os.path.exists(a.c4_params) else None
        c4 = bench_c4(gs, torch, d4, pf, a.c4_piece, a.c4_lambdas, a.c4_learned_lambdas)
    scr = None
    if not a.no_screening:
        _log("screening proportion: five safe rules on the c1 path")
        scr = bench_screening(gs, torch, synth)
        _log(f"screening: {scr['seconds']} s, lambdas under half active "
             f"{scr['lambdas_below_half']}")
    cpu = None
    if not a.no_cpu:
        _log("cpu baseline: oracle, whole c1 path")
        cb = cpu_baseline(synth, a.cpu_reps)
        cpu = {"value": round(cb["value"], 4), "unit": "s", "cores": 1, "kind": "oracle",
               "sample": f"whole c1 path (100 lambdas), median of {cb['reps']} runs, "
                         "FP64 C oracle, one thread"}
    if path is None:
        print(json.dumps({"roofline": roof, "batched": {"c2": c2, "c3": c3},
                          "learned_warm_start": c4, "screening_proportion": scr}), flush=True)
        return
    line = {
        "metric": "Lasso path seconds to gap\u22641e-8\u2016y\u2016\u00b2; X\u1d40\u03b8 HBM GB/s; "
                  "learned vs plain warm start",
        "value": round(path["seconds"], 5),
        "unit": "s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(path["seconds"] * 1e3, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "c1: lasso path, n=72 p=7129 FP32 X, AR(1) rho=0.5, "
                               "T=100 lambda_max..lambda_max/1000, f=10, eps=1e-8||y||^2",
                   "n": path["n"], "p": path["p"], "T": 100, "lambda_min_ratio": 1e-3,
                   "screen_every": 10, "eps_rel": 1e-8, "parallelism": "single problem, one wavefront",
                   "arithmetic": "FP32 X, Gram block and pattern-mode updates; FP64 residual, "
                                 "coefficients, reductions, gap and radius"},
        "certified": path["ok"],
        "path_kernel": {"kernel": "k_path_narrow", "bound": "latency",
                        "avg_ms": round(path["path_ms"], 3), "launches": path["path_launches"],
                        "epochs_per_path": path["epochs"],
                        "epochs_per_s": round(path["epochs"] / path["seconds"], 1),
                        "counters_per_path": path["stats"]},
        "roofline": roof,
        "cpu_baseline": cpu,
        "batched": {"c2": c2, "c3": c3},
        "learned_warm_start": {"c1": path.get("learned_driver"), "c4": c4},
        "screening_proportion": scr,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
