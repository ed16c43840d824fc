"""Trains the warm-start network on the device and writes its parameters.

Training problems have the block-equicorrelated structure of the C4
workload (blocks of 50 columns, within-block correlation 0.7, unit columns,
50 signed unit coefficients, SNR 5) at a reduced width p (the network's
inputs are scale-free), seeds 10000, 10001, ...  Each problem's plain path
(100 lambdas down to lambda_max / 1000) is solved with lasso_solve_batch;
then for every lambda_t, t >= 1, a screening pass at beta^{lambda_{t-1}}
gives the safe set A_plain and c = X^T (y - X beta^{lambda_{t-1}}), and every
j in A_plain yields one example: inputs u_j (gs_warm_features) and targets
((beta^{lambda_t}_j - beta^{lambda_{t-1}}_j) ||x_j||^2 / lambda_t,
1[beta^{lambda_t}_j != 0], mask 1).  The
network is then fitted with device Adam steps on random minibatches; the
last problems are held out for a validation loss.

  python -m paper_1505_03410_amd.train_warm --problems 64 --p 10000 \\
      --out paper_1505_03410_amd/warm_mlp.npy
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def _log(*a):
    print(*a, flush=True)


def solve_paths_in_pieces(gs, torch, probs, T, ratio, piece, nl=None, log=_log):
    """Plain paths of a batch of problems over the first nl (default T) of
    the lambdas lambda_t = lambda_max ratio^(t/(T-1)), solved `piece` lambdas
    at a time (each piece warm-started from the previous one's last
    solution), so that progress is visible.  Returns per problem
    (betas (nl, p), lambdas (nl,))."""
    rel = ratio ** (np.arange(T) / (T - 1))
    rel = rel[:nl or T]
    T = len(rel)
    dev = probs[0]["X"].device
    betas = [torch.empty((T, pb["X"].shape[1]), dtype=torch.float64, device=dev) for pb in probs]
    lams = [torch.empty(T, dtype=torch.float64, device=dev) for _ in probs]
    prev = [None] * len(probs)
    t0 = time.time()
    for k in range(0, T, piece):
        sub = rel[k:k + piece]
        outs = gs.lasso_solve_batch([dict(X=pb["X"], y=pb["y"], lambdas=sub, relative=True,
                                          beta_init=prev[b]) for b, pb in enumerate(probs)])
        torch.cuda.synchronize()
        st = max(int(o["status"].max()) for o in outs)
        ep = sum(int(o["epochs"].sum()) for o in outs)
        log(f"  lambdas {k}..{k + len(sub) - 1}: {ep} epochs, status max {st}, "
            f"{time.time() - t0:.1f} s")
        for b, o in enumerate(outs):
            betas[b][k:k + len(sub)] = o["beta"]
            lams[b][k:k + len(sub)] = o["lambdas"]
            prev[b] = o["beta"][-1].contiguous()
    return list(zip(betas, lams))


def make_examples(gs, torch, synth, seeds, p, n=1000, T=100, ratio=1e-3, block=50, piece=5,
                  nl=None):
    """Per seed, the examples (U rows, target rows) of its plain path."""
    dev = torch.device("cuda")
    probs, host = [], []
    for s in seeds:
        d = synth.c4(seed=s, n=n, p=p, block=block)
        X = d["X"]
        Xd = gs.colmajor_to_device(X)
        yd = torch.from_numpy(np.ascontiguousarray(d["y"])).to(dev)
        probs.append(dict(X=Xd, y=yd))
        host.append((np.sum(X.astype(np.float64) ** 2, axis=0),
                     float(np.linalg.norm(d["y"].astype(np.float64)))))
    sols = solve_paths_in_pieces(gs, torch, probs, T, ratio, piece, nl)
    per = []
    for pb, (B, lam_d), (nrm2, ynorm) in zip(probs, sols, host):
        Us, Ts = [], []
        lam = lam_d.cpu().numpy()
        bmc = gs.block_corr(pb["X"], block)
        nrm2_d = torch.from_numpy(nrm2).to(dev)
        for t in range(1, len(lam)):
            sc = gs.screen(pb["X"], pb["y"], B[t - 1].contiguous(), float(lam[t]))
            q = int(sc["q"].item())
            if q == 0:
                continue
            U = gs.warm_features(sc["c"].contiguous(), B[t - 1].contiguous(), nrm2_d, bmc,
                                 float(lam[t]), float(lam[0]), ynorm)
            act = sc["active"][:q].long()
            bt = B[t][act]
            dt = (bt - B[t - 1][act]) * nrm2_d[act] / float(lam[t])
            tg = torch.stack([dt, (bt != 0).double(), torch.ones_like(bt)], dim=1).float()
            Us.append(U[act])
            Ts.append(tg)
        per.append((torch.cat(Us), torch.cat(Ts)))
    return per


def init_params(rng):
    """He-style initialisation of the 4 -> 64 -> 64 -> 2 network."""
    return dict(W1=rng.normal(0, np.sqrt(2 / 4), (64, 4)), b1=np.zeros(64),
                W2=rng.normal(0, np.sqrt(2 / 64), (64, 64)), b2=np.zeros(64),
                W3=rng.normal(0, np.sqrt(1 / 64), (2, 64)), b3=np.zeros(2))


def train(gs, torch, U, Tg, Uv, Tv, steps, batch, lr, seed=0):
    rng = np.random.default_rng(seed)
    flat = gs.mlp_params_to_flat(init_params(rng))
    mom, vel = torch.zeros_like(flat), torch.zeros_like(flat)
    loss = torch.empty(1, dtype=torch.float32, device=flat.device)
    gen = torch.Generator(device=flat.device)
    gen.manual_seed(seed)
    m = U.shape[0]
    ws = None
    hist = []
    for t in range(1, steps + 1):
        idx = torch.randint(0, m, (min(batch, m),), device=flat.device, generator=gen)
        # cosine decay of the step size
        lr_t = lr * 0.5 * (1 + np.cos(np.pi * (t - 1) / steps))
        ws = gs.mlp_train_step(flat, mom, vel, t, float(lr_t), U[idx].contiguous(),
                               Tg[idx].contiguous(), loss, workspace=ws)
        if t % max(1, steps // 10) == 0 or t == steps:
            _, vl = gs.mlp_grad(flat, Uv, Tv)
            hist.append((t, float(loss.item()), float(vl.item())))
            _log(f"  step {t}: train loss {hist[-1][1]:.5f}  validation loss {hist[-1][2]:.5f}")
    return flat, hist


def entrant_scores(gs, torch, flat, Uv, Tv):
    """Validation scores of the support logit on the entrants (features with
    beta_prev = 0, the third input): precision and recall of logit > 0
    against the support at lambda_t, and the BCE-plus-MSE validation loss."""
    out = torch.cat([gs.mlp_forward(flat, Uv[i:i + (1 << 22)].contiguous())
                     for i in range(0, Uv.shape[0], 1 << 22)])
    fresh = Uv[:, 2] == 0
    pred = (out[:, 1] > 0) & fresh
    tgt = (Tv[:, 1] > 0.5) & fresh
    tp = float((pred & tgt).sum())
    _, vl = gs.mlp_grad(flat, Uv, Tv)
    return dict(validation_loss=float(vl.item()),
                entrant_precision=tp / max(float(pred.sum()), 1.0),
                entrant_recall=tp / max(float(tgt.sum()), 1.0),
                entrants=int(tgt.sum()), candidates=int(fresh.sum()))


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--problems", type=int, default=64)
    ap.add_argument("--holdout", type=int, default=8, help="last seeds kept for validation (>= 1)")
    ap.add_argument("--p", type=int, default=10000)
    ap.add_argument("--chunk", type=int, default=32, help="problems solved per batch")
    ap.add_argument("--lambdas", type=int, default=60,
                    help="lambdas of the 100-point grid (lambda_max..lambda_max/1000) used")
    ap.add_argument("--steps", type=int, default=6000)
    ap.add_argument("--batch", type=int, default=65536)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--first-seed", type=int, default=10000)
    ap.add_argument("--out", default=os.path.join(HERE, "warm_mlp.npy"))
    ap.add_argument("--curve", default="",
                    help="comma-separated training-set sizes: one network per size (the first "
                         "k training problems), scored on the same held-out problems; writes "
                         "the table to --curve-out instead of training --out")
    ap.add_argument("--curve-out", default="warm_mlp_curve.json")
    a = ap.parse_args(argv)
    if not 1 <= a.holdout < a.problems:
        raise SystemExit("--holdout must be between 1 and --problems - 1")
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import torch
    import synth
    import paper_1505_03410_amd as gs
    if not torch.cuda.is_available():
        raise SystemExit("training runs on the GPU")
    gs.load_library()
    seeds = list(range(a.first_seed, a.first_seed + a.problems))
    per = []
    for i in range(0, len(seeds), a.chunk):
        _log(f"examples from seeds {seeds[i]}..{seeds[min(i + a.chunk, len(seeds)) - 1]}")
        per += make_examples(gs, torch, synth, seeds[i:i + a.chunk], a.p, nl=a.lambdas)
    ntrain = a.problems - a.holdout
    Utr = torch.cat([u for u, _ in per[:ntrain]])
    Ttr = torch.cat([t for _, t in per[:ntrain]])
    Uv = torch.cat([u for u, _ in per[ntrain:]])
    Tv = torch.cat([t for _, t in per[ntrain:]])
    _log(f"{Utr.shape[0]} training and {Uv.shape[0]} validation examples; "
         f"support fraction {float(Ttr[:, 1].mean()):.3f}")
    if a.curve:
        rows = []
        for k in [int(v) for v in a.curve.split(",")]:
            if not 1 <= k <= ntrain:
                raise SystemExit(f"curve size {k} outside 1..{ntrain}")
            Uk = torch.cat([u for u, _ in per[:k]])
            Tk = torch.cat([t for _, t in per[:k]])
            _log(f"curve: {k} training problems, {Uk.shape[0]} examples")
            flat, hist = train(gs, torch, Uk, Tk, Uv, Tv, a.steps, a.batch, a.lr)
            row = dict(problems=k, examples=int(Uk.shape[0]), train_loss=hist[-1][1])
            row.update(entrant_scores(gs, torch, flat, Uv, Tv))
            _log(f"curve: {row}")
            rows.append(row)
            del Uk, Tk
        meta = dict(holdout=a.holdout, p=a.p, n=1000, lambdas=a.lambdas, steps=a.steps,
                    batch=a.batch, lr=a.lr, first_seed=a.first_seed,
                    validation_examples=int(Uv.shape[0]), rows=rows)
        with open(a.curve_out, "w") as f:
            json.dump(meta, f, indent=1)
        _log(f"wrote {a.curve_out}")
        return
    t0 = time.time()
    flat, hist = train(gs, torch, Utr, Ttr, Uv, Tv, a.steps, a.batch, a.lr)
    torch.cuda.synchronize()
    _log(f"trained in {time.time() - t0:.1f} s")
    np.save(a.out, flat.cpu().numpy().astype(np.float32))
    meta = dict(problems=a.problems, holdout=a.holdout, p=a.p, n=1000, T=100, lambdas=a.lambdas,
                lambda_min_ratio=1e-3, first_seed=a.first_seed, steps=a.steps, batch=a.batch,
                lr=a.lr, examples=int(Utr.shape[0]), validation_examples=int(Uv.shape[0]),
                history=hist)
    with open(os.path.splitext(a.out)[0] + ".json", "w") as f:
        json.dump(meta, f, indent=1)
    _log(f"wrote {a.out}")


if __name__ == "__main__":
    main()
