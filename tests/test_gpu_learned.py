"""GPU parity of the learned warm start: block max correlation, network
inputs, inference (BF16 matrix-core second layer), training gradients and
the Adam step against the NumPy oracle, and the learned path against the
certification bounds of the plain one.

Tolerances.  FP32 accumulation of a length-k sum is off by at most
gamma_k = k u / (1 - k u) (u = 2^-24) times the sum of the absolute terms.
Networks built from short dyadic numbers make every BF16 rounding exact and
every hidden value exact in FP32, so the device and the oracle take the same
ReLU and rounding decisions and differ only by that accumulation bound.  For
general weights a first-hidden-layer value may round to the neighbouring
BF16 number on one side only (the value itself carries FP32 error); the
forward tolerance then adds one BF16 step (2^-7 relative) on every entry of
h1, propagated through |W3| |W2|.
"""
import numpy as np
import pytest

import oracle as O
import paper_1505_03410_amd as gs
import synth
from test_gpu_parity import _check_path, _dev, _np

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def _gamma(k):
    return k * U32 / (1 - k * U32)


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    gs.load_library()
    return torch


def _dyadic_params(rng):
    """Weights with at most 4 significant bits and small exponent ranges: BF16
    exact, and with dyadic inputs every hidden pre-activation is exact in
    FP32 (and in FP64)."""
    return dict(W1=rng.integers(-2, 3, (64, 4)) / 16.0, b1=rng.integers(-8, 9, 64) / 64.0,
                W2=rng.integers(-8, 9, (64, 64)) / 128.0, b2=rng.integers(-8, 9, 64) / 64.0,
                W3=rng.integers(-8, 9, (2, 64)) / 64.0, b3=rng.integers(-8, 9, 2) / 16.0)


def _dyadic_inputs(rng, m):
    return rng.integers(-8, 9, (m, 4)) / 8.0


def _random_params(rng):
    return dict(W1=rng.normal(0, 0.6, (64, 4)), b1=rng.normal(0, 0.1, 64),
                W2=rng.normal(0, 0.15, (64, 64)), b2=rng.normal(0, 0.1, 64),
                W3=rng.normal(0, 0.15, (2, 64)), b3=rng.normal(0, 0.1, 2))


def _as_f32(params):
    return {k: np.asarray(v, np.float32).astype(np.float64) for k, v in params.items()}


def _targets(rng, m):
    return np.stack([rng.normal(0, 0.5, m), (rng.uniform(size=m) < 0.4).astype(np.float64),
                     (rng.uniform(size=m) < 0.7).astype(np.float64)], axis=1)


def _t32(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


# ------------------------------------------------------------ block corr

@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_block_corr_matches_oracle(torch, dtype):
    """C4-style blocks (equicorrelated, unit columns) with a ragged last
    block, a zero column and a block of one column; block widths 50 and 64."""
    d = synth.c4(seed=7, n=200, p=1037, block=50)
    X = d["X"].astype(dtype)
    X[:, 3] = 0.0
    for block in (50, 64, 1037 % 64 or 64):
        got = _np(gs.block_corr(_dev(torch, X, d["y"].astype(dtype))[0], block))
        want = O.block_max_corr(X.astype(np.float64), block)
        n = X.shape[0]
        tol = 2 * _gamma(n + 2) + 4 * U32
        assert np.max(np.abs(got - want)) <= tol, (block, np.max(np.abs(got - want)))
        assert got[3] == 0.0
    # a last block of exactly one column
    got = _np(gs.block_corr(_dev(torch, X[:, :1001], d["y"].astype(dtype))[0], 50))
    assert got[1000] == 0.0
    # equicorrelation 0.7 within blocks shows in the values
    assert 0.55 < np.median(got[:1000]) < 0.9


def test_block_corr_full_c4_sampled(torch):
    """Full-size C4 design (1000 x 100000 FP32): 40 sampled blocks against
    the oracle."""
    d = synth.c4()
    X = d["X"]
    Xd, _ = _dev(torch, X, d["y"])
    got = _np(gs.block_corr(Xd, 50))
    rng = np.random.default_rng(0)
    tol = 2 * _gamma(1002) + 4 * U32
    for b in rng.choice(2000, 40, replace=False):
        sl = slice(50 * b, 50 * b + 50)
        want = O.block_max_corr(X[:, sl].astype(np.float64), 50)
        assert np.max(np.abs(got[sl] - want)) <= tol, b


# -------------------------------------------------------------- features

def test_warm_features_match_oracle(torch):
    rng = np.random.default_rng(1)
    p = 777
    c = rng.normal(0, 3, p)
    bprev = np.where(rng.uniform(size=p) < 0.2, rng.normal(0, 1, p), 0.0)
    nrm2 = rng.uniform(0.5, 2.0, p)
    bmc = rng.uniform(0, 1, p).astype(np.float32)
    lam, lmax, yn = 1.7, 9.3, 4.1
    f64 = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()
    got = _np(gs.warm_features(f64(c), f64(bprev), f64(nrm2), _t32(torch, bmc), lam, lmax, yn))
    want = O.warm_features(c, lam, lmax, bprev, np.sqrt(nrm2), yn, bmc.astype(np.float64))
    # FP64 on both sides, then one rounding to FP32
    np.testing.assert_allclose(got, want.astype(np.float32), rtol=2 * U32 * 2, atol=0)


# --------------------------------------------------------------- forward

@pytest.mark.parametrize("m", [1, 64, 5 * 64 + 37])
def test_mlp_forward_dyadic_exact_decisions(torch, m):
    rng = np.random.default_rng(10 + m)
    P = _dyadic_params(rng)
    U = _dyadic_inputs(rng, m)
    got = _np(gs.mlp_forward(gs.mlp_params_to_flat(P), _t32(torch, U))).astype(np.float64)
    want, cache = O.mlp_forward_bf16(P, U)
    h2 = cache[4]
    scale = np.abs(h2) @ np.abs(P["W3"]).T + np.abs(P["b3"])
    assert np.all(np.abs(got - want) <= _gamma(66) * scale + 1e-30)


def test_mlp_forward_general_weights(torch):
    rng = np.random.default_rng(3)
    m = 11 * 64 + 5
    P = _as_f32(_random_params(rng))
    U = rng.normal(0, 1, (m, 4)).astype(np.float32).astype(np.float64)
    got = _np(gs.mlp_forward(gs.mlp_params_to_flat(P), _t32(torch, U))).astype(np.float64)
    want, cache = O.mlp_forward_bf16(P, U)
    Pb = O.bf16_params(P)
    h1, h2 = cache[2], cache[4]
    A3, A2 = np.abs(Pb["W3"]), np.abs(Pb["W2"])
    acc = (_gamma(70) * (np.abs(h2) @ A3.T + (np.abs(h1) @ A2.T + np.abs(Pb["b2"])) @ A3.T)
           + np.abs(Pb["b3"]) * U32)
    # one-sided BF16 rounding of h1, or a ReLU kink within the FP32 error of
    # the first layer
    z_err = _gamma(6) * (np.abs(U) @ np.abs(Pb["W1"]).T + np.abs(Pb["b1"]))
    flip = ((2.0 ** -7 * np.abs(h1) + z_err) @ A2.T) @ A3.T
    err = np.abs(got - want)
    assert np.all(err <= acc + flip + 1e-30)
    # all but a handful of outputs agree to the accumulation bound alone
    assert np.mean(err <= 4 * acc + 1e-30) >= 0.98


# -------------------------------------------------------------- training

def test_mlp_grad_matches_oracle_backward(torch):
    rng = np.random.default_rng(4)
    m = 9 * 64 + 21
    P = _dyadic_params(rng)
    U = _dyadic_inputs(rng, m)
    tg = _targets(rng, m)
    tg[:, 0] = rng.integers(-8, 9, m) / 8.0
    g, loss = gs.mlp_grad(gs.mlp_params_to_flat(P), _t32(torch, U), _t32(torch, tg))
    g = gs.mlp_flat_to_params(g)
    Pb = O.bf16_params(P)
    out, cache = O.mlp_forward_bf16(P, U)
    want = O.mlp_backward(Pb, cache, out, tg[:, 0], tg[:, 1], tg[:, 2])
    L = O.mlp_loss(out, tg[:, 0], tg[:, 1], tg[:, 2])
    assert abs(float(_np(loss)[0]) - L) <= 1e-5 * (abs(L) + 1)
    for k in want:
        s = np.max(np.abs(want[k])) + 1e-30
        assert np.max(np.abs(g[k] - want[k])) <= 2e-5 * s, k
    # a transposed W2 gradient or a dropped mask would be far outside this
    assert np.max(np.abs(g["W2"] - want["W2"].T)) > 1e-3 * np.max(np.abs(want["W2"]))


def test_mlp_grad_general_weights_direction(torch):
    """Realistic weights: per layer the device gradient is the oracle's up to
    rare one-sided BF16 and ReLU decisions (cosine > 0.999)."""
    rng = np.random.default_rng(5)
    m = 40 * 64
    P = _as_f32(_random_params(rng))
    U = rng.normal(0, 1, (m, 4)).astype(np.float32).astype(np.float64)
    tg = _targets(rng, m)
    g, loss = gs.mlp_grad(gs.mlp_params_to_flat(P), _t32(torch, U), _t32(torch, tg))
    g = gs.mlp_flat_to_params(g)
    out, cache = O.mlp_forward_bf16(P, U)
    want = O.mlp_backward(O.bf16_params(P), cache, out, tg[:, 0], tg[:, 1], tg[:, 2])
    for k in want:
        a, b = g[k].ravel(), want[k].ravel()
        cos = a @ b / (np.linalg.norm(a) * np.linalg.norm(b) + 1e-300)
        assert cos > 0.999, (k, cos)
    L = O.mlp_loss(out, tg[:, 0], tg[:, 1], tg[:, 2])
    assert abs(float(_np(loss)[0]) - L) <= 1e-3 * abs(L)


def test_adam_matches_oracle(torch):
    """Three Adam steps from oracle-made gradients (FP32 inputs on both
    sides); the update of each step is at most lr, the FP32 error of the
    moments a few ulps of it."""
    rng = np.random.default_rng(6)
    P0 = _as_f32(_random_params(rng))
    flat = gs.mlp_params_to_flat(P0)
    mom = torch.zeros_like(flat)
    vel = torch.zeros_like(flat)
    ref = {k: v.copy() for k, v in P0.items()}
    st = {}
    lr = 1e-2
    for t in range(1, 4):
        G = {k: rng.normal(0, 10.0 ** rng.integers(-4, 1), v.shape).astype(np.float32).astype(np.float64)
             for k, v in P0.items()}
        gs.mlp_adam(flat, mom, vel, gs.mlp_params_to_flat(G), t, lr)
        O.adam_step(ref, G, st, lr=lr)
    got = gs.mlp_flat_to_params(flat)
    for k in ref:
        tol = 3 * lr * 1e-5 + 4 * U32 * np.abs(ref[k]) * 3
        assert np.all(np.abs(got[k] - ref[k]) <= tol), k


def test_train_step_equals_grad_then_adam(torch):
    """The fused step is the two calls in sequence, bit for bit."""
    rng = np.random.default_rng(7)
    m = 3 * 64 + 10
    P = _as_f32(_random_params(rng))
    U = _t32(torch, rng.normal(0, 1, (m, 4)))
    tg = _t32(torch, _targets(rng, m))
    a = gs.mlp_params_to_flat(P)
    b = a.clone()
    ma, va = torch.zeros_like(a), torch.zeros_like(a)
    mb, vb = torch.zeros_like(a), torch.zeros_like(a)
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    for t in (1, 2):
        gs.mlp_train_step(a, ma, va, t, 1e-3, U, tg, loss)
        g, l2 = gs.mlp_grad(b, U, tg)
        gs.mlp_adam(b, mb, vb, g, t, 1e-3)
        torch.cuda.synchronize()
        assert float(loss[0]) == float(l2[0])
    assert torch.equal(a, b) and torch.equal(ma, mb) and torch.equal(va, vb)


def test_training_reduces_loss(torch):
    """A few hundred device Adam steps fit a learnable target (support =
    first input above 1, step = half the third input)."""
    rng = np.random.default_rng(8)
    m = 4096
    U = rng.normal(0, 1, (m, 4))
    tg = np.stack([0.5 * U[:, 2], (U[:, 0] > 1.0).astype(np.float64), np.ones(m)], axis=1)
    flat = gs.mlp_params_to_flat(_random_params(rng))
    mom, vel = torch.zeros_like(flat), torch.zeros_like(flat)
    Ud, td = _t32(torch, U), _t32(torch, tg)
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    ws = None
    first = None
    for t in range(1, 301):
        ws = gs.mlp_train_step(flat, mom, vel, t, 3e-3, Ud, td, loss, workspace=ws)
        if t == 1:
            first = float(loss[0])
    last = float(loss[0])
    assert last < 0.5 * first, (first, last)
    # the oracle's loss of the trained device weights agrees
    out, _ = O.mlp_forward_bf16(gs.mlp_flat_to_params(flat), U.astype(np.float32).astype(np.float64))
    assert abs(O.mlp_loss(out, tg[:, 0], tg[:, 1], tg[:, 2]) - last) <= 0.05 * first


# ------------------------------------------------------- restricted solve

def _rs_case(seed, n, p, m, dtype):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, p)).astype(dtype)
    y = rng.standard_normal(n).astype(dtype)
    W = np.sort(rng.choice(p, m, replace=False)).astype(np.int32)
    sg = np.where(rng.uniform(size=m) < 0.5, -1.0, 1.0)
    lam = 0.1 * float(np.abs(X.astype(np.float64).T @ y.astype(np.float64)).max())
    return X, y, W, sg, lam


def _rs_run(torch, X, y, W, sg, lam):
    Xd = gs.colmajor_to_device(X)
    yd = torch.from_numpy(np.ascontiguousarray(y)).cuda()
    b, info = gs.restricted_solve(Xd, yd, torch.from_numpy(W).cuda(),
                                  torch.from_numpy(sg).cuda(), lam)
    torch.cuda.synchronize()
    return _np(b), int(info.item())


@pytest.mark.parametrize("m", [1, 63, 64, 65, 200, 700, 999])
def test_restricted_solve_matches_oracle(torch, m):
    """The blocked FP64 Cholesky solve against the oracle's library solve on
    the same (FP32-stored) values: relative error within 1e-14 times the
    condition number of X_W^T X_W (and 1e-11 at least); tiles of 64 with a
    ragged last one, up to m = n - 1."""
    X, y, W, sg, lam = _rs_case(100 + m, 1000, 3000, m, np.float32)
    b, info = _rs_run(torch, X, y, W, sg, lam)
    assert info == 0
    ref = O.restricted_solve(X.astype(np.float64), y.astype(np.float64), W, sg, lam)
    XW = X[:, W].astype(np.float64)
    cond = np.linalg.cond(XW.T @ XW)
    err = np.linalg.norm(b - ref) / np.linalg.norm(ref)
    assert err <= max(1e-11, 1e-14 * cond), (m, err, cond)


def test_restricted_solve_f64(torch):
    X, y, W, sg, lam = _rs_case(7, 50, 500, 30, np.float64)
    b, info = _rs_run(torch, X, y, W, sg, lam)
    assert info == 0
    ref = O.restricted_solve(X, y, W, sg, lam)
    assert np.linalg.norm(b - ref) <= 1e-11 * np.linalg.norm(ref)


def test_restricted_solve_reports_rank_deficiency_and_bad_index(torch):
    """A zero column makes its pivot exactly zero: info is its 1-based row
    in W; an index outside [0, p) gives info = -1; sizes outside the limits
    are rejected before any launch."""
    X, y, W, sg, lam = _rs_case(8, 300, 800, 150, np.float32)
    X[:, W[70]] = 0.0
    _, info = _rs_run(torch, X, y, W, sg, lam)
    assert info == 71
    X, y, W, sg, lam = _rs_case(9, 300, 800, 150, np.float32)
    W[5] = 800
    _, info = _rs_run(torch, X, y, W, sg, lam)
    assert info == -1
    Xd = gs.colmajor_to_device(X)
    yd = torch.from_numpy(y).cuda()
    Wd = torch.arange(300, dtype=torch.int32, device="cuda")
    with pytest.raises(Exception):
        gs.restricted_solve(Xd, yd, Wd, torch.ones(300, dtype=torch.float64, device="cuda"), lam)


# ----------------------------------------------------------- learned path

def _c4_small(seed, p=2000, n=120):
    d = synth.c4(seed=seed, n=n, p=p, block=50)
    return d["X"], d["y"]


def test_learned_path_f64_and_small_n(torch, orc):
    """The learned driver on the 50 x 500 FP64 problem (working sets capped at
    n - 1 = 49 columns, down to lambda_max / 1000 where the support nears n)
    and on a 30 x 40 FP32 problem (p close to n): every lambda certified and
    within the oracle's bounds, whichever start each lambda took."""
    import os
    wfile = os.path.join(os.path.dirname(gs.__file__), "warm_mlp.npy")
    P = torch.from_numpy(np.load(wfile).astype(np.float32)).cuda()
    d = synth.c0()
    X, y = d["X"], d["y"]
    Xd, yd = _dev(torch, X, y, 2)
    got = gs.lasso_path_learned(Xd, yd, P, T=40, lambda_min_ratio=1e-3)
    _check_path(X, y, got, orc, _np(got["lambdas"]))
    taken_c0 = int(_np(got["learned"]).sum())
    d = synth.gaussian(77, 30, 40, k=5)
    X, y = d["X"].astype(np.float32), d["y"].astype(np.float32)
    Xd, yd = _dev(torch, X, y)
    got = gs.lasso_path_learned(Xd, yd, P, T=30, lambda_min_ratio=1e-3)
    _check_path(X, y, got, orc, _np(got["lambdas"]))
    print(f"learned driver: c0 started {taken_c0} of 39 lambdas from the network, "
          f"30 x 40 {int(_np(got['learned']).sum())} of 29")


def test_learned_path_plain_mode_certified(torch, orc):
    """params = None: every lambda warm-starts from the previous solution,
    one lasso_path call per lambda; the same certified answers as the plain
    path, on the same grid."""
    X, y = _c4_small(21)
    Xd, yd = _dev(torch, X, y)
    got = gs.lasso_path_learned(Xd, yd, None, T=20, lambda_min_ratio=1e-2)
    lams = _np(got["lambdas"])
    ref = orc.grid(orc.precompute(X, y)["lambda_max"], 20, 2.0)
    np.testing.assert_allclose(lams, ref, rtol=1e-12)
    _check_path(X, y, got, orc, lams)
    assert np.all(_np(got["learned"]) == 0)


@pytest.mark.parametrize("kind", ["random", "no_change", "huge"])
def test_learned_path_any_network_certified(torch, orc, kind):
    """Whatever the network proposes, every lambda ends certified with the
    plain path's guarantees: a random network, one whose support logit is
    positive exactly on the previous support, and one that calls every
    feature an entrant (the entrant limit then admits none, and the working
    set grows from the previous support by the rounds' violators)."""
    X, y = _c4_small(22)
    rng = np.random.default_rng(23)
    if kind == "random":
        P = _random_params(rng)
    else:
        P = {k: np.zeros(s) for k, (_, s) in gs.MLP_LAYOUT.items()}
        # h0 = relu(u2), h1 = relu(-u2), passed through the second layer;
        # o0 = 0 (no change); o1 = h0 + h1 - 2^-20 > 0 exactly where
        # beta_prev != 0, so the proposal is the previous point restricted
        # to the safe set
        P["W1"][0, 2], P["W1"][1, 2] = 1.0, -1.0
        P["W2"][0, 0], P["W2"][1, 1] = 1.0, 1.0
        P["W3"][1, 0], P["W3"][1, 1] = 1.0, 1.0
        P["b3"][1] = -2.0 ** -20
        if kind == "huge":
            P["b3"][0], P["b3"][1] = 1e6, 10.0
    Xd, yd = _dev(torch, X, y)
    got = gs.lasso_path_learned(Xd, yd, gs.mlp_params_to_flat(P), T=20, lambda_min_ratio=1e-2)
    lams = _np(got["lambdas"])
    _check_path(X, y, got, orc, lams)
    flags = _np(got["learned"])
    assert flags[0] == 0 and set(np.unique(flags)) <= {0, 1}


def test_learned_path_wide_c4_shape(torch, orc):
    """A C4-shaped problem large enough for the wide schedule (n = 1000,
    p = 20000), 8 lambdas down to lambda_max / 10, a random network."""
    X, y = _c4_small(24, p=20000, n=1000)
    Xd, yd = _dev(torch, X, y)
    P = _random_params(np.random.default_rng(25))
    got = gs.lasso_path_learned(Xd, yd, gs.mlp_params_to_flat(P), T=8, lambda_min_ratio=0.1)
    lams = _np(got["lambdas"])
    _check_path(X, y, got, orc, lams)


def test_learned_path_in_pieces(torch, orc):
    """A path run in two pieces (the second warm-started from the first's
    last solution, where the network may already propose) certifies every
    lambda of the whole grid."""
    X, y = _c4_small(26)
    Xd, yd = _dev(torch, X, y)
    P = gs.mlp_params_to_flat(_random_params(np.random.default_rng(27)))
    rel = 0.01 ** (np.arange(16) / 15)
    a = gs.lasso_path_learned(Xd, yd, P, lambdas=rel[:7], relative=True)
    b = gs.lasso_path_learned(Xd, yd, P, lambdas=rel[7:], relative=True,
                              beta_init=a["beta"][-1].contiguous())
    got = {k: torch.cat([a[k], b[k]]) for k in ("beta", "gap", "status", "lambdas")}
    lams = _np(got["lambdas"])
    lmax = orc.precompute(X, y)["lambda_max"]
    np.testing.assert_allclose(lams, lmax * rel, rtol=1e-12)
    _check_path(X, y, got, orc, lams)
    assert _np(a["learned"])[0] == 0


def test_trained_network_against_plain_start(torch, orc):
    """The committed trained network on a held-out c4-structured problem
    (seed 20000, p = 4000, the first 30 lambdas of the c4 grid): both paths
    certify every lambda; the network's start is taken only where its reduced
    gap is smaller, and up to the first lambda where it is taken the two runs
    are the same computation (identical epochs)."""
    import os
    wfile = os.path.join(os.path.dirname(gs.__file__), "warm_mlp.npy")
    P = torch.from_numpy(np.load(wfile).astype(np.float32)).cuda()
    assert P.numel() == gs.MLP_PARAMS
    X, y = _c4_small(20000, p=4000, n=1000)
    Xd, yd = _dev(torch, X, y)
    rel = 1e-3 ** (np.arange(100) / 99)
    plain = gs.lasso_path_learned(Xd, yd, None, lambdas=rel[:30], relative=True)
    learned = gs.lasso_path_learned(Xd, yd, P, lambdas=rel[:30], relative=True)
    lams = _np(plain["lambdas"])
    _check_path(X, y, plain, orc, lams)
    _check_path(X, y, learned, orc, lams)
    flags = _np(learned["learned"])
    ep_p, ep_l = _np(plain["epochs"]), _np(learned["epochs"])
    first = int(np.argmax(flags)) if flags.any() else len(flags)
    assert np.array_equal(ep_p[:first], ep_l[:first])
    print(f"trained network: started {int(flags.sum())} of {len(flags) - 1} lambdas, "
          f"epochs {int(ep_l.sum())} learned vs {int(ep_p.sum())} plain")


def test_trained_network_gain_held_out(torch):
    """The gain of the learned start at equal certified gap: a held-out
    c4-structured problem (seed 20001, n = 1000, p = 20000, the first 70
    lambdas of the c4 grid down to lambda_max / 120), every lambda certified
    (gap <= 1e-8 ||y||^2) on both paths; the learned path needs at most half
    the CD epochs and less time than the plain one (both printed)."""
    import os
    import time
    wfile = os.path.join(os.path.dirname(gs.__file__), "warm_mlp.npy")
    P = torch.from_numpy(np.load(wfile).astype(np.float32)).cuda()
    X, y = _c4_small(20001, p=20000, n=1000)
    Xd, yd = _dev(torch, X, y)
    yy = float(np.sum(y.astype(np.float64) ** 2))
    rel = 1e-3 ** (np.arange(100) / 99)
    res = {}
    for name, prm in (("plain", None), ("learned", P)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = gs.lasso_path_learned(Xd, yd, prm, lambdas=rel[:70], relative=True)
        torch.cuda.synchronize()
        res[name] = (r, time.perf_counter() - t0)
        assert np.all(_np(r["status"]) == 0) and np.all(_np(r["gap"]) <= 1e-8 * yy)
    (rp, sp), (rl, sl) = res["plain"], res["learned"]
    ep_p, ep_l = int(_np(rp["epochs"]).sum()), int(_np(rl["epochs"]).sum())
    taken = int(_np(rl["learned"]).sum())
    print(f"learned start gain (held-out seed 20001, 1000 x 20000, 70 lambdas): "
          f"epochs {ep_l} vs {ep_p} plain, seconds {sl:.3f} vs {sp:.3f} plain, "
          f"network start taken at {taken} of 69 lambdas")
    assert taken > 0
    assert 2 * ep_l <= ep_p
    assert sl < sp


def test_zero_response_paths(torch):
    """y = 0: lambda_max = 0, the solution is beta = 0 at once (gap 0); the
    plain path and the learned driver (which then defers to the plain path)
    both return zeros, certified, with zero epochs."""
    d = synth.gaussian(31, 40, 300)
    X = d["X"].astype(np.float32)
    y = np.zeros(40, dtype=np.float32)
    Xd, yd = _dev(torch, X, y)
    P = gs.mlp_params_to_flat(_random_params(np.random.default_rng(32)))
    for got in (gs.lasso_path(Xd, yd, T=5, lambda_min_ratio=0.1),
                gs.lasso_path_learned(Xd, yd, P, T=5, lambda_min_ratio=0.1)):
        torch.cuda.synchronize()
        assert np.all(_np(got["beta"]) == 0)
        assert np.all(_np(got["status"]) == 0)
        assert np.all(_np(got["gap"]) == 0)
        assert np.all(_np(got["epochs"]) == 0)
