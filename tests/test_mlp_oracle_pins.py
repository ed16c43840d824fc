"""Pins of the oracle's learned-warm-start reference (NumPy, FP64): the MLP
forward, loss, backward and Adam step, the block max correlation, the bf16
rounding and the features.  Each is checked against something other than
itself: finite differences, closed forms on hand-built networks, textbook
properties, brute force and torch's own bfloat16 conversion."""
import numpy as np
import pytest

import oracle as O


def _params(rng, scale=0.5):
    return dict(W1=rng.normal(0, scale, (64, 4)), b1=rng.normal(0, 0.1, 64),
                W2=rng.normal(0, scale / 4, (64, 64)), b2=rng.normal(0, 0.1, 64),
                W3=rng.normal(0, scale / 4, (2, 64)), b3=rng.normal(0, 0.1, 2))


def _data(rng, m=7):
    U = rng.normal(0, 1, (m, 4))
    ts = rng.normal(0, 1, m)
    tp = (rng.uniform(size=m) < 0.5).astype(np.float64)
    mk = (rng.uniform(size=m) < 0.7).astype(np.float64)
    return U, ts, tp, mk


def _loss(params, U, ts, tp, mk):
    out, _ = O.mlp_forward(params, U)
    return O.mlp_loss(out, ts, tp, mk)


def _fd_check(backward, seed=0, h=1e-6):
    rng = np.random.default_rng(seed)
    P = _params(rng)
    U, ts, tp, mk = _data(rng)
    out, cache = O.mlp_forward(P, U)
    g = backward(P, cache, out, ts, tp, mk)
    worst = 0.0
    for k in P:
        flat = P[k].reshape(-1)
        idx = rng.choice(flat.size, size=min(12, flat.size), replace=False)
        for i in idx:
            old = flat[i]
            flat[i] = old + h
            lp = _loss(P, U, ts, tp, mk)
            flat[i] = old - h
            lm = _loss(P, U, ts, tp, mk)
            flat[i] = old
            num = (lp - lm) / (2 * h)
            ana = g[k].reshape(-1)[i]
            worst = max(worst, abs(num - ana) / max(1e-6, abs(num) + abs(ana)))
    return worst


def test_backward_matches_finite_differences():
    for seed in range(3):
        assert _fd_check(O.mlp_backward, seed) < 1e-5


def test_planted_backward_mistakes_are_caught():
    """A sign flip, a dropped ReLU mask or a transposed weight in the
    backward pass fails the finite-difference pin."""
    def flip_sign(P, cache, out, ts, tp, mk):
        g = O.mlp_backward(P, cache, out, ts, tp, mk)
        g["W2"] = -g["W2"]
        return g

    def no_mask(P, cache, out, ts, tp, mk):
        U, h1p, h1, h2p, h2 = cache
        return O.mlp_backward(P, (U, np.abs(h1p) + 1, h1, np.abs(h2p) + 1, h2), out, ts, tp, mk)

    def transposed(P, cache, out, ts, tp, mk):
        g = O.mlp_backward(P, cache, out, ts, tp, mk)
        g["W2"] = g["W2"].T
        return g

    for bad in (flip_sign, no_mask, transposed):
        assert _fd_check(bad) > 1e-3, bad.__name__


def test_forward_closed_form():
    """W1 copies the 4 inputs into hidden units 0..3 (and their negatives
    into 4..7), W2 is the identity, W3 sums units 0..7 into output 0 and
    unit 0 into output 1: out0 = sum |u|, out1 = relu(u0)."""
    P = dict(W1=np.zeros((64, 4)), b1=np.zeros(64), W2=np.eye(64), b2=np.zeros(64),
             W3=np.zeros((2, 64)), b3=np.zeros(2))
    P["W1"][:4] = np.eye(4)
    P["W1"][4:8] = -np.eye(4)
    P["W3"][0, :8] = 1.0
    P["W3"][1, 0] = 1.0
    U = np.array([[1.0, -2.0, 0.5, 0.0], [-1.5, 3.0, -0.25, 2.0]])
    out, _ = O.mlp_forward(P, U)
    np.testing.assert_allclose(out[:, 0], np.abs(U).sum(1), rtol=1e-15)
    np.testing.assert_allclose(out[:, 1], np.maximum(U[:, 0], 0), rtol=1e-15)


def test_loss_special_values():
    """BCE at logit 0 is log 2 whatever the label; a confident right logit
    costs ~0 and a confident wrong one ~|logit|; the step term is the masked
    squared error."""
    out = np.array([[1.0, 0.0], [1.0, 0.0], [0.0, 40.0], [0.0, -40.0]])
    tp = np.array([1.0, 0.0, 1.0, 1.0])
    ts = np.array([1.0, 1.0, 0.0, 0.0])
    mk = np.zeros(4)
    L = O.mlp_loss(out, ts, tp, mk)
    np.testing.assert_allclose(L, (2 * np.log(2) + 0.0 + 40.0) / 4, rtol=1e-12)
    mk = np.array([1.0, 0.0, 0.0, 0.0])
    out2 = out.copy()
    out2[0, 0] = 3.0
    assert abs(O.mlp_loss(out2, ts, tp, mk) - L - 4.0 / 4) < 1e-12


def test_adam_first_step_is_signed_lr():
    """With zero moments, bias correction makes the first update
    lr * g / (|g| + eps): lr times the sign of each gradient entry."""
    rng = np.random.default_rng(3)
    P = {"W": rng.normal(size=(5, 3))}
    G = {"W": rng.normal(size=(5, 3))}
    P0 = P["W"].copy()
    st = {}
    O.adam_step(P, G, st, lr=0.01, eps=1e-12)
    np.testing.assert_allclose(P0 - P["W"], 0.01 * np.sign(G["W"]), rtol=1e-9)
    # second step with the same gradient: still lr * sign (m, v keep ratios)
    P1 = P["W"].copy()
    O.adam_step(P, G, st, lr=0.01, eps=1e-12)
    np.testing.assert_allclose(P1 - P["W"], 0.01 * np.sign(G["W"]), rtol=1e-9)
    assert st["t"] == 2


def test_block_max_corr_brute_force():
    rng = np.random.default_rng(4)
    n, p, block = 9, 23, 5
    X = rng.normal(size=(n, p))
    X[:, 7] = 0.0  # a zero column
    got = O.block_max_corr(X, block)
    for j in range(p):
        b0 = (j // block) * block
        best = 0.0
        for k in range(b0, min(p, b0 + block)):
            if k == j:
                continue
            nj, nk = np.linalg.norm(X[:, j]), np.linalg.norm(X[:, k])
            if nj == 0 or nk == 0:
                continue
            best = max(best, abs(X[:, j] @ X[:, k]) / (nj * nk))
        assert abs(got[j] - best) < 1e-14, j
    assert got[7] == 0.0
    # a last block of one column has no partner
    assert O.block_max_corr(X[:, :21], block)[20] == 0.0


def test_block_max_corr_equicorrelated():
    """Two identical columns have correlation 1, opposite ones 1 too (the
    absolute value), and orthogonal columns 0."""
    X = np.zeros((4, 4))
    X[:, 0] = [1, 2, 3, 4]
    X[:, 1] = [2, 4, 6, 8]
    X[:, 2] = [-1, -2, -3, -4]
    X[:, 3] = [4, -3, 2, -1.25]  # orthogonal to column 0: 4 - 6 + 6 - 5 = -1?
    X[:, 3] -= (X[:, 3] @ X[:, 0]) / (X[:, 0] @ X[:, 0]) * X[:, 0]
    got = O.block_max_corr(X, 4)
    np.testing.assert_allclose(got[:3], 1.0, rtol=1e-15)
    assert got[3] < 1e-15


def test_bf16_round_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(5)
    a = np.concatenate([rng.normal(0, 1, 1000), rng.normal(0, 1e-3, 100), [0.0, -0.0, 1.0,
                        1.0 + 2 ** -8, 1.0 + 2 ** -9, 1.0 + 3 * 2 ** -9, 65504.0]])
    a32 = a.astype(np.float32)
    want = torch.from_numpy(a32).to(torch.bfloat16).to(torch.float32).numpy().astype(np.float64)
    np.testing.assert_array_equal(O.bf16_round(a32), want)
    # ties to even: 1 + 2^-8 is halfway between 1 and 1 + 2^-7
    assert O.bf16_round(np.float32(1.0 + 2 ** -8)) == 1.0
    assert O.bf16_round(np.float32(1.0 + 3 * 2 ** -8)) == 1.0 + 2 ** -6


def test_warm_features_definition():
    c = np.array([2.0, -6.0])
    f = O.warm_features(c, lam=4.0, lam_max=8.0, beta_prev=np.array([0.5, 0.0]),
                        nrm=np.array([2.0, 3.0]), ynorm=10.0, bmc=np.array([0.1, 0.9]))
    np.testing.assert_allclose(f, [[0.5, 0.5, 0.1, 0.1], [1.5, 0.5, 0.0, 0.9]])
