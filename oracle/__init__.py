"""CPU FP64 oracle for GAP SAFE screened coordinate descent on the Lasso.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this
package: only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg
of ``bench.py`` use it.  It shares no code with the HIP library.

Two parts:
* ``gapsafe_oracle.c`` (built into ``liboracle.so`` with gcc): Algorithm 1 of
  Fercoq, Gramfort & Salmon (ICML 2015) in plain FP64 loops, one screening pass,
  the plain primal/dual gap.  Loaded through ctypes.
* numpy FP64 code for the learned warm start: the 4-64-64-2 MLP forward and
  backward pass with Adam, per-feature inputs and block-maximum correlation.
  These follow textbook definitions; the paper does not cover them.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gapsafe_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)
_bp = ctypes.POINTER(ctypes.c_uint8)


def build(src: str = _SRC, out: str = _LIB, extra_flags=()) -> str:
    """Compile the C oracle (plain -O2, IEEE semantics, no fast-math)."""
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fno-fast-math",
           "-ffp-contract=off", *extra_flags, src, "-o", out, "-lm"]
    subprocess.run(cmd, check=True)
    return out


def _declare(lib):
    lib.orc_precompute.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64,
                                   _dp, _dp, _dp, _dp, _dp, _dp]
    lib.orc_precompute.restype = ctypes.c_int
    lib.orc_grid.argtypes = [ctypes.c_double, ctypes.c_int, ctypes.c_double, _dp]
    lib.orc_grid.restype = None
    lib.orc_gap.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64, _dp, _dp,
                            _dp, _dp, ctypes.c_double, _dp, _dp]
    lib.orc_gap.restype = ctypes.c_double
    lib.orc_screen.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64, _dp,
                               _dp, _dp, ctypes.c_double, _ip, ctypes.c_int,
                               ctypes.c_int, _dp, _bp, _bp, _dp]
    lib.orc_screen.restype = ctypes.c_int
    lib.orc_lasso_path.argtypes = [
        ctypes.c_int, ctypes.c_int, ctypes.c_int64, _dp, _dp, ctypes.c_int, _dp,
        ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int,
        ctypes.c_int, ctypes.c_int, _dp, _dp, _dp, _ip, _ip, _ip, _ip, _bp, _dp]
    lib.orc_lasso_path.restype = ctypes.c_int
    lib.orc_dome_mu.argtypes = [ctypes.c_double] * 7
    lib.orc_dome_mu.restype = ctypes.c_double
    return lib


_lib_cache = {}


def load(path: str = _LIB, src: str = _SRC):
    """Load (building first if missing or stale) the C oracle library."""
    if path in _lib_cache:
        return _lib_cache[path]
    if (not os.path.exists(path)) or os.path.getmtime(path) < os.path.getmtime(src):
        build(src, path)
    lib = _declare(ctypes.CDLL(path))
    _lib_cache[path] = lib
    return lib


def _ptr(a, t=_dp):
    return None if a is None else a.ctypes.data_as(t)


def _design(X):
    """Column-major float64 view (widened exactly from fp32 when needed)."""
    X = np.asarray(X)
    Xf = np.asfortranarray(X, dtype=np.float64)
    return Xf, Xf.shape[0], Xf.shape[1]


class Oracle:
    """ctypes front-end of the C oracle; ``lib`` may be a mutated build."""

    def __init__(self, lib=None):
        self.lib = lib if lib is not None else load()

    def precompute(self, X, y):
        Xf, n, p = _design(X)
        y = np.ascontiguousarray(y, dtype=np.float64)
        nrm2 = np.empty(p)
        xty = np.empty(p)
        lmax = ctypes.c_double()
        yy = ctypes.c_double()
        rc = self.lib.orc_precompute(n, p, n, _ptr(Xf), _ptr(y), _ptr(nrm2),
                                     _ptr(xty), ctypes.byref(lmax), ctypes.byref(yy))
        if rc != 0:
            raise ValueError(f"orc_precompute: {rc}")
        return dict(nrm2=nrm2, xty=xty, lambda_max=lmax.value, ynorm2=yy.value)

    def grid(self, lambda_max, T, delta):
        out = np.empty(T)
        self.lib.orc_grid(lambda_max, T, delta, _ptr(out))
        return out

    def gap(self, X, y, beta, theta, lam):
        Xf, n, p = _design(X)
        y = np.ascontiguousarray(y, dtype=np.float64)
        beta = np.ascontiguousarray(beta, dtype=np.float64)
        theta = np.ascontiguousarray(theta, dtype=np.float64)
        P = ctypes.c_double()
        D = ctypes.c_double()
        g = self.lib.orc_gap(n, p, n, _ptr(Xf), _ptr(y), _ptr(beta), _ptr(theta),
                             lam, ctypes.byref(P), ctypes.byref(D))
        return g, P.value, D.value

    RULES = {"sphere": 0, "dome": 1, "static": 2, "dynamic_safe": 3, "st3": 4}

    def screen(self, X, y, beta, lam, active=None, rule="sphere"):
        Xf, n, p = _design(X)
        y = np.ascontiguousarray(y, dtype=np.float64)
        beta = np.ascontiguousarray(beta, dtype=np.float64)
        act = None if active is None else np.ascontiguousarray(active, dtype=np.int32)
        q = p if act is None else len(act)
        c = np.empty(max(q, 1))
        ke = np.zeros(max(q, 1), dtype=np.uint8)
        ks = np.zeros(max(q, 1), dtype=np.uint8)
        sc = np.empty(10)
        rc = self.lib.orc_screen(n, p, n, _ptr(Xf), _ptr(y), _ptr(beta), lam,
                                 _ptr(act, _ip), q, self.RULES[rule], _ptr(c),
                                 _ptr(ke, _bp), _ptr(ks, _bp), _ptr(sc))
        if rc < 0:
            raise ValueError(f"orc_screen: {rc}")
        idx = np.arange(p, dtype=np.int32) if act is None else act
        return dict(c=c[:q], active=idx, keep_exact=ke[:q].astype(bool),
                    keep_safe=ks[:q].astype(bool), gap=sc[0], alpha=sc[1],
                    radius=sc[2], radius_inflated=sc[3], M=sc[4], rho_norm2=sc[5],
                    y_rho=sc[6], l1=sc[7], alpha_safe=sc[8], err_gap=sc[9])

    def dome_mu(self, xty, c, xn, alpha, lam, R_hat, r_check2):
        """mu_D(x_j) of the GAP SAFE dome (exact formula) for one column."""
        return self.lib.orc_dome_mu(float(xty), float(c), float(xn), float(alpha), float(lam),
                                    float(R_hat), float(r_check2))

    def lasso_path(self, X, y, T=100, lambdas=None, relative=False, delta=3.0,
                   eps_rel=1e-8, f=10, K=100000, beta_init=None,
                   want_screened=False, rule="sphere"):
        Xf, n, p = _design(X)
        y = np.ascontiguousarray(y, dtype=np.float64)
        lam_in = None
        if lambdas is not None:
            lam_in = np.ascontiguousarray(lambdas, dtype=np.float64)
            T = len(lam_in)
        b0 = None if beta_init is None else np.ascontiguousarray(beta_init, dtype=np.float64)
        beta = np.zeros((T, p))
        gap = np.zeros(T)
        ep = np.zeros(T, dtype=np.int32)
        na = np.zeros(T, dtype=np.int32)
        st = np.zeros(T, dtype=np.int32)
        ps = np.zeros(T, dtype=np.int32)
        scr = np.zeros((T, p), dtype=np.uint8) if want_screened else None
        lam_out = np.zeros(T)
        rc = self.lib.orc_lasso_path(
            n, p, n, _ptr(Xf), _ptr(y), T, _ptr(lam_in), int(bool(relative)),
            float(delta), float(eps_rel), int(f), int(K), self.RULES[rule], _ptr(b0), _ptr(beta),
            _ptr(gap), _ptr(ep, _ip), _ptr(na, _ip), _ptr(st, _ip), _ptr(ps, _ip),
            _ptr(scr, _bp), _ptr(lam_out))
        if rc < 0:
            raise ValueError(f"orc_lasso_path: {rc}")
        return dict(beta=beta, gap=gap, epochs=ep, nactive=na, status=st,
                    passes=ps, lambdas=lam_out, screened=scr, rc=rc)


    def enet_path(self, X, y, alpha, T=100, lambdas=None, relative=False, delta=3.0,
                  eps_rel=1e-8, f=10, K=100000, beta_init=None, rule="sphere"):
        """The elastic net min 1/2||X b - y||^2 + alpha lam ||b||_1 +
        (1 - alpha) lam/2 ||b||^2 along a lambda grid (appendix,
        "Elastic-Net"): at each lambda_t, Algorithm 1 on the Lasso with
        parameter alpha lambda_t, design [X; sqrt((1 - alpha) lambda_t) I_p]
        and response [y; 0], written out explicitly, warm-started from the
        previous lambda.  The grid starts at ||X^T y||_inf / alpha, the
        smallest lambda with a zero solution.  Returns the lasso_path fields
        (gap and passes of the augmented problems)."""
        X = np.asarray(X, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        n, p = X.shape
        lmax = np.abs(X.T @ y).max() / alpha
        if lambdas is None:
            lams = lmax * 10.0 ** (-delta * np.arange(T) / max(T - 1, 1))
        else:
            lams = np.asarray(lambdas, dtype=np.float64) * (lmax if relative else 1.0)
        yt = np.concatenate([y, np.zeros(p)])
        keys = ("beta", "gap", "epochs", "nactive", "status", "passes")
        out = {k: [] for k in keys}
        b = None if beta_init is None else np.asarray(beta_init, dtype=np.float64)
        for lam in lams:
            Xt = np.vstack([X, np.sqrt((1.0 - alpha) * lam) * np.eye(p)])
            r = self.lasso_path(Xt, yt, lambdas=[alpha * lam], eps_rel=eps_rel, f=f, K=K,
                                beta_init=b, rule=rule)
            b = r["beta"][0]
            for k in keys:
                out[k].append(r[k][0])
        res = {k: np.array(v) for k, v in out.items()}
        res["lambdas"] = lams
        return res


_default: Optional[Oracle] = None


def oracle() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle()
    return _default


# ---------------------------------------------------------------------------
# Learned warm start: textbook FP64 definitions (not covered by the paper).
# ---------------------------------------------------------------------------

def bf16_round(a):
    """Round float64 values to bfloat16 (round to nearest, ties to even) and
    return them as float64.  Goes through float32 first, which is exact for
    the weights stored here (they are float32 master weights)."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def mlp_forward(params, U, round_h1=None):
    """4 -> 64 -> 64 -> 2 perceptron with ReLU hidden layers.
    params: dict W1 (64x4), b1 (64), W2 (64x64), b2 (64), W3 (2x64), b3 (2).
    U: (m, 4) inputs.  Returns outputs (m, 2) and the cache for backward.
    round_h1 (optional): a rounding applied to the first hidden layer before
    it enters the second (the cache then holds the rounded values)."""
    h1p = U @ params["W1"].T + params["b1"]
    h1 = np.maximum(h1p, 0.0)
    if round_h1 is not None:
        h1 = round_h1(h1)
    h2p = h1 @ params["W2"].T + params["b2"]
    h2 = np.maximum(h2p, 0.0)
    out = h2 @ params["W3"].T + params["b3"]
    return out, (U, h1p, h1, h2p, h2)


def bf16_params(params):
    """The weights as the device network uses them: every weight matrix
    rounded to bfloat16, biases kept."""
    return {k: (bf16_round(v) if k.startswith("W") else np.asarray(v, dtype=np.float64))
            for k, v in params.items()}


def mlp_forward_bf16(params, U):
    """The forward pass at the device's precision points: bfloat16 weight
    matrices and a bfloat16 first hidden layer entering the second layer
    (the matrix-core operands); everything else exact."""
    return mlp_forward(bf16_params(params), U, round_h1=bf16_round)


def mlp_loss(out, tgt_step, tgt_support, mask_step):
    """Mean over m features of  BCE(logit=out[:,1], tgt_support)
    + mask_step * (out[:,0] - tgt_step)^2 ."""
    m = out.shape[0]
    s = out[:, 1]
    bce = np.maximum(s, 0) - s * tgt_support + np.log1p(np.exp(-np.abs(s)))
    d = out[:, 0] - tgt_step
    mse = mask_step * d * d
    return float(np.sum(bce + mse) / m)


def mlp_backward(params, cache, out, tgt_step, tgt_support, mask_step):
    """Gradients of ``mlp_loss`` with respect to every parameter."""
    U, h1p, h1, h2p, h2 = cache
    m = out.shape[0]
    s = out[:, 1]
    sig = 1.0 / (1.0 + np.exp(-s))
    g_out = np.zeros_like(out)
    g_out[:, 1] = (sig - tgt_support) / m
    g_out[:, 0] = 2.0 * mask_step * (out[:, 0] - tgt_step) / m
    gW3 = g_out.T @ h2
    gb3 = g_out.sum(0)
    g_h2 = g_out @ params["W3"]
    g_h2p = g_h2 * (h2p > 0)
    gW2 = g_h2p.T @ h1
    gb2 = g_h2p.sum(0)
    g_h1 = g_h2p @ params["W2"]
    g_h1p = g_h1 * (h1p > 0)
    gW1 = g_h1p.T @ U
    gb1 = g_h1p.sum(0)
    return dict(W1=gW1, b1=gb1, W2=gW2, b2=gb2, W3=gW3, b3=gb3)


def adam_step(params, grads, state, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015) of FP64 master weights in place."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in params:
        m = state.setdefault("m_" + k, np.zeros_like(params[k]))
        v = state.setdefault("v_" + k, np.zeros_like(params[k]))
        m[...] = b1 * m + (1 - b1) * grads[k]
        v[...] = b2 * v + (1 - b2) * grads[k] * grads[k]
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        params[k] -= lr * mh / (np.sqrt(vh) + eps)


def block_max_corr(X, block):
    """bmc_j = max over k != j in j's block of |x_j^T x_k| / (||x_j|| ||x_k||);
    blocks are ``block`` contiguous columns (the last one may be shorter).
    A block of one column, or a zero column, gives 0."""
    Xf = np.asarray(X, dtype=np.float64)
    n, p = Xf.shape
    out = np.zeros(p)
    for b0 in range(0, p, block):
        B = Xf[:, b0:b0 + block]
        G = B.T @ B
        d = np.sqrt(np.diag(G))
        with np.errstate(divide="ignore", invalid="ignore"):
            C = np.abs(G) / np.outer(d, d)
        C[~np.isfinite(C)] = 0.0
        np.fill_diagonal(C, 0.0)
        out[b0:b0 + B.shape[1]] = C.max(axis=1) if B.shape[1] > 1 else 0.0
    return out


def warm_features(c, lam, lam_max, beta_prev, nrm, ynorm, bmc):
    """Per-feature inputs of the learned warm start:
    (|x_j^T r| / lambda, lambda / lambda_max, beta_prev_j ||x_j|| / ||y||, bmc_j).
    ``c`` holds x_j^T r at the previous solution."""
    return np.stack([np.abs(c) / lam,
                     np.full_like(c, lam / lam_max),
                     beta_prev * nrm / ynorm,
                     bmc], axis=1)



def restricted_solve(X, y, W, sigma, lam):
    """The restricted solve of the learned start (Sec. 2, optimality
    conditions of the Lasso: at a solution, x_j^T (y - X beta) = lambda
    sign(beta_j) on the support).  For the columns W with signs sigma, the
    coefficients b on W that satisfy those conditions with equality solve
        (X_W^T X_W) b = X_W^T y - lambda sigma.
    FP64, through a library linear solve."""
    XW = np.asarray(X, dtype=np.float64)[:, np.asarray(W)]
    rhs = XW.T @ np.asarray(y, dtype=np.float64) - lam * np.asarray(sigma, dtype=np.float64)
    return np.linalg.solve(XW.T @ XW, rhs)
