"""Seeded synthetic Lasso workloads.

This module only draws data: designs, responses and row subsamples.  It holds
none of the solver's arithmetic (no lambda_max, no grid, no gap), so that both
the HIP library's tests and the CPU oracle can use it without sharing method
code.

Every workload is a stand-in for the shapes of the paper's experiments
(Leukemia is dense 72 x 7129) or for the configurations the project measures:

  c0  single Lasso, FP64, 50 x 500, i.i.d. N(0,1), unit-norm columns,
      10-sparse +-1 truth, noise 0.1 N(0,1), lambda = lambda_max / 10.
  c1  72 x 7129, AR(1) correlation 0.5 along the column index, standardized
      columns (mean 0, variance 1), 20-sparse +-1 truth, SNR 3, FP32.
  c2  256 subsamples of 36 distinct rows of the c1 problem.
  c3  512 problems, n log-uniform in [50, 2000], p log-uniform in
      [1000, 50000], AR(1) correlation U[0, 0.8], unit-norm columns,
      k-sparse truth (k uniform in 5..100), SNR 3, lambda/lambda_max uniform
      in [0.01, 0.5].
  c4  1000 x 100000 (400 MB FP32), 2000 blocks of 50 equicorrelated columns
      (rho = 0.7), unit-norm columns, 50-sparse truth, SNR 5.
  sparse_text  CSC designs shaped like the paper's sparse text data
      (20newsgroup 961 x 10094, RCV1 20242 x 47236): Zipf column counts.

SNR s means the noise vector is drawn with sigma = ||X beta*|| / (s sqrt(n)).
Column-major layout: ``colmajor(X, ld)`` returns a (p, ld) C-contiguous array
whose row j holds column j (zero padding below row n).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.signal import lfilter


def _rng(seed):
    return np.random.default_rng(np.random.SeedSequence(seed))


def ar1_columns(rng, n, p, rho):
    """Rows ~ N(0, Sigma), Sigma_jk = rho^|j-k|: x_1 = z_1 and
    x_j = rho x_{j-1} + sqrt(1-rho^2) z_j along the column index."""
    z = rng.standard_normal((n, p))
    if rho == 0.0:
        return z
    s = math.sqrt(1.0 - rho * rho)
    z[:, 0] /= s
    return lfilter([s], [1.0, -rho], z, axis=1)


def _truth(rng, p, k):
    beta = np.zeros(p)
    idx = rng.choice(p, size=k, replace=False)
    beta[idx] = rng.choice([-1.0, 1.0], size=k)
    return beta


def _response(rng, X, beta, snr=None, sigma=None):
    signal = X @ beta
    n = X.shape[0]
    if sigma is None:
        sigma = np.linalg.norm(signal) / (snr * math.sqrt(n))
    return signal + sigma * rng.standard_normal(n)


def colmajor(X, ld=None, dtype=None):
    """(n, p) array -> (p, ld) C-contiguous column-major storage."""
    X = np.asarray(X)
    n, p = X.shape
    ld = n if ld is None else ld
    dtype = X.dtype if dtype is None else dtype
    out = np.zeros((p, ld), dtype=dtype)
    out[:, :n] = X.T
    return out


def pad_ld(n, mult=4):
    return ((n + mult - 1) // mult) * mult


def c0(seed=0, n=50, p=500, k=10):
    rng = _rng(seed)
    X = rng.standard_normal((n, p))
    X /= np.linalg.norm(X, axis=0)
    beta = _truth(rng, p, k)
    y = _response(rng, X, beta, sigma=0.1)
    return dict(X=X, y=y, beta_star=beta, lambda_ratio=0.1, dtype="f64")


def c1(seed=1, n=72, p=7129, k=20, rho=0.5, snr=3.0):
    rng = _rng(seed)
    X = ar1_columns(rng, n, p, rho)
    X -= X.mean(axis=0)
    X /= X.std(axis=0)
    beta = _truth(rng, p, k)
    y = _response(rng, X, beta, snr=snr)
    return dict(X=X.astype(np.float32), y=y.astype(np.float32), beta_star=beta,
                T=100, delta=3.0, dtype="f32")


def c2(seed=2, base_seed=1, B=256, m=36):
    base = c1(base_seed)
    n = base["X"].shape[0]
    rows = np.empty((B, m), dtype=np.int32)
    for b, ss in enumerate(np.random.SeedSequence(seed).spawn(B)):
        r = np.random.default_rng(ss)
        rows[b] = np.sort(r.choice(n, size=m, replace=False))
    return dict(X=base["X"], y=base["y"], rows=rows, T=100, delta=2.0,
                dtype="f32")


def c3_params(seed=3, B=512):
    """Shapes and scalars of every c3 problem without drawing the designs."""
    out = []
    for ss in np.random.SeedSequence(seed).spawn(B):
        r = np.random.default_rng(ss)
        n = int(round(math.exp(r.uniform(math.log(50), math.log(2000)))))
        p = int(round(math.exp(r.uniform(math.log(1000), math.log(50000)))))
        rho = float(r.uniform(0.0, 0.8))
        k = int(r.integers(5, 101))
        lam_ratio = float(r.uniform(0.01, 0.5))
        out.append(dict(n=n, p=p, rho=rho, k=k, lambda_ratio=lam_ratio,
                        seedseq=ss))
    return out


def c3_problem(params, snr=3.0):
    """Draw the design and response of one c3 problem (from c3_params)."""
    r = np.random.default_rng(params["seedseq"].spawn(1)[0])
    n, p = params["n"], params["p"]
    X = ar1_columns(r, n, p, params["rho"])
    X /= np.linalg.norm(X, axis=0)
    beta = _truth(r, p, min(params["k"], p))
    y = _response(r, X, beta, snr=snr)
    return dict(X=X.astype(np.float32), y=y.astype(np.float32), beta_star=beta,
                lambda_ratio=params["lambda_ratio"], dtype="f32")


def c4(seed=4, n=1000, p=100000, block=50, rho=0.7, k=50, snr=5.0):
    rng = _rng(seed)
    nb = (p + block - 1) // block
    g = rng.standard_normal((n, nb))
    X = np.empty((n, p), dtype=np.float64)
    for b in range(nb):
        j0, j1 = b * block, min(p, (b + 1) * block)
        X[:, j0:j1] = math.sqrt(rho) * g[:, b:b + 1] + \
            math.sqrt(1.0 - rho) * rng.standard_normal((n, j1 - j0))
    X /= np.linalg.norm(X, axis=0)
    beta = _truth(rng, p, k)
    y = _response(rng, X, beta, snr=snr)
    return dict(X=X.astype(np.float32), y=y.astype(np.float32), beta_star=beta,
                T=100, delta=3.0, block=block, dtype="f32")


def sparse_text(seed, n, p, density, k=20, snr=3.0, zipf=1.0):
    """A sparse design in CSC form shaped like a bag-of-words matrix (the
    paper's 20newsgroup, 961 x 10094, and RCV1, 20242 x 47236): column j has
    about density * n nonzeros scaled by a Zipf weight (a few frequent
    terms, many rare ones; at least 1, at most n), at distinct uniformly
    drawn rows (ascending), with |N(0,1)| values; columns scaled to unit
    norm; y = X beta* + noise at the given SNR with a k-sparse +-1 beta*.
    Returns col_ptr (p+1 int64), row_idx (int32), values (float32), y
    (float32), beta_star and n."""
    rng = _rng(seed)
    w = 1.0 / (np.arange(1, p + 1) ** zipf)
    w = rng.permutation(w)
    counts = np.clip(np.round(w / w.mean() * density * n), 1, n).astype(np.int64)
    col_ptr = np.zeros(p + 1, dtype=np.int64)
    col_ptr[1:] = np.cumsum(counts)
    row_idx = np.empty(col_ptr[-1], dtype=np.int32)
    vals = np.empty(col_ptr[-1], dtype=np.float64)
    for j in range(p):
        a, b = col_ptr[j], col_ptr[j + 1]
        row_idx[a:b] = np.sort(rng.choice(n, size=b - a, replace=False))
        v = np.abs(rng.standard_normal(b - a))
        vals[a:b] = v / np.linalg.norm(v)
    beta = _truth(rng, p, k)
    signal = np.zeros(n)
    for j in np.flatnonzero(beta):
        a, b = col_ptr[j], col_ptr[j + 1]
        signal[row_idx[a:b]] += beta[j] * vals[a:b]
    sigma = np.linalg.norm(signal) / (snr * math.sqrt(n))
    y = signal + sigma * rng.standard_normal(n)
    return dict(col_ptr=col_ptr, row_idx=row_idx, values=vals.astype(np.float32),
                y=y.astype(np.float32), beta_star=beta, n=n, p=p)


def csc_to_dense(d):
    """Dense (n, p) float64 copy of a sparse_text design (values widened)."""
    X = np.zeros((d["n"], d["p"]))
    cp, ri, v = d["col_ptr"], d["row_idx"], d["values"].astype(np.float64)
    for j in range(d["p"]):
        X[ri[cp[j]:cp[j + 1]], j] = v[cp[j]:cp[j + 1]]
    return X


def orthonormal(seed, n, p):
    """Design with orthonormal columns (QR of a Gaussian matrix), n >= p."""
    rng = _rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, p)))
    y = rng.standard_normal(n)
    return dict(X=Q, y=y)


def gaussian(seed, n, p, k=3, sigma=0.1, unit=True):
    """Small i.i.d. Gaussian problem for brute-force and edge-case checks."""
    rng = _rng(seed)
    X = rng.standard_normal((n, p))
    if unit:
        X /= np.linalg.norm(X, axis=0)
    beta = _truth(rng, p, min(k, p))
    y = _response(rng, X, beta, sigma=sigma)
    return dict(X=X, y=y, beta_star=beta)
