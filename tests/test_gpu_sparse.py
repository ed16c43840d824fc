"""GPU parity for sparse (CSC) designs: Algorithm 1 with the transposed sparse
sweep and sparse CD steps (the paper's sparse implementation, Sec. 4.1)
against the CPU oracle on the same matrix written out densely, on synthetic
bag-of-words designs of the paper's 20newsgroup shape (961 x 10094) and an
RCV1-like row count (20242 rows, residual in global memory)."""
import numpy as np
import pytest

import paper_1505_03410_amd as gs
import synth
from test_gpu_parity import BETA_TOL, _check_path, _np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    gs.load_library()
    return torch


def _dev(torch, d):
    X = gs.CscDesign.from_host(d["col_ptr"], d["row_idx"], d["values"], d["n"])
    return X, torch.from_numpy(d["y"]).cuda()


def _oracle_design(d):
    return synth.csc_to_dense(d), d["y"].astype(np.float64)


@pytest.mark.parametrize("rule", ["sphere", "dome"])
def test_csc_path_20newsgroup_shape(torch, orc, rule):
    """961 x 10094 with 0.8% of the entries (Zipf column counts), 12
    lambdas to lambda_max/10: certified, beta against the tight oracle, the
    same epochs and final active set sizes as the oracle."""
    d = synth.sparse_text(5, 961, 10094, 0.008)
    X, y = _dev(torch, d)
    got = gs.lasso_path(X, y, T=12, lambda_min_ratio=0.1, rule=rule)
    torch.cuda.synchronize()
    assert got["rc"] == gs.GS_OK
    Xf, yf = _oracle_design(d)
    lams = _np(got["lambdas"])
    ref = orc.grid(orc.precompute(Xf, yf)["lambda_max"], 12, 1.0)
    np.testing.assert_allclose(lams, ref, rtol=1e-12)
    _check_path(Xf, yf, got, orc, lams, label=f"csc 20ng {rule}")
    o = orc.lasso_path(Xf, yf, lambdas=lams, rule=rule)
    np.testing.assert_array_equal(_np(got["epochs"]), o["epochs"])
    np.testing.assert_array_equal(_np(got["nactive"]), o["nactive"])
    # duplicate sparse columns make beta_hat non-unique (sigma_min = 0 above),
    # so the iterates themselves are compared: same gap target, same epochs
    B = _np(got["beta"])
    for t in range(1, len(lams)):
        nb = np.linalg.norm(o["beta"][t])
        assert np.linalg.norm(B[t] - o["beta"][t]) <= BETA_TOL * nb, t


def test_csc_residual_in_global_memory(torch, orc):
    """20242 rows (the RCV1 row count): the residual (162 KB) does not fit in
    LDS and lives in global memory; 2000 columns so the dense oracle stays
    small."""
    d = synth.sparse_text(6, 20242, 2000, 0.003)
    X, y = _dev(torch, d)
    got = gs.lasso_path(X, y, T=8, lambda_min_ratio=0.1)
    torch.cuda.synchronize()
    assert got["rc"] == gs.GS_OK
    Xf, yf = _oracle_design(d)
    lams = _np(got["lambdas"])
    _check_path(Xf, yf, got, orc, lams, label="csc 20242 rows")
    o = orc.lasso_path(Xf, yf, lambdas=lams)
    np.testing.assert_array_equal(_np(got["epochs"]), o["epochs"])


def test_csc_batch_and_edge_cases(torch, orc):
    """A batch of CSC problems of different shapes in one launch, including
    an empty column and a column with every row, and y = 0."""
    probs, host = [], []
    for i, (n, p, dens) in enumerate([(300, 900, 0.02), (961, 2000, 0.01), (64, 500, 0.05)]):
        d = synth.sparse_text(50 + i, n, p, dens)
        if i == 0:  # an empty column and a full one
            cp, ri, v = d["col_ptr"], d["row_idx"], d["values"]
            counts = np.diff(cp)
            counts[3], counts[4] = 0, n
            rows = [ri[cp[j]:cp[j + 1]] for j in range(p)]
            vals = [v[cp[j]:cp[j + 1]] for j in range(p)]
            rows[3], vals[3] = np.zeros(0, np.int32), np.zeros(0, np.float32)
            rows[4] = np.arange(n, dtype=np.int32)
            vals[4] = (np.ones(n) / np.sqrt(n)).astype(np.float32)
            d["col_ptr"] = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
            d["row_idx"] = np.concatenate(rows).astype(np.int32)
            d["values"] = np.concatenate(vals).astype(np.float32)
        X, y = _dev(torch, d)
        probs.append(dict(X=X, y=y, T=10, lambda_min_ratio=0.1))
        host.append(d)
    outs = gs.lasso_solve_batch(probs)
    torch.cuda.synchronize()
    for d, o in zip(host, outs):
        Xf, yf = _oracle_design(d)
        _check_path(Xf, yf, o, orc, _np(o["lambdas"]), label=f"csc batch {d['n']}x{d['p']}")
    assert np.all(_np(outs[0]["beta"])[:, 3] == 0)
    # y = 0: zero paths at once
    d = host[2]
    X, _ = _dev(torch, d)
    got = gs.lasso_path(X, torch.zeros(d["n"], dtype=torch.float32, device="cuda"), T=3,
                        lambdas=[1.0, 0.5, 0.1])
    torch.cuda.synchronize()
    assert np.all(_np(got["beta"]) == 0) and np.all(_np(got["epochs"]) == 0)


def test_csc_rcv1_shape(torch):
    """The RCV1 shape, 20242 x 47236 with 0.16% of the entries (1.3 M
    nonzeros), 5 lambdas to lambda_max/3: every lambda certified, and the
    duality gap of the returned beta, recomputed on the host with a sparse
    product over all p columns, is within eps."""
    sp = pytest.importorskip("scipy.sparse")
    d = synth.sparse_text(6, 20242, 47236, 0.0016)
    X, y = _dev(torch, d)
    got = gs.lasso_path(X, y, T=5, lambda_min_ratio=1 / 3)
    torch.cuda.synchronize()
    assert got["rc"] == gs.GS_OK
    A = sp.csc_matrix((d["values"].astype(np.float64), d["row_idx"], d["col_ptr"]),
                      shape=(d["n"], d["p"]))
    yf = d["y"].astype(np.float64)
    eps = 1e-8 * (yf @ yf)
    B = _np(got["beta"])
    for t, lam in enumerate(_np(got["lambdas"])):
        rho = yf - A @ B[t]
        c = A.T @ rho
        M = np.abs(c).max()
        r2, ry = rho @ rho, yf @ rho
        al = np.clip(ry / (lam * r2), -1 / M, 1 / M) if r2 > 0 else 0.0
        G = 0.5 * r2 + lam * np.abs(B[t]).sum() - lam * al * ry + 0.5 * lam * lam * al * al * r2
        assert G <= eps * (1 + 1e-6), (t, G, eps)
