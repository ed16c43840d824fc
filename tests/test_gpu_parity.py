"""GPU parity: the HIP library (through its C ABI) against the CPU oracle on
the same seeded inputs.

Tolerances follow from the method (Sec. 3.2 and Proposition 1 of Fercoq,
Gramfort & Salmon): a gap G certifies ||X(beta - beta_hat)||^2 <= 2G and
||theta - theta_hat|| <= sqrt(2G)/lambda, so two certified solutions are
compared through these bounds; the oracle also re-certifies every GPU
iterate by recomputing its gap independently.  FP64 reductions on both sides
differ only by summation order, so pass-level scalars agree to ~1e-12.
"""
import numpy as np
import pytest

import paper_1505_03410_amd as gs
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    gs.load_library()  # fails loudly when the HIP library is missing
    return torch


def _dev(torch, X, y, ld_multiple=4):
    Xd = gs.colmajor_to_device(X, ld_multiple=ld_multiple)
    yd = torch.from_numpy(np.ascontiguousarray(y)).cuda()
    return Xd, yd


def _np(t):
    return t.detach().cpu().numpy()


def _f64(a):
    return np.asarray(a, dtype=np.float64)


# ------------------------------------------------------------------ screen

def _screen_case(torch, orc, X, y, beta, lam, active=None, ld_multiple=4):
    Xd, yd = _dev(torch, X, y, ld_multiple)
    bd = torch.from_numpy(np.ascontiguousarray(beta, dtype=np.float64)).cuda()
    ad = None if active is None else torch.from_numpy(active.astype(np.int32)).cuda()
    g = gs.screen(Xd, yd, bd, lam, ad)
    torch.cuda.synchronize()
    o = orc.screen(_f64(X), _f64(y), _f64(beta), lam, active)
    q = int(_np(g["q"])[0])
    kept = set(_np(g["active"])[:q].tolist())
    # scalars
    scale = 0.5 * o["rho_norm2"] + lam * o["l1"] + 1e-300
    assert abs(float(_np(g["gap"])[0]) - o["gap"]) <= 1e-10 * scale
    assert abs(float(_np(g["alpha"])[0]) - o["alpha"]) <= 1e-12 * abs(o["alpha"]) + 1e-300
    # the inflated radius the test uses: same rounding bound, computed apart
    r_dev = float(_np(g["radius"])[0])
    assert abs(r_dev - o["radius_inflated"]) <= 1e-9 * o["radius_inflated"] + 1e-300, \
        (r_dev, o["radius_inflated"])
    # c_j = x_j^T rho in FP64
    xn = np.linalg.norm(_f64(X)[:, o["active"]], axis=0)
    err = np.abs(_np(g["c"]) - o["c"])
    assert np.all(err <= 1e-12 * xn * np.sqrt(o["rho_norm2"]) + 1e-300)
    # safe: everything the exact formula keeps is kept; and the GPU keeps
    # nothing the test would drop with a margin of 1e-6
    ex = set(o["active"][o["keep_exact"]].tolist())
    assert ex <= kept
    mu = np.abs(o["alpha"] * o["c"]) + o["radius"] * xn
    loose = set(o["active"][mu >= 1 - 1e-6].tolist())
    assert kept <= loose
    assert list(_np(g["active"])[:q]) == sorted(kept)
    return g, o


def test_screen_c0_f64(torch, orc):
    d = synth.c0()
    X, y = d["X"], d["y"]
    lmax = np.abs(X.T @ y).max()
    rng = np.random.default_rng(0)
    for ratio in (0.9, 0.3, 0.1):
        beta = np.zeros(500)
        beta[rng.choice(500, 8, replace=False)] = 0.1 * rng.standard_normal(8)
        _screen_case(torch, orc, X, y, beta, ratio * lmax, ld_multiple=2)


def test_screen_null_active_takes_all_columns(torch):
    """Through the C ABI with active_in NULL and q_in 0 (the header's "all p"):
    the pass covers every column, exactly as with q_in = p."""
    import ctypes
    d = synth.c1()
    X, y = d["X"], d["y"]
    Xd, yd = _dev(torch, X, y)
    n, p = X.shape
    lam = 0.3 * float(np.abs(_f64(X).T @ _f64(y)).max())
    beta = torch.zeros(p, dtype=torch.float64, device="cuda")
    ref = gs.screen(Xd, yd, beta, lam)
    lib = gs.load_library()
    ws = torch.empty(lib.screen_workspace_size(n, p), dtype=torch.uint8, device="cuda")
    act = torch.empty(p, dtype=torch.int32, device="cuda")
    q = torch.zeros(1, dtype=torch.int32, device="cuda")
    sc = [torch.empty(1, dtype=torch.float64, device="cuda") for _ in range(3)]
    rc = lib.screen(n, p, Xd.stride(1), 0, Xd.data_ptr(), yd.data_ptr(), beta.data_ptr(),
                    lam, 0, None, 0, act.data_ptr(), q.data_ptr(), sc[0].data_ptr(),
                    sc[1].data_ptr(), sc[2].data_ptr(), None, ws.data_ptr(), ws.numel(), None)
    assert rc == 0
    torch.cuda.synchronize()
    qr = int(ref["q"].item())
    assert int(q.item()) == qr > 0
    assert torch.equal(act[:qr], ref["active"][:qr])
    assert float(sc[0].item()) == float(ref["gap"].item())


def test_screen_c1_f32_with_active_set(torch, orc):
    d = synth.c1()
    X, y = d["X"], d["y"]
    lmax = np.abs(_f64(X).T @ _f64(y)).max()
    lam = 0.2 * lmax
    r = orc.lasso_path(X, y, lambdas=[lmax, lam], K=40)  # a mid-run iterate
    beta = r["beta"][1]
    g, o = _screen_case(torch, orc, X, y, beta, lam)
    act = np.sort(np.random.default_rng(1).choice(7129, 3000, replace=False)).astype(np.int32)
    act = np.union1d(act, np.flatnonzero(beta)).astype(np.int32)
    _screen_case(torch, orc, X, y, beta, lam, active=act)


def test_screen_ragged_and_small(torch, orc):
    """n not a multiple of the vector width (scalar loads), tiny p, empty A."""
    for (n, p, ldm) in [(37, 5, 1), (37, 300, 4), (1, 40, 1), (130, 1, 4)]:
        d = synth.gaussian(n * 7 + p, n, p, k=min(3, p))
        X = d["X"].astype(np.float32)
        y = d["y"].astype(np.float32)
        lam = 0.3 * np.abs(_f64(X).T @ _f64(y)).max()
        _screen_case(torch, orc, X, y, np.zeros(p), lam, ld_multiple=ldm)
    d = synth.gaussian(3, 20, 50)
    X, y = d["X"].astype(np.float32), d["y"].astype(np.float32)
    g, o = _screen_case(torch, orc, X, y, np.zeros(50), 0.5,
                        active=np.zeros(0, np.int32))
    assert int(_np(g["q"])[0]) == 0


def test_screen_radius_covers_cancelling_y_rho(torch, orc):
    """The device's inflated radius contains the exact gap sphere of the dual
    point it returns (theta = alpha (y - X beta)) on a design where y^T rho
    cancels catastrophically, so the computed y^T rho is far from the exact
    one (Proposition 1 with the rounding bound)."""
    from fractions import Fraction as F
    import test_oracle_pins as pins
    x, y, rho = pins.cancelling_y_rho_case()
    X = x[:, None]
    lam = 1e-6
    Xd, yd = _dev(torch, X, y, 2)
    g = gs.screen(Xd, yd, torch.ones(1, dtype=torch.float64, device="cuda"), lam)
    torch.cuda.synchronize()
    alpha = float(_np(g["alpha"])[0])
    r = float(_np(g["radius"])[0])
    Gex = pins.exact_gap(y, rho, 1.0, lam, alpha)
    assert Gex <= F(0.5 * (lam * r) ** 2), (float(Gex), 0.5 * (lam * r) ** 2)


@pytest.mark.parametrize("full", [True])
def test_screen_c4_full_size_sampled(torch, orc, full):
    """The 1000 x 100000 (400 MB) sweep in the launch configuration the
    benchmark times: gap and alpha against the oracle, c_j on a sample of
    columns against FP64 dot products."""
    d = synth.c4()
    X, y = d["X"], d["y"]
    Xd, yd = _dev(torch, X, y)
    rng = np.random.default_rng(4)
    beta = np.zeros(X.shape[1])
    beta[rng.choice(X.shape[1], 40, replace=False)] = 0.05 * rng.standard_normal(40)
    bd = torch.from_numpy(beta).cuda()
    lmax = float(np.abs(_f64(X).T @ _f64(y)).max())
    lam = 0.3 * lmax
    g = gs.screen(Xd, yd, bd, lam)
    torch.cuda.synchronize()
    o = orc.screen(X, y, beta, lam)
    scale = 0.5 * o["rho_norm2"] + lam * o["l1"]
    assert abs(float(_np(g["gap"])[0]) - o["gap"]) <= 1e-10 * scale
    c = _np(g["c"])
    rho = _f64(y) - _f64(X) @ _f64(beta)
    js = rng.choice(X.shape[1], 2000, replace=False)
    ref = _f64(X)[:, js].T @ rho
    xn = np.linalg.norm(_f64(X)[:, js], axis=0)
    assert np.all(np.abs(c[js] - ref) <= 1e-12 * xn * np.linalg.norm(rho))
    q = int(_np(g["q"])[0])
    ex = set(o["active"][o["keep_exact"]].tolist())
    kept = set(_np(g["active"])[:q].tolist())
    assert ex <= kept and len(kept) - len(ex) <= max(5, len(ex) // 1000)


# ------------------------------------------------------------ GAP SAFE dome

def _dome_mu_all(orc, X, y, beta, lam, o):
    """mu_D(x_j) of the exact GAP SAFE dome for every column of o's active
    set, from the oracle's pass scalars (no rounding inflation)."""
    Xf, yf = _f64(X), _f64(y)
    al = o["alpha"]
    R = np.sqrt(max(al * al * o["rho_norm2"] - 2 * al * o["y_rho"] / lam + yf @ yf / lam ** 2, 0.0))
    rc2 = max(yf @ yf - o["rho_norm2"] - 2 * lam * o["l1"], 0.0) / lam ** 2
    act = o["active"]
    xty = Xf[:, act].T @ yf
    xn = np.linalg.norm(Xf[:, act], axis=0)
    return np.array([orc.dome_mu(xty[k], o["c"][k], xn[k], al, lam, R, rc2)
                     for k in range(len(act))])


def _screen_dome_case(torch, orc, X, y, beta, lam, active=None, ld_multiple=4):
    Xd, yd = _dev(torch, X, y, ld_multiple)
    bd = torch.from_numpy(np.ascontiguousarray(beta, dtype=np.float64)).cuda()
    ad = None if active is None else torch.from_numpy(active.astype(np.int32)).cuda()
    g = gs.screen(Xd, yd, bd, lam, ad, rule="dome")
    gsph = gs.screen(Xd, yd, bd, lam, ad, rule="sphere")
    torch.cuda.synchronize()
    o = orc.screen(_f64(X), _f64(y), _f64(beta), lam, active, rule="dome")
    q = int(_np(g["q"])[0])
    kept = set(_np(g["active"])[:q].tolist())
    qs = int(_np(gsph["q"])[0])
    kept_sph = set(_np(gsph["active"])[:qs].tolist())
    # gap, alpha and radius are those of the sphere pass
    assert abs(float(_np(g["gap"])[0]) - float(_np(gsph["gap"])[0])) == 0.0
    ex = set(o["active"][o["keep_exact"]].tolist())          # exact dome and sphere
    assert ex <= kept, sorted(ex - kept)[:10]
    mu = _dome_mu_all(orc, X, y, beta, lam, o)
    xn = np.linalg.norm(_f64(X)[:, o["active"]], axis=0)
    mu_s = np.abs(o["alpha"] * o["c"]) + o["radius"] * xn
    loose = set(o["active"][(mu >= 1 - 1e-6) & (mu_s >= 1 - 1e-6)].tolist())
    assert kept <= loose, sorted(kept - loose)[:10]
    assert kept <= kept_sph
    assert list(_np(g["active"])[:q]) == sorted(kept)
    return len(kept), len(kept_sph)


def test_screen_dome_kept_sets(torch, orc):
    """The device's GAP SAFE dome test (Sec. 3.2; appendix dome support
    function) keeps every column the exact dome and sphere keep, nothing the
    exact tests would drop with a margin of 1e-6, and a subset of the
    sphere's kept set; on these iterates it drops more than the sphere."""
    fewer = 0
    d = synth.c0()
    X, y = d["X"], d["y"]
    lmax = np.abs(X.T @ y).max()
    for ratio in (0.7, 0.3, 0.1):
        lam = ratio * lmax
        r = orc.lasso_path(X, y, lambdas=[lmax, lam], K=5)
        kd, ks = _screen_dome_case(torch, orc, X, y, r["beta"][1], lam, ld_multiple=2)
        fewer += kd < ks
    d = synth.c1()
    X, y = d["X"], d["y"]
    lmax = np.abs(_f64(X).T @ _f64(y)).max()
    for ratio, K in ((0.5, 10), (0.2, 30), (0.05, 60)):
        lam = ratio * lmax
        r = orc.lasso_path(X, y, lambdas=[lmax, lam], K=K)
        kd, ks = _screen_dome_case(torch, orc, X, y, r["beta"][1], lam)
        fewer += kd < ks
        act = np.union1d(np.sort(np.random.default_rng(K).choice(7129, 2500, replace=False)),
                         np.flatnonzero(r["beta"][1])).astype(np.int32)
        _screen_dome_case(torch, orc, X, y, r["beta"][1], lam, active=act)
    assert fewer >= 1


@pytest.mark.parametrize("schedule", ["narrow", "wide"])
def test_path_dome_c1(torch, orc, schedule):
    """The 72 x 7129 path (40 lambdas down to lambda_max/100) with the dome
    test on the narrow and the wide schedule: certified, beta against the
    tight oracle, and the same epochs and final active sets as the oracle
    running Algorithm 1 with the dome."""
    d = synth.c1()
    X, y = d["X"], d["y"]
    Xd, yd = _dev(torch, X, y)
    got = gs.lasso_path(Xd, yd, T=40, lambda_min_ratio=1e-2, rule="dome", schedule=schedule)
    torch.cuda.synchronize()
    assert got["rc"] == gs.GS_OK
    lams = _np(got["lambdas"])
    _check_path(X, y, got, orc, lams, label=f"c1 dome {schedule}")
    o = orc.lasso_path(X, y, lambdas=lams, rule="dome")
    np.testing.assert_array_equal(_np(got["epochs"]), o["epochs"])
    np.testing.assert_array_equal(_np(got["nactive"]), o["nactive"])
    sph = orc.lasso_path(X, y, lambdas=lams, rule="sphere")
    print(f"c1 dome [{schedule}]: epochs {int(o['epochs'].sum())} (sphere "
          f"{int(sph['epochs'].sum())}), final active {int(o['nactive'].sum())} (sphere "
          f"{int(sph['nactive'].sum())})")


@pytest.mark.parametrize("rule", ["static", "dynamic_safe", "st3"])
def test_path_comparison_rules(torch, orc, rule):
    """The comparison rules of Table 1 (wide schedule) on the 72 x 7129 path
    down to lambda_max/10: certified, beta against the tight oracle, and the
    same epochs and final active set sizes as the oracle with that rule."""
    d = synth.c1()
    X, y = d["X"], d["y"]
    Xd, yd = _dev(torch, X, y)
    got = gs.lasso_path(Xd, yd, T=12, lambda_min_ratio=0.1, rule=rule)
    torch.cuda.synchronize()
    assert got["rc"] == gs.GS_OK
    lams = _np(got["lambdas"])
    _check_path(X, y, got, orc, lams, label=f"c1 {rule}")
    o = orc.lasso_path(X, y, lambdas=lams, rule=rule)
    np.testing.assert_array_equal(_np(got["epochs"]), o["epochs"])
    np.testing.assert_array_equal(_np(got["nactive"]), o["nactive"])
    print(f"c1 {rule}: final active {_np(got['nactive']).tolist()}")


@pytest.mark.parametrize("alpha", [0.5, 0.9])
def test_path_elastic_net(torch, orc, alpha):
    """The elastic net (appendix, "Elastic-Net") through its augmented Lasso,
    kept implicit on the device, against the oracle that writes the augmented
    design out: certified gaps, the elastic net KKT conditions at the tight
    oracle solution's accuracy, beta against the oracle's at the same gap
    target, and the same epochs at every lambda."""
    d = synth.c1()
    X, y = d["X"][:, :1500], d["y"]
    Xd, yd = _dev(torch, X, y)
    got = gs.lasso_path(Xd, yd, T=15, lambda_min_ratio=0.05, enet_alpha=alpha)
    torch.cuda.synchronize()
    assert got["rc"] == gs.GS_OK
    lams = _np(got["lambdas"])
    Xf, yf = _f64(X), _f64(y)
    o = orc.enet_path(Xf, yf, alpha, T=15, delta=-np.log10(0.05))
    np.testing.assert_allclose(lams, o["lambdas"], rtol=1e-12)
    tight = orc.enet_path(Xf, yf, alpha, lambdas=lams, eps_rel=1e-13, K=10_000_000)
    B, gap = _np(got["beta"]), _np(got["gap"])
    yy = float(yf @ yf)
    assert np.all(_np(got["status"]) == 0) and np.all(gap <= 1e-8 * yy)
    for t, lam in enumerate(lams):
        # the augmented problem is strongly convex (ridge term): the gap
        # bounds ||beta - beta*||^2 <= 2 (G + G*) / ((1 - alpha) lam)
        db = np.linalg.norm(B[t] - tight["beta"][t])
        bound = np.sqrt(2 * (max(gap[t], 0) + max(tight["gap"][t], 0)) / ((1 - alpha) * lam))
        assert db <= bound * (1 + 1e-6) + 1e-12, (t, db, bound)
        nb = np.linalg.norm(o["beta"][t])
        if nb > 0:
            assert np.linalg.norm(B[t] - o["beta"][t]) / nb <= BETA_TOL
    np.testing.assert_array_equal(_np(got["epochs"]), o["epochs"])


# -------------------------------------------------------------------- paths

def _primal(Xf, yf, b, lam):
    r = Xf @ b - yf
    return 0.5 * r @ r + lam * np.abs(b).sum()


BETA_TOL = 1e-5  # relative l2 distance to the tight oracle solution


def _check_path(X, y, got, orc, lambdas, eps_rel=1e-8, tight=None, beta_tol=BETA_TOL,
                label="path"):
    """Check each returned beta against a tight oracle solution beta*
    (gap <= 1e-13 ||y||^2):
      * the reported gap bounds the suboptimality, P(beta) - P(beta*) <= G + G*,
        and ||X(beta - beta*)|| <= sqrt(2G) + sqrt(2G*) (Sec. 3.2 weak duality
        and the strong convexity of the quadratic in X beta);
      * ||beta - beta*|| / ||beta*|| <= beta_tol, or, where the design does not
        determine beta that closely from a gap of eps, within the bound those
        two facts give: beta - beta* lives on U = supp(beta) u supp(beta*), so
        ||beta - beta*|| <= (sqrt(2G) + sqrt(2G*)) / sigma_min(X_U).
    Returns the worst relative error and the lambdas that needed the bound
    (t, relative error, bound, sigma_min)."""
    Xf, yf = _f64(X), _f64(y)
    yy = float(yf @ yf)
    eps = eps_rel * yy
    B = _np(got["beta"])
    gap = _np(got["gap"])
    st = _np(got["status"])
    assert np.all(st == 0), st
    assert np.all(gap <= eps)
    if tight is None:
        tight = orc.lasso_path(Xf, yf, lambdas=lambdas, eps_rel=1e-13)
    worst, h4 = 0.0, []
    for t, lam in enumerate(lambdas):
        Gs = max(tight["gap"][t], 0.0)
        sub = _primal(Xf, yf, B[t], lam) - _primal(Xf, yf, tight["beta"][t], lam)
        assert sub <= gap[t] + Gs + 1e-12 * yy, (t, sub, gap[t])
        d = Xf @ (B[t] - tight["beta"][t])
        xbound = np.sqrt(2 * max(gap[t], 0)) + np.sqrt(2 * Gs)
        assert np.linalg.norm(d) <= xbound + 1e-9 * np.sqrt(yy)
        nb = np.linalg.norm(tight["beta"][t])
        if nb == 0:
            assert np.all(B[t] == 0)
            continue
        rel = np.linalg.norm(B[t] - tight["beta"][t]) / nb
        worst = max(worst, rel)
        if beta_tol is not None and rel > beta_tol:
            U = np.flatnonzero((B[t] != 0) | (tight["beta"][t] != 0))
            smin = np.linalg.svd(Xf[:, U], compute_uv=False).min() if len(U) <= Xf.shape[0] else 0.0
            bound = (xbound + 1e-9 * np.sqrt(yy)) / smin / nb if smin > 0 else np.inf
            assert rel <= bound, (label, t, rel, bound, smin)
            h4.append((t, rel, bound, smin))
    if h4:
        print(f"{label}: {len(h4)} of {len(lambdas)} lambdas beyond {beta_tol:g} relative, each "
              f"within its sigma_min bound: " +
              ", ".join(f"t={t} rel={r:.1e} bound={b:.1e} smin={s:.1e}" for t, r, b, s in h4[:8]))
    return worst, h4


@pytest.mark.parametrize("cd_mode", ["auto", "residual"])
def test_path_c0_f64(torch, orc, cd_mode):
    d = synth.c0()
    X, y = d["X"], d["y"]
    lmax = orc.precompute(X, y)["lambda_max"]
    lams = [lmax, lmax * d["lambda_ratio"]]
    Xd, yd = _dev(torch, X, y, 2)
    got = gs.lasso_path(Xd, yd, lambdas=lams, cd_mode=cd_mode)
    torch.cuda.synchronize()
    _check_path(X, y, got, orc, lams, beta_tol=1e-5)
    assert int(_np(got["epochs"])[0]) == 0
    assert np.all(_np(got["beta"])[0] == 0)


@pytest.mark.parametrize("cd_mode", ["auto", "residual"])
def test_path_c1_full(torch, orc, cd_mode):
    """The benchmark workload: 72 x 7129 FP32, 100 lambdas, delta = 3."""
    d = synth.c1()
    X, y = d["X"], d["y"]
    Xd, yd = _dev(torch, X, y)
    got = gs.lasso_path(Xd, yd, T=100, lambda_min_ratio=1e-3, cd_mode=cd_mode)
    torch.cuda.synchronize()
    assert got["rc"] == gs.GS_OK
    lams = _np(got["lambdas"])
    ref = orc.grid(orc.precompute(X, y)["lambda_max"], 100, 3.0)
    np.testing.assert_allclose(lams, ref, rtol=1e-13)
    worst, h4 = _check_path(X, y, got, orc, lams, label=f"c1[{cd_mode}]")
    # the integer trace of Algorithm 1: epochs run and the final safe active
    # set size at every lambda equal the oracle's (same readings, same eps)
    o = orc.lasso_path(X, y, T=100, delta=3.0)
    np.testing.assert_array_equal(_np(got["epochs"]), o["epochs"])
    np.testing.assert_array_equal(_np(got["nactive"]), o["nactive"])
    # and the same iterates: beta within 1e-5 relative l2 of the oracle's at
    # the same certified gap (gap <= 1e-8 ||y||^2), at every lambda
    B = _np(got["beta"])
    same = [np.linalg.norm(B[t] - o["beta"][t]) / max(np.linalg.norm(o["beta"][t]), 1e-300)
            for t in range(1, 100)]
    assert max(same) <= BETA_TOL, max(same)
    print(f"c1 path [{cd_mode}]: worst relative beta difference to the oracle at the same "
          f"gap target {max(same):.2e}")
    print(f"c1 path [{cd_mode}]: worst relative beta error vs tight oracle {worst:.2e} "
          f"({len(h4)} lambdas within the sigma_min bound instead of 1e-5), "
          f"epochs {int(_np(got['epochs']).sum())}")


def _wide_case(torch, orc, X, y, T, ratio, label):
    Xd, yd = _dev(torch, X, y)
    stats = torch.zeros(len(gs.STAT_NAMES), dtype=torch.int64, device="cuda")
    got = gs.lasso_path(Xd, yd, T=T, lambda_min_ratio=ratio, schedule="wide", stats=stats)
    torch.cuda.synchronize()
    assert got["rc"] == gs.GS_OK
    lams = _np(got["lambdas"])
    _check_path(X, y, got, orc, lams, label=label)
    # the CD rounds are cyclic CD itself: the same epochs and final active
    # set sizes as the oracle at every lambda
    o = orc.lasso_path(X, y, lambdas=lams)
    np.testing.assert_array_equal(_np(got["epochs"]), o["epochs"])
    np.testing.assert_array_equal(_np(got["nactive"]), o["nactive"])
    st = dict(zip(gs.STAT_NAMES, stats.cpu().tolist()))
    assert st["residual_epochs"] == int(o["epochs"].sum())
    assert st["passes"] == int(o["passes"].sum())
    print(f"{label}: epochs {int(o['epochs'].sum())}, exact visits {st['wide_visits']}, "
          f"rounds {st['wide_rounds']}, re-anchors {st['wide_stops']}")
    return got, o, st


def test_path_wide_matches(torch, orc):
    """The wide schedule (sweeps over all CUs, CD rounds on one wavefront) on
    a C1-shaped problem."""
    d = synth.c1()
    X, y = d["X"][:, :3000], d["y"]
    _wide_case(torch, orc, X, y, 30, 1e-2, "wide c1-shaped")


def test_path_wide_c4_shaped(torch, orc):
    """The wide schedule on the 1000-row block-correlated design of the
    learned warm start workload at p = 4000, 20 lambdas down to
    lambda_max / 333: supports of up to 800 coefficients, so the CD rounds
    visit hundreds of coordinates exactly per epoch, skip the zero ones their
    anchor bound clears, and re-anchor when the residual moves too far."""
    d = synth.c4(seed=44, p=4000)
    got, o, st = _wide_case(torch, orc, d["X"], d["y"], 20, 0.003, "wide c4-shaped")
    # most of the design is never visited: at most a small multiple of the
    # supports' visits
    nnz = (o["beta"] != 0).sum(axis=1)
    assert st["wide_visits"] < 2 * int((o["epochs"] * np.maximum(nnz, 1)).sum()) + 4000 * 20


@pytest.mark.parametrize("cd_mode", ["auto", "residual"])
def test_path_large_n_configs(torch, orc, cd_mode):
    """Rows spread over 16 and 64 lanes (n = 300 and n = 1000), and a ragged
    n with scalar loads."""
    for n, p in [(300, 800), (1000, 600), (203, 500)]:
        d = synth.gaussian(n + p, n, p, k=20, sigma=0.5)
        X, y = d["X"].astype(np.float32), d["y"].astype(np.float32)
        Xd, yd = _dev(torch, X, y)
        got = gs.lasso_path(Xd, yd, T=12, lambda_min_ratio=0.01, cd_mode=cd_mode)
        torch.cuda.synchronize()
        _check_path(X, y, got, orc, _np(got["lambdas"]))


@pytest.mark.parametrize("cd_mode", ["auto", "residual"])
def test_path_n_above_1024(torch, orc, cd_mode):
    """The layouts for 1024 < n <= 2048: 16-byte loads (n = 1500, 2000) and
    scalar loads (n = 1203, 1999), p about 3000."""
    for n, p in [(1500, 3000), (2000, 2800), (1203, 3100), (1999, 2900)]:
        d = synth.gaussian(n * 3 + p, n, p, k=40, sigma=0.5)
        X, y = d["X"].astype(np.float32), d["y"].astype(np.float32)
        Xd, yd = _dev(torch, X, y)
        got = gs.lasso_path(Xd, yd, T=6, lambda_min_ratio=0.05, cd_mode=cd_mode,
                            schedule="narrow")
        torch.cuda.synchronize()
        _check_path(X, y, got, orc, _np(got["lambdas"]), label=f"n={n} p={p}")


def _c3_class(n):
    """The narrow layout class the library picks for an FP32 problem of n rows
    stored with ldx a multiple of 4: (16-byte loads?, smallest row capacity)."""
    vec = n % 4 == 0
    caps = ([32, 48, 64, 80, 96, 128, 192, 256, 384, 512, 768, 1024, 1536, 2048] if vec
            else [32, 48, 64, 96, 128, 256, 512, 1024, 2048])
    return vec, next(c for c in caps if c >= n)


def test_batch_c3_every_layout_class(torch, orc):
    """Problems drawn from the 512-problem uneven batch, two per layout class
    present in it (19 classes: every row capacity from 64 to 2048 rows, with
    16-byte and with scalar loads), solved together in one batch (groups of
    different layouts side by side) and each checked against the oracle at
    its full size."""
    params = synth.c3_params()
    classes = {}
    for b, pr in enumerate(params):
        classes.setdefault(_c3_class(pr["n"]), []).append(b)
    assert len(classes) == 19
    picks = []
    for key in sorted(classes):
        mem = sorted(classes[key], key=lambda b: params[b]["n"] * params[b]["p"] /
                     params[b]["lambda_ratio"] ** 0.5)
        picks += sorted({mem[0], mem[len(mem) // 3]})
    probs, host = [], []
    for b in picks:
        d = synth.c3_problem(params[b])
        Xd, yd = _dev(torch, d["X"], d["y"])
        probs.append(dict(X=Xd, y=yd, lambdas=[d["lambda_ratio"]], relative=True))
        host.append((b, d))
    outs = gs.lasso_solve_batch(probs)
    torch.cuda.synchronize()
    for (b, d), o in zip(host, outs):
        n, p = d["X"].shape
        _check_path(d["X"], d["y"], o, orc, _np(o["lambdas"]), label=f"c3[{b}] {n}x{p}")


def test_batch_c2_full(torch, orc):
    """The whole stability-selection workload: 256 row subsamples (36 rows) of
    the 72 x 7129 design, 100 lambdas each down to lambda_max / 100, replayed
    from the captured graph.  Every path is certified; 8 of them are checked
    against the tight oracle; the selection counts equal the nonzero counts
    of the returned paths."""
    d = synth.c2()
    X, y, rows = d["X"], d["y"], d["rows"]
    Xd, yd = _dev(torch, X, y)
    T = 100
    probs = [dict(X=Xd, y=yd, rows=torch.from_numpy(rows[b]).cuda(), T=T, lambda_min_ratio=1e-2)
             for b in range(rows.shape[0])]
    counts = torch.zeros((T, X.shape[1]), dtype=torch.int32, device="cuda")
    plan = gs.BatchPlan(probs, select_counts=counts)
    try:
        outs = plan.run()
        torch.cuda.synchronize()
        yy = (y.astype(np.float64)[rows] ** 2).sum(axis=1)
        sel = np.zeros((T, X.shape[1]), np.int64)
        for b, o in enumerate(outs):
            assert np.all(_np(o["status"]) == 0), b
            assert np.all(_np(o["gap"]) <= 1e-8 * yy[b]), b
            sel += (_np(o["beta"]) != 0)
        np.testing.assert_array_equal(_np(counts), sel)
        for b in np.random.default_rng(2).choice(rows.shape[0], 8, replace=False):
            _check_path(X[rows[b]], y[rows[b]], outs[b], orc, _np(outs[b]["lambdas"]),
                        label=f"c2[{b}]")
    finally:
        plan.close()


def test_batch_row_subsamples(torch, orc):
    """lasso_solve_batch with row subsamples of the C1 matrix (the stability
    selection workload at reduced count), plus the selection counts."""
    d = synth.c2(B=6)
    X, y, rows = d["X"], d["y"], d["rows"]
    Xd, yd = _dev(torch, X, y)
    probs, T = [], 40
    for b in range(rows.shape[0]):
        probs.append(dict(X=Xd, y=yd, rows=torch.from_numpy(rows[b]).cuda(), T=T,
                          lambda_min_ratio=1e-2))
    counts = torch.zeros((T, X.shape[1]), dtype=torch.int32, device="cuda")
    outs = gs.lasso_solve_batch(probs, select_counts=counts)
    torch.cuda.synchronize()
    sel = np.zeros((T, X.shape[1]), np.int32)
    for b, out in enumerate(outs):
        Xs, ys = X[rows[b]], y[rows[b]]
        _check_path(Xs, ys, out, orc, _np(out["lambdas"]))
        sel += (_np(out["beta"]) != 0)
    np.testing.assert_array_equal(_np(counts), sel)


# --------------------------------------------------------------- edge cases

def test_lambda_above_max_gives_zero(torch, orc):
    d = synth.c0()
    X, y = d["X"], d["y"]
    lmax = orc.precompute(X, y)["lambda_max"]
    Xd, yd = _dev(torch, X, y, 2)
    got = gs.lasso_path(Xd, yd, lambdas=[3.0, 1.0 + 1e-9], relative=True)
    torch.cuda.synchronize()
    assert np.all(_np(got["beta"]) == 0)
    assert np.all(_np(got["epochs"]) == 0)
    np.testing.assert_allclose(_np(got["lambdas"]), [3 * lmax, lmax * (1 + 1e-9)], rtol=1e-14)


def test_nonfinite_input_flagged(torch):
    d = synth.gaussian(1, 40, 100)
    X, y = d["X"].astype(np.float32), d["y"].astype(np.float32)
    X[3, 17] = np.nan
    Xd, yd = _dev(torch, X, y)
    got = gs.lasso_path(Xd, yd, T=5, lambda_min_ratio=0.1)
    torch.cuda.synchronize()
    assert np.all(_np(got["status"]) == 2)
    assert np.all(_np(got["beta"]) == 0)


def test_epoch_budget(torch, orc):
    """max_epochs reached: status 1 and a gap that is the true gap of the
    returned beta (the oracle recomputes it)."""
    d = synth.c1()
    X, y = d["X"][:, :2000], d["y"]
    Xd, yd = _dev(torch, X, y)
    lmax = orc.precompute(X, y)["lambda_max"]
    lam = 0.01 * lmax
    got = gs.lasso_path(Xd, yd, lambdas=[lam], max_epochs=7, schedule="narrow")
    torch.cuda.synchronize()
    assert got["rc"] == gs.GS_NOT_CONVERGED
    assert int(_np(got["status"])[0]) == 1 and int(_np(got["epochs"])[0]) == 7
    # the gap of the returned beta, recomputed by the oracle on the same
    # (full) active set: the first pass after the budget has not screened
    o1 = orc.screen(X, y, _np(got["beta"])[0], lam)
    assert _np(got["gap"])[0] <= o1["gap"] * (1 + 1e-9)
    # same budget in the oracle: same iterate up to rounding
    o = orc.lasso_path(X, y, lambdas=[lam], K=7)
    assert np.linalg.norm(_f64(X) @ (_np(got["beta"])[0] - o["beta"][0])) <= \
        1e-4 * np.linalg.norm(_f64(y))


def test_zero_column_and_tiny_shapes(torch, orc):
    d = synth.gaussian(5, 33, 70)
    X = d["X"].astype(np.float32)
    X[:, 10] = 0.0
    y = d["y"].astype(np.float32)
    for ldm in (1, 4):
        Xd, yd = _dev(torch, X, y, ldm)
        got = gs.lasso_path(Xd, yd, T=8, lambda_min_ratio=0.05)
        torch.cuda.synchronize()
        _check_path(X, y, got, orc, _np(got["lambdas"]))
        assert np.all(_np(got["beta"])[:, 10] == 0)
    for n, p in [(1, 3), (5, 1), (64, 2)]:
        d = synth.gaussian(n * 10 + p, n, p, k=1)
        X, y = d["X"].astype(np.float32), d["y"].astype(np.float32)
        Xd, yd = _dev(torch, X, y, 1)
        got = gs.lasso_path(Xd, yd, T=4, lambda_min_ratio=0.1)
        torch.cuda.synchronize()
        _check_path(X, y, got, orc, _np(got["lambdas"]))


def test_determinism_and_resume(torch, orc):
    """Two runs are bitwise equal; a path resumed at t = 6 from the stored
    beta^{lambda_5} (FP64, so the state is exact) equals the uninterrupted run."""
    d = synth.c0()
    X, y = d["X"], d["y"]
    Xd, yd = _dev(torch, X, y, 2)
    a = gs.lasso_path(Xd, yd, T=12, lambda_min_ratio=0.05)
    b = gs.lasso_path(Xd, yd, T=12, lambda_min_ratio=0.05)
    torch.cuda.synchronize()
    for k in ("beta", "gap", "epochs", "nactive"):
        assert np.array_equal(_np(a[k]), _np(b[k])), k
    lams = _np(a["lambdas"])
    c = gs.lasso_path(Xd, yd, lambdas=lams[6:], beta_init=a["beta"][5].contiguous())
    torch.cuda.synchronize()
    for k in ("beta", "gap", "epochs", "nactive"):
        assert np.array_equal(_np(c[k]), _np(a[k])[6:]), k


# ---------------------------------------------------- graph plans, autotuner

def test_batch_plan_replays_match(torch, orc):
    """A batch captured into a graph and replayed several times, with eager
    work and synchronizations between the replays: every replay reproduces
    the eager lasso_solve_batch results bit for bit, and those match the
    oracle."""
    d = synth.c2(B=8)
    X, y, rows = d["X"], d["y"], d["rows"]
    Xd, yd = _dev(torch, X, y)
    T = 30
    probs = [dict(X=Xd, y=yd, rows=torch.from_numpy(rows[b]).cuda(), T=T, lambda_min_ratio=1e-2)
             for b in range(rows.shape[0])]
    eager = gs.lasso_solve_batch(probs)
    torch.cuda.synchronize()
    ref = [(_np(o["beta"]).copy(), _np(o["gap"]).copy(), _np(o["epochs"]).copy()) for o in eager]
    for b in (0, 5):
        _check_path(X[rows[b]], y[rows[b]], eager[b], orc, _np(eager[b]["lambdas"]))
    counts = torch.zeros((T, X.shape[1]), dtype=torch.int32, device="cuda")
    plan = gs.BatchPlan(probs, select_counts=counts)
    try:
        for rep in range(3):
            for o in plan.outputs:
                o["beta"].fill_(7.0)
                o["gap"].fill_(-1.0)
            junk = torch.randn(1 << 16, device="cuda").sum()  # eager work between replays
            torch.cuda.synchronize()
            outs = plan.run()
            torch.cuda.synchronize()
            assert float(junk) == float(junk)
            for b, o in enumerate(outs):
                np.testing.assert_array_equal(_np(o["beta"]), ref[b][0])
                np.testing.assert_array_equal(_np(o["gap"]), ref[b][1])
                np.testing.assert_array_equal(_np(o["epochs"]), ref[b][2])
        sel = sum((r[0] != 0).astype(np.int32) for r in ref)
        np.testing.assert_array_equal(_np(counts), 3 * sel)  # counts accumulate per replay
    finally:
        plan.close()


def test_autotune_choices_and_results(torch, orc):
    """The autotuner picks, per class, a compiled layout that holds the
    class's rows; solving after tuning still matches the oracle."""
    gs.tune_reset()
    cases = [(36, 400, 11), (72, 600, 12), (150, 500, 13), (300, 700, 14)]
    probs, data = [], []
    for n, p, seed in cases:
        dd = synth.gaussian(seed, n, p)
        X, y = dd["X"].astype(np.float32), dd["y"].astype(np.float32)
        Xd, yd = _dev(torch, X, y)
        probs.append(dict(X=Xd, y=yd, T=8, lambda_min_ratio=0.05))
        data.append((X, y))
    choice = gs.autotune(probs, max_lambdas=3, sample=2)
    for (n, _p, _s), (S, NG) in zip(cases, choice):
        vec = 4 if n % 4 == 0 else 1  # 16-byte loads need n a multiple of 4
        assert S in (4, 16, 64) and NG >= 1
        assert S * NG * vec >= n
    outs = gs.lasso_solve_batch(probs)
    torch.cuda.synchronize()
    for (X, y), o in zip(data, outs):
        _check_path(X, y, o, orc, _np(o["lambdas"]))
    gs.tune_reset()


def test_batch_mixed_configs_concurrent_groups(torch, orc):
    """A batch whose problems need different tile configurations (row counts
    from 40 to 1000, FP32 and FP64): the groups run side by side on several
    streams, eagerly and from a captured graph; every path certifies against
    the oracle and the graph replays reproduce the eager results bit for
    bit."""
    shapes = [(40, 300, np.float32), (300, 800, np.float32), (1000, 600, np.float32),
              (203, 500, np.float32), (50, 500, np.float64), (120, 2000, np.float32)]
    probs, host = [], []
    for i, (n, p, dt) in enumerate(shapes):
        d = synth.gaussian(700 + i, n, p, k=10, sigma=0.3)
        X, y = d["X"].astype(dt), d["y"].astype(dt)
        Xd, yd = _dev(torch, X, y)
        probs.append(dict(X=Xd, y=yd, T=8, lambda_min_ratio=0.05))
        host.append((X, y))
    eager = gs.lasso_solve_batch(probs)
    torch.cuda.synchronize()
    for (X, y), o in zip(host, eager):
        _check_path(X, y, o, orc, _np(o["lambdas"]))
    ref = [(_np(o["beta"]).copy(), _np(o["epochs"]).copy()) for o in eager]
    plan = gs.BatchPlan(probs)
    try:
        for rep in range(2):
            for o in plan.outputs:
                o["beta"].fill_(3.0)
            torch.cuda.synchronize()
            outs = plan.run()
            torch.cuda.synchronize()
            for b, o in enumerate(outs):
                np.testing.assert_array_equal(_np(o["beta"]), ref[b][0])
                np.testing.assert_array_equal(_np(o["epochs"]), ref[b][1])
    finally:
        plan.close()


def test_autotune_schedule_moves_threshold(torch):
    """The schedule autotuner times both schedules on a small and a large
    problem (Gaussian designs, the first 3 lambdas of the grid: one wavefront
    for a whole large correlated design would take minutes); the FP32
    threshold ends on the right side of each measured size (between them
    when the small one is narrow-faster and the large one wide-faster), and
    lasso_path's auto schedule then runs the faster one on the large problem
    (its sweep or its path kernel shows in the timing)."""
    gs.tune_reset()
    small = synth.gaussian(31, 100, 2000)
    big = synth.gaussian(32, 400, 50000)
    res = []
    for d in (small, big):
        X, y = d["X"].astype(np.float32), d["y"].astype(np.float32)
        Xd, yd = _dev(torch, X, y)
        print(f"schedule autotuner: timing {X.shape}", flush=True)
        ch = gs.autotune_schedule(Xd, yd, T=100, lambda_min_ratio=1e-3, max_lambdas=3)
        print(f"schedule autotuner: {X.shape} -> {ch}", flush=True)
        res.append((X.shape[0] * X.shape[1], ch, Xd, yd, y))
    thr = gs.wide_threshold("f32")
    for npv, ch, *_ in res:
        assert (npv > thr) == (ch == "wide") or res[0][1] == "wide" and res[1][1] == "narrow", \
            (npv, ch, thr)
    npv, ch, Xd, yd, y = res[1]
    gs.timing_enable(True)
    gs.timing_reset()
    rel = 1e-3 ** (np.arange(100) / 99)
    r = gs.lasso_path(Xd, yd, lambdas=rel[:10], relative=True)
    torch.cuda.synchronize()
    sweep_n = gs.timing_query("sweep")[1]
    path_n = gs.timing_query("path")[1]
    gs.timing_enable(False)
    yy = float(np.sum(y.astype(np.float64) ** 2))
    assert np.all(_np(r["status"]) == 0) and np.all(_np(r["gap"]) <= 1e-8 * yy)
    ran_wide = sweep_n > 0 and path_n == 0
    assert ran_wide == (npv > thr)
    print(f"schedule autotuner: small {res[0][1]}, large {res[1][1]}, f32 threshold {thr:.4g}")
    gs.tune_reset()
    assert gs.wide_threshold("f32") == 16.0 * 1024 * 1024
