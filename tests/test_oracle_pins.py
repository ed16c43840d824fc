"""Pins for the CPU oracle: facts fixed by the paper or by mathematics, checked
without the oracle's own formulas.  These run without a GPU.

Each test names the passage of Fercoq, Gramfort & Salmon (ICML 2015) or the
textbook fact it relies on.
"""
import itertools

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _st(u, x):
    return np.sign(x) * np.maximum(np.abs(x) - u, 0.0)


def _small_c1_like(seed=11, n=72, p=400):
    rng = np.random.default_rng(seed)
    X = synth.ar1_columns(rng, n, p, 0.5)
    X -= X.mean(0)
    X /= X.std(0)
    beta = np.zeros(p)
    idx = rng.choice(p, 8, replace=False)
    beta[idx] = rng.choice([-1.0, 1.0], 8)
    s = X @ beta
    y = s + np.linalg.norm(s) / (3 * np.sqrt(n)) * rng.standard_normal(n)
    return X.astype(np.float32).astype(np.float64), y.astype(np.float32).astype(np.float64)


# --------------------------------------------------------------- lambda_max

def test_lambda_max_gives_zero(orc):
    """Sec. 1.2: for lambda >= lambda_max = ||X^T y||_inf, beta = 0 solves the
    Lasso, and theta = y/lambda makes the gap vanish."""
    d = synth.c0()
    X, y = d["X"], d["y"]
    lmax = np.abs(X.T @ y).max()
    r = orc.lasso_path(X, y, lambdas=[lmax * 2.0, lmax * (1 + 1e-9)])
    assert np.all(r["beta"] == 0.0)
    assert np.all(r["epochs"] == 0)
    assert np.all(np.abs(r["gap"]) <= 1e-12 * (y @ y))
    # Just below lambda_max the solution is nonzero, on the argmax coordinate.
    r2 = orc.lasso_path(X, y, lambdas=[lmax * (1 - 1e-3)], eps_rel=1e-14)
    nz = np.flatnonzero(r2["beta"][0])
    assert list(nz) == [int(np.argmax(np.abs(X.T @ y)))]
    # The largest correlation is taken in absolute value: flip y so that the
    # sign of the extreme correlation changes.
    for yy in (y, -y):
        assert np.isclose(orc.precompute(X, yy)["lambda_max"], lmax, rtol=1e-14)
        rr = orc.lasso_path(X, yy, lambdas=[1.0 + 1e-9], relative=True)
        assert np.isclose(rr["lambdas"][0], lmax * (1 + 1e-9), rtol=1e-14)
        assert np.all(rr["beta"] == 0.0)


# ----------------------------------------------------- orthonormal closed form

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_orthonormal_soft_threshold(orc, seed):
    """With X^T X = I the Lasso separates: beta_j = ST(lambda, x_j^T y)
    (Algorithm 1's update with ||x_j|| = 1 and x_j^T(X beta - y) =
    beta_j - x_j^T y).  CD reaches it in one epoch; at the solution the sphere
    test keeps exactly the equicorrelation set {j : |x_j^T y| >= lambda}
    (Sec. 2, equicorrelation set; Theorem 1).  At the exact solution those
    coordinates sit on the boundary |x_j^T theta| = 1, so the comparison uses
    the kept set with the rounding-inflated radius."""
    d = synth.orthonormal(seed, 60, 25)
    X, y = d["X"], d["y"]
    xty = X.T @ y
    a = np.sort(np.abs(xty))
    lam = 0.5 * (a[-8] + a[-9])               # 8 active, margin on both sides
    r = orc.lasso_path(X, y, lambdas=[lam], f=1, eps_rel=1e-13)
    want = _st(lam, xty)
    assert r["status"][0] == 0
    assert r["epochs"][0] == 1
    np.testing.assert_allclose(r["beta"][0], want, rtol=0, atol=1e-13)
    s = orc.screen(X, y, r["beta"][0], lam)
    assert s["gap"] <= 1e-12 * (y @ y)
    assert set(np.flatnonzero(s["keep_safe"])) == set(np.flatnonzero(np.abs(xty) >= lam))


# --------------------------------------------------------------------- KKT

@pytest.mark.parametrize("which", ["c0", "c1small"])
def test_kkt_at_tight_solution(orc, which):
    """Sec. 1.2 KKT: x_j^T theta = sign(beta_j) on the support and lies in
    [-1, 1] elsewhere, with theta = (y - X beta)/lambda (primal-dual link)."""
    if which == "c0":
        d = synth.c0()
        X, y = d["X"], d["y"]
    else:
        X, y = _small_c1_like()
    lmax = np.abs(X.T @ y).max()
    lams = lmax * np.array([0.5, 0.1, 0.02])
    r = orc.lasso_path(X, y, lambdas=lams, eps_rel=1e-14)
    assert np.all(r["status"] == 0)
    for t, lam in enumerate(lams):
        b = r["beta"][t]
        corr = X.T @ (y - X @ b) / lam
        assert np.abs(corr).max() <= 1 + 1e-6
        S = b != 0
        np.testing.assert_allclose(corr[S], np.sign(b[S]), atol=1e-6)


# ----------------------------------------------------- brute force, tiny p

def _brute_force_lasso(X, y, lam):
    """Textbook KKT enumeration: for every sign pattern s in {-1,0,1}^p with
    support S solve X_S^T X_S b = X_S^T y - lam s_S; accept when signs agree
    and |x_j^T (y - X_S b)| <= lam off S; return the minimum-objective one."""
    n, p = X.shape
    best, best_obj = None, np.inf
    for s in itertools.product((-1, 0, 1), repeat=p):
        s = np.array(s, dtype=float)
        S = np.flatnonzero(s)
        b = np.zeros(p)
        if len(S):
            XS = X[:, S]
            try:
                bS = np.linalg.solve(XS.T @ XS, XS.T @ y - lam * s[S])
            except np.linalg.LinAlgError:
                continue
            if np.any(np.sign(bS) != s[S]):
                continue
            b[S] = bS
        r = y - X @ b
        off = np.setdiff1d(np.arange(p), S)
        if len(off) and np.abs(X[:, off].T @ r).max() > lam * (1 + 1e-12):
            continue
        obj = 0.5 * r @ r + lam * np.abs(b).sum()
        if obj < best_obj:
            best, best_obj = b, obj
    return best


@pytest.mark.parametrize("n,p,seed", [(5, 7, 0), (20, 8, 1), (20, 6, 2), (5, 8, 3)])
def test_brute_force_tiny(orc, n, p, seed):
    d = synth.gaussian(100 + seed, n, p, k=3, sigma=0.3)
    X, y = d["X"], d["y"]
    lmax = np.abs(X.T @ y).max()
    for ratio in (0.6, 0.25, 0.08):
        lam = ratio * lmax
        want = _brute_force_lasso(X, y, lam)
        r = orc.lasso_path(X, y, lambdas=[lam], eps_rel=1e-15, K=2_000_000)
        np.testing.assert_allclose(r["beta"][0], want, rtol=0, atol=1e-7)


# -------------------------------------------- independent solver cross-check

def test_sklearn_cross_check(orc):
    """An independent coordinate-descent implementation (scikit-learn, whose
    objective is (1/2n)||y - X b||^2 + a||b||_1, so a = lambda/n) agrees at a
    tight tolerance."""
    sk = pytest.importorskip("sklearn.linear_model")
    d = synth.c0()
    X, y = d["X"], d["y"]
    n = X.shape[0]
    lam = 0.1 * np.abs(X.T @ y).max()
    r = orc.lasso_path(X, y, lambdas=[lam], eps_rel=1e-15, K=10_000_000)
    m = sk.Lasso(alpha=lam / n, fit_intercept=False, tol=1e-16,
                 max_iter=10_000_000).fit(X, y)
    np.testing.assert_allclose(r["beta"][0], m.coef_, atol=1e-7)


# ------------------------------------------------------------------ safety

def test_safety_invariant(orc):
    """Sec. 2, eq. of the safe test: every coordinate screened out at any pass
    is zero at the optimum.  The optimum is a separate, tighter run."""
    X, y = _small_c1_like()
    lmax = np.abs(X.T @ y).max()
    lams = lmax * np.geomspace(1, 1e-2, 15)
    r = orc.lasso_path(X, y, lambdas=lams, want_screened=True)
    tight = orc.lasso_path(X, y, lambdas=lams, eps_rel=1e-14)
    for t in range(len(lams)):
        scr = r["screened"][t].astype(bool)
        assert scr.sum() > 0 or t == 0
        assert np.all(tight["beta"][t][scr] == 0.0), t


def test_finite_identification(orc):
    """Theorem 1: as the GAP sphere shrinks, the safe active set equals the
    equicorrelation set {j : |x_j^T theta_hat| = 1}, computed here with numpy
    from the tight solution."""
    X, y = _small_c1_like(seed=5)
    lmax = np.abs(X.T @ y).max()
    lam = 0.05 * lmax
    r = orc.lasso_path(X, y, lambdas=[lam], eps_rel=1e-15, K=10_000_000)
    b = r["beta"][0]
    theta = (y - X @ b) / lam
    E = set(np.flatnonzero(np.abs(X.T @ theta) >= 1 - 1e-7))
    s = orc.screen(X, y, b, lam)
    assert set(np.flatnonzero(s["keep_exact"])) == E
    assert set(np.flatnonzero(b)) <= E


# ---------------------------------------------------------- gap and radius

def _feasible_theta(X, rng, scale=0.9):
    th = rng.standard_normal(X.shape[0])
    return scale * th / np.abs(X.T @ th).max()


def test_weak_duality_random_points(orc):
    """Sec. 3.2 (proof of Theorem 2): D(theta) <= P(beta) for every beta and
    every dual-feasible theta."""
    rng = np.random.default_rng(0)
    d = synth.gaussian(7, 30, 80)
    X, y = d["X"], d["y"]
    for _ in range(50):
        beta = rng.standard_normal(80) * (rng.random(80) < 0.2)
        th = _feasible_theta(X, rng, rng.uniform(0.1, 1.0))
        lam = rng.uniform(0.01, 1.0) * np.abs(X.T @ y).max()
        g, P, D = orc.gap(X, y, beta, th, lam)
        assert g >= -1e-12 * max(1.0, abs(P))


def test_prop3_sequential_identity(orc):
    """Proposition 3: r_t^2 = (l_{t-1}/l_t) r_{t-1}^2 + (1 - l_t/l_{t-1})
    ||(X beta - y)/l_t||^2 - (l_{t-1}/l_t - 1) ||theta||^2, r^2 = 2G/l^2."""
    rng = np.random.default_rng(1)
    d = synth.gaussian(8, 40, 120)
    X, y = d["X"], d["y"]
    for _ in range(20):
        beta = rng.standard_normal(120) * (rng.random(120) < 0.1)
        th = _feasible_theta(X, rng)
        l0 = rng.uniform(0.1, 1.0) * np.abs(X.T @ y).max()
        l1 = l0 * rng.uniform(0.3, 0.99)
        g0 = orc.gap(X, y, beta, th, l0)[0]
        g1 = orc.gap(X, y, beta, th, l1)[0]
        lhs = 2 * g1 / l1 ** 2
        res = X @ beta - y
        rhs = (l0 / l1) * 2 * g0 / l0 ** 2 + (1 - l1 / l0) * (res @ res) / l1 ** 2 \
            - (l0 / l1 - 1) * (th @ th)
        assert abs(lhs - rhs) <= 1e-10 * max(1.0, abs(lhs))


def test_pass_gap_matches_definition(orc):
    """The screening pass's gap equals P(beta) - D(alpha rho) with theta from
    the rescaled residual (Sec. 2.3), and theta is dual feasible."""
    rng = np.random.default_rng(2)
    X, y = _small_c1_like(seed=3)
    lmax = np.abs(X.T @ y).max()
    for _ in range(10):
        beta = 0.3 * rng.standard_normal(X.shape[1]) * (rng.random(X.shape[1]) < 0.05)
        lam = rng.uniform(0.01, 0.9) * lmax
        s = orc.screen(X, y, beta, lam)
        rho = y - X @ beta
        theta = s["alpha"] * rho
        assert np.abs(X.T @ theta).max() <= 1 + 1e-12
        g = orc.gap(X, y, beta, theta, lam)[0]
        assert abs(s["gap"] - g) <= 1e-9 * max(1.0, abs(g))
        # theta is the point of Delta along rho closest to y/lambda (Sec. 2.3)
        ts = np.linspace(-1, 1, 2001) / np.abs(X.T @ rho).max()
        dist = [np.linalg.norm(a * rho - y / lam) for a in ts]
        assert np.linalg.norm(theta - y / lam) <= min(dist) + 1e-12


def test_radius_bounds_thm2_prop1(orc):
    """Theorem 2 / Proposition 1: r_tilde = sqrt(R^2 - r_check^2) <= r =
    sqrt(2G)/lambda, and the ball B(theta, r) contains theta_hat (from a
    tight solve)."""
    rng = np.random.default_rng(4)
    X, y = _small_c1_like(seed=4)
    lmax = np.abs(X.T @ y).max()
    lam = 0.1 * lmax
    tight = orc.lasso_path(X, y, lambdas=[lam], eps_rel=1e-15, K=10_000_000)
    th_hat = (y - X @ tight["beta"][0]) / lam
    for K in (0, 3, 10, 30, 100):
        r = orc.lasso_path(X, y, lambdas=[lam], K=K, eps_rel=1e-30)
        b = r["beta"][0]
        s = orc.screen(X, y, b, lam)
        theta = s["alpha"] * (y - X @ b)
        R = np.linalg.norm(theta - y / lam)
        res = X @ b - y
        rc2 = max(y @ y - res @ res - 2 * lam * np.abs(b).sum(), 0.0) / lam ** 2
        # R^2 - r_check^2 cancels: its rounding error scales with R^2 + r_check^2
        assert R * R - rc2 <= s["radius"] ** 2 * (1 + 1e-9) + 1e-13 * (R * R + rc2)
        assert np.linalg.norm(theta - th_hat) <= s["radius"] * (1 + 1e-9) + 1e-12
    # Proposition 2: the radius goes to zero with the iterates.
    assert s["radius"] < 1e-3


def test_inflated_test_is_superset(orc):
    """The rounding-inflated kept set contains the exact-formula one."""
    X, y = _small_c1_like(seed=6)
    rng = np.random.default_rng(6)
    lmax = np.abs(X.T @ y).max()
    for _ in range(5):
        beta = 0.2 * rng.standard_normal(X.shape[1]) * (rng.random(X.shape[1]) < 0.05)
        s = orc.screen(X, y, beta, rng.uniform(0.05, 0.9) * lmax)
        assert np.all(s["keep_safe"] >= s["keep_exact"])
        # Proposition 1's radius sqrt(2G)/lambda, inflated only by rounding.
        assert s["radius"] <= s["radius_inflated"] <= s["radius"] * (1 + 1e-6) + 1e-9


def cancelling_y_rho_case(n=1000):
    """A one-column design whose residual rho = y - x (beta = 1, computed
    exactly) makes y^T rho cancel catastrophically in ascending-row order:
    a product of 2^20, n - 3 products of -2^-34 (each below half an ulp of
    the running sum, so all are lost), -2^20, then v = 2^-19.  The computed
    y^T rho is v; the exact value is v - (n - 3) 2^-34.  Returns (x, y, rho)
    with every entry exactly representable and y - x == rho exactly."""
    v = 2.0 ** -19
    rho = np.full(n, -2.0 ** -34)
    y = np.ones(n)
    rho[0], y[0] = 2.0 ** -10, 2.0 ** 30
    rho[n - 2], y[n - 2] = -2.0 ** -10, 2.0 ** 30
    rho[n - 1], y[n - 1] = v, 1.0
    x = y - rho
    assert np.all(y - x == rho) and np.all(x + rho == y)
    return x, y, rho


def exact_gap(y, rho, beta_l1, lam, alpha):
    """P(beta) - D(alpha rho) in exact rational arithmetic for a beta whose
    exact residual is rho (Sec. 1.1: primal and dual objectives)."""
    from fractions import Fraction as F
    L, a = F(lam), F(alpha)
    yF = [F(t) for t in y]
    rF = [F(t) for t in rho]
    P = sum(t * t for t in rF) / 2 + L * F(beta_l1)
    D = sum(t * t for t in yF) / 2 - L * L / 2 * sum((a * r - t / L) ** 2 for r, t in zip(rF, yF))
    return P - D


def test_rounding_bound_covers_cancelling_y_rho(orc):
    """The inflated radius must contain the true gap sphere at the dual point
    the pass actually uses, theta = alpha_s rho~ (Proposition 1 applied to
    the exact gap of that point).  y^T rho is a dot product whose terms have
    both signs, so its rounding error is bounded by gamma_n ||y|| ||rho||,
    not by a multiple of its own value: in this constructed case the exact
    gap exceeds the computed one by lambda alpha (n - 3) 2^-34, which only
    that term of the bound covers."""
    from fractions import Fraction as F
    x, y, rho = cancelling_y_rho_case()
    n = len(y)
    lam = 1e-6
    s = orc.screen(x[:, None], y, np.array([1.0]), lam)
    assert s["y_rho"] == 2.0 ** -19                      # the lost terms are gone
    Gex = exact_gap(y, rho, 1.0, lam, s["alpha_safe"])
    R2, Ry, al = s["rho_norm2"], s["y_rho"], s["alpha_safe"]
    Gs = 0.5 * R2 + lam * 1.0 - lam * al * Ry + 0.5 * lam * lam * al * al * R2
    # the computed gap misses lambda alpha times the lost part of y^T rho
    miss = Gex - F(Gs)
    assert abs(miss - F(lam) * F(al) * (n - 3) * F(2.0 ** -34)) <= F(1e-3) * miss
    assert Gex <= F(max(Gs, 0.0) + s["err_gap"])          # covered by the bound
    assert Gex <= F(0.5 * (lam * s["radius_inflated"]) ** 2)
    # a bound charging only a relative error of the computed y^T rho (its
    # other terms are below 1e-9 here) would not cover it
    assert miss > F(1e-9)


# ----------------------------------------------------------------- the grid

def test_grid(orc):
    """Sec. 3.3: lambda_t = lambda_max 10^(-delta t/(T-1)), t = 0..T-1."""
    g = orc.grid(2.5, 100, 3.0)
    assert g[0] == 2.5
    assert np.isclose(g[-1], 2.5e-3, rtol=1e-14)
    ratios = g[1:] / g[:-1]
    np.testing.assert_allclose(ratios, 10 ** (-3 / 99), rtol=1e-13)


# ------------------------------------------------------------- edge cases

def test_zero_column_and_duplicates(orc):
    """A zero column is always screened and stays zero (its test value is 0).
    Duplicated columns make beta non-unique but theta unique (Sec. 1.1): the
    fit X beta and theta agree with the de-duplicated problem."""
    d = synth.gaussian(9, 30, 40)
    X, y = d["X"].copy(), d["y"]
    X[:, 5] = 0.0
    Xd = np.concatenate([X, X[:, :3]], axis=1)
    lam = 0.2 * np.abs(X.T @ y).max()
    r = orc.lasso_path(X, y, lambdas=[lam], eps_rel=1e-14)
    assert r["beta"][0][5] == 0.0
    rd = orc.lasso_path(Xd, y, lambdas=[lam], eps_rel=1e-14)
    np.testing.assert_allclose(X @ r["beta"][0], Xd @ rd["beta"][0], atol=1e-6)
    s = orc.screen(X, y, r["beta"][0], lam)
    assert not s["keep_exact"][5]


def test_epoch_budget_not_converged(orc):
    """With a tiny epoch budget the path reports 'not converged' and a gap that
    is the true gap of the returned beta (certified)."""
    X, y = _small_c1_like(seed=8)
    lam = 0.01 * np.abs(X.T @ y).max()
    r = orc.lasso_path(X, y, lambdas=[lam], K=5)
    assert r["status"][0] == 1 and r["rc"] == 1
    assert r["epochs"][0] == 5
    s = orc.screen(X, y, r["beta"][0], lam)
    assert np.isclose(r["gap"][0], s["gap"], rtol=1e-9)
    assert r["gap"][0] > 1e-8 * (y @ y)


def test_invalid_arguments(orc):
    d = synth.gaussian(1, 10, 12)
    with pytest.raises(ValueError):
        orc.lasso_path(d["X"], d["y"], lambdas=[1.0, 2.0])      # increasing grid
    with pytest.raises(ValueError):
        orc.lasso_path(d["X"], d["y"], lambdas=[-1.0])          # lambda <= 0
    with pytest.raises(ValueError):
        orc.lasso_path(d["X"], d["y"], lambdas=[1.0], f=0)      # f < 1


def test_all_zero_design(orc):
    """With X = 0 every beta is optimal at 0 and theta_hat = y/lambda (the dual
    set is all of R^n): the gap vanishes with no epoch and nothing is kept."""
    X = np.zeros((12, 9))
    y = np.random.default_rng(0).standard_normal(12)
    r = orc.lasso_path(X, y, lambdas=[0.5, 0.1])
    assert np.all(r["beta"] == 0) and np.all(r["status"] == 0)
    assert np.all(r["epochs"] == 0)
    s = orc.screen(X, y, np.zeros(9), 0.1)
    assert not s["keep_safe"].any()
    assert abs(s["gap"]) <= 1e-12 * (y @ y)


# ------------------------------------------------------------ GAP SAFE dome

def _dome_geometry(X, y, beta, lam, alpha):
    """Center, radius, ratio and normal of the GAP SAFE dome (Sec. 3.2,
    appendix "Dome test") at (beta, theta = alpha rho), from the definitions
    (numpy, not the oracle's formulas): c = (y/lambda + theta)/2,
    r = R_hat/2, a = 2 (r_check[beta]/R_hat)^2 - 1, w = (y/lambda - theta)/R_hat."""
    rho = y - X @ beta
    theta = alpha * rho
    R = np.linalg.norm(theta - y / lam)
    rc2 = max(y @ y - rho @ rho - 2 * lam * np.abs(beta).sum(), 0.0) / lam ** 2
    return (y / lam + theta) / 2, R / 2, 2 * rc2 / R ** 2 - 1, (y / lam - theta) / R, R, rc2


def _dome_iterates(orc, seed):
    X, y = _small_c1_like(seed=seed, n=12, p=30)
    lmax = np.abs(X.T @ y).max()
    lam = 0.2 * lmax
    out = []
    for K in (1, 3, 8, 20):
        b = orc.lasso_path(X, y, lambdas=[lam], K=K, eps_rel=1e-30)["beta"][0]
        out.append((X, y, b, lam))
    return out


def _dome_max_brute(x, c, r, a, w, m=400001):
    """max of x^T t over the dome by brute force: t = c + u w + v e with e the
    unit direction of x's part orthogonal to w (any component of t - c
    outside span{w, x} leaves x^T t unchanged and only uses up radius, so the
    maximum lies in that plane); the maximum of a linear function over the
    cut disk lies on its boundary, which is sampled densely: the arc of the
    circle of radius r with u <= -a r, and the chord u = -a r."""
    xw = x @ w
    xo = np.linalg.norm(x - xw * w)
    ph = np.linspace(0.0, 2.0 * np.pi, m)
    u, v = r * np.cos(ph), r * np.sin(ph)
    arc = np.where(u <= -a * r, u * xw + v * xo, -np.inf).max()
    half = r * np.sqrt(max(1.0 - a * a, 0.0))
    vc = np.linspace(-half, half, m)
    chord = (-a * r * xw + vc * xo).max()
    return c @ x + max(arc, chord)


def test_dome_support_matches_brute_force(orc):
    """The closed-form support function of the dome (appendix, "Dome test")
    equals a brute-force maximum of |x_j^T t| over the dome."""
    checked = 0
    for seed in (21, 22):
        for X, y, b, lam in _dome_iterates(orc, seed):
            s = orc.screen(X, y, b, lam)
            c, r, a, w, R, rc2 = _dome_geometry(X, y, b, lam, s["alpha"])
            for j in range(0, X.shape[1], 3):
                x = X[:, j]
                best = max(_dome_max_brute(x, c, r, a, w), _dome_max_brute(-x, c, r, a, w))
                mu = orc.dome_mu(x @ y, s["c"][j], np.linalg.norm(x), s["alpha"], lam, R, rc2)
                # boundary sampled every 2 pi / 400000 radians: error ~1e-10 r ||x||
                tol = 1e-8 * (1.0 + r * np.linalg.norm(x))
                assert abs(mu - best) <= tol, (j, mu, best)
                checked += 1
    assert checked >= 50


def test_dome_contains_dual_optimum_and_lies_in_sphere(orc):
    """The GAP SAFE dome holds theta_hat (Theorem 2's annulus intersected
    with the ball of diameter [theta, y/lambda], since theta_hat is the
    projection of y/lambda on the dual set), and it lies inside the GAP SAFE
    sphere: its kept set is a subset of the sphere's."""
    for seed in (23, 24, 25):
        X, y = _small_c1_like(seed=seed, n=20, p=60)
        lmax = np.abs(X.T @ y).max()
        for ratio in (0.5, 0.1):
            lam = ratio * lmax
            tight = orc.lasso_path(X, y, lambdas=[lam], eps_rel=1e-15, K=10_000_000)
            th = (y - X @ tight["beta"][0]) / lam
            for K in (0, 2, 10, 40):
                b = orc.lasso_path(X, y, lambdas=[lam], K=K, eps_rel=1e-30)["beta"][0]
                s = orc.screen(X, y, b, lam, rule="dome")
                c, r, a, w, R, rc2 = _dome_geometry(X, y, b, lam, s["alpha"])
                assert np.linalg.norm(th - c) <= r * (1 + 1e-9) + 1e-12
                assert w @ (th - c) <= -a * r + 1e-9 * r + 1e-12
                sph = orc.screen(X, y, b, lam, rule="sphere")
                assert np.all(s["keep_exact"] <= sph["keep_exact"])
                assert np.all(s["keep_safe"] >= s["keep_exact"])
                assert np.all(s["keep_safe"] <= sph["keep_safe"])


def test_dome_reduces_to_ball_when_r_check_vanishes(orc):
    """With r_check = 0 the ratio is -1: the dome is the whole ball of
    diameter [theta, y/lambda] and mu_D(x) = |c^T x| + r ||x||."""
    rng = np.random.default_rng(26)
    for _ in range(20):
        n = 6
        x, y, rho = rng.standard_normal(n), rng.standard_normal(n), rng.standard_normal(n)
        alpha, lam = rng.uniform(0.5, 2), rng.uniform(0.5, 2)
        R = np.linalg.norm(alpha * rho - y / lam)
        mu = orc.dome_mu(x @ y, x @ rho, np.linalg.norm(x), alpha, lam, R, 0.0)
        cx = 0.5 * (x @ y / lam + alpha * (x @ rho))
        assert abs(mu - (abs(cx) + 0.5 * R * np.linalg.norm(x))) <= 1e-13 * (1 + abs(mu))


def test_dome_path_is_safe_and_matches_sphere_path(orc):
    """Algorithm 1 with the dome test: every coordinate the dome screens is
    zero at the tight solution, and the certified path agrees with the
    sphere path within the gap bound."""
    X, y = _small_c1_like(seed=27, n=40, p=300)
    lmax = np.abs(X.T @ y).max()
    lams = lmax * 10 ** (-np.arange(12) / 11 * 1.5)
    dome = orc.lasso_path(X, y, lambdas=lams, rule="dome", want_screened=True)
    sph = orc.lasso_path(X, y, lambdas=lams, rule="sphere")
    tight = orc.lasso_path(X, y, lambdas=lams, eps_rel=1e-15, K=10_000_000)
    assert np.all(dome["status"] == 0)
    for t in range(len(lams)):
        scr = dome["screened"][t].astype(bool)
        assert np.all(tight["beta"][t][scr] == 0)
        d = X @ (dome["beta"][t] - sph["beta"][t])
        assert np.linalg.norm(d) <= np.sqrt(2 * dome["gap"][t]) + np.sqrt(2 * sph["gap"][t]) + 1e-12
    # the dome never keeps more than the sphere at the first pass of a lambda
    assert dome["nactive"].sum() <= sph["nactive"].sum()


# ------------------------------------------------ comparison rules (Table 1)

def _rule_ball(X, y, beta, lam, alpha, rule):
    """Center and radius of the comparison rules of Table 1 from their
    definitions: static SAFE B(y/lambda, ||y|| |1/lambda - 1/lambda_max|)
    (Sec. 2.1), Dynamic Safe B(y/lambda, ||theta - y/lambda||) (Sec. 2.3),
    Dynamic ST3: B(y/lambda, R_hat) cut by s* x*^T t <= 1, held in the ball
    around the projection of y/lambda on that plane."""
    xty = X.T @ y
    js = int(np.argmax(np.abs(xty)))
    lmax, s = abs(xty[js]), np.sign(xty[js])
    xs = X[:, js]
    theta = alpha * (y - X @ beta)
    R = np.linalg.norm(theta - y / lam)
    if rule == "static":
        return y / lam, np.linalg.norm(y) * abs(1 / lam - 1 / lmax)
    if rule == "dynamic_safe" or lam >= lmax:
        return y / lam, R
    # projection of y/lambda on the plane s x*^T t = 1
    h = (s * xs @ (y / lam) - 1.0) / (xs @ xs)
    center = y / lam - h * s * xs
    dist = np.linalg.norm(center - y / lam)
    return center, np.sqrt(max(R * R - dist * dist, 0.0))


@pytest.mark.parametrize("rule", ["static", "dynamic_safe", "st3"])
def test_comparison_rules_hold_dual_optimum(orc, rule):
    """Each comparison region of Table 1 holds theta_hat (from a tight
    solve), and the oracle's exact kept set for the rule is the sphere test
    of that region; the rounding-safe kept set contains it."""
    for seed in (31, 32):
        X, y = _small_c1_like(seed=seed, n=20, p=80)
        lmax = np.abs(X.T @ y).max()
        for ratio in (0.9, 0.5, 0.2):
            lam = ratio * lmax
            tight = orc.lasso_path(X, y, lambdas=[lam], eps_rel=1e-15, K=10_000_000)
            th = (y - X @ tight["beta"][0]) / lam
            for K in (0, 3, 20):
                b = orc.lasso_path(X, y, lambdas=[lam], K=K, eps_rel=1e-30)["beta"][0]
                o = orc.screen(X, y, b, lam, rule=rule)
                c, r = _rule_ball(X, y, b, lam, o["alpha"], rule)
                assert np.linalg.norm(th - c) <= r * (1 + 1e-9) + 1e-12, (rule, ratio, K)
                mu = np.abs(X.T @ c) + r * np.linalg.norm(X, axis=0)
                sure = (mu >= 1 + 1e-9) | (mu < 1 - 1e-9)
                assert np.array_equal(o["keep_exact"][sure], (mu >= 1)[sure])
                assert np.all(o["keep_safe"] >= o["keep_exact"])


def test_static_safe_critical_ratio(orc):
    """Sec. 2.1, first example: the static SAFE rule screens nothing once
    lambda/lambda_max <= min_j (1 + |x_j^T y|/(||x_j|| ||y||)) /
    (1 + lambda_max/(||x_j|| ||y||)), and at lambda = lambda_max it keeps
    only the columns reaching the maximum."""
    X, y = _small_c1_like(seed=33, n=30, p=200)
    xty = X.T @ y
    lmax = np.abs(xty).max()
    xn = np.linalg.norm(X, axis=0)
    yn = np.linalg.norm(y)
    crit = np.min((1 + np.abs(xty) / (xn * yn)) / (1 + lmax / (xn * yn)))
    below = orc.screen(X, y, np.zeros(200), crit * lmax * (1 - 1e-6), rule="static")
    assert below["keep_exact"].all()
    above = orc.screen(X, y, np.zeros(200), crit * lmax * (1 + 1e-3), rule="static")
    assert not above["keep_exact"].all()
    at = orc.screen(X, y, np.zeros(200), lmax, rule="static")
    assert np.array_equal(np.flatnonzero(at["keep_exact"]),
                          np.flatnonzero(np.abs(xty) >= lmax))


@pytest.mark.parametrize("rule", ["static", "dynamic_safe", "st3"])
def test_comparison_rule_paths_are_safe(orc, rule):
    """Algorithm 1 with each comparison rule: certified, every screened
    coordinate is zero at the tight solution, and the path agrees with the
    GAP SAFE one within the gap bound."""
    X, y = _small_c1_like(seed=34, n=40, p=300)
    lmax = np.abs(X.T @ y).max()
    lams = lmax * 10 ** (-np.arange(10) / 9 * 1.5)
    got = orc.lasso_path(X, y, lambdas=lams, rule=rule, want_screened=True)
    gap = orc.lasso_path(X, y, lambdas=lams, rule="sphere")
    tight = orc.lasso_path(X, y, lambdas=lams, eps_rel=1e-15, K=10_000_000)
    assert np.all(got["status"] == 0)
    for t in range(len(lams)):
        scr = got["screened"][t].astype(bool)
        assert np.all(tight["beta"][t][scr] == 0)
        d = X @ (got["beta"][t] - gap["beta"][t])
        assert np.linalg.norm(d) <= np.sqrt(2 * got["gap"][t]) + np.sqrt(2 * gap["gap"][t]) + 1e-12


# ------------------------------------------------------------ elastic net

def test_enet_orthonormal_closed_form(orc):
    """Orthonormal X: the elastic net solution is
    ST(alpha lambda, x_j^T y) / (1 + (1 - alpha) lambda) (Zou & Hastie's
    naive elastic net on an orthonormal design)."""
    d = synth.orthonormal(41, 30, 12)
    X, y = d["X"], d["y"]
    for alpha in (0.3, 0.7):
        r = orc.enet_path(X, y, alpha, T=6, delta=1.0, eps_rel=1e-14)
        for t, lam in enumerate(r["lambdas"]):
            want = _st(alpha * lam, X.T @ y) / (1 + (1 - alpha) * lam)
            np.testing.assert_allclose(r["beta"][t], want, rtol=1e-9, atol=1e-12)


def test_enet_kkt_and_lasso_limit(orc):
    """KKT of the elastic net at a tight solution:
    x_j^T (y - X b) - (1 - alpha) lambda b_j = alpha lambda sign(b_j) on the
    support, |.| <= alpha lambda off it; and alpha = 1 gives the Lasso path."""
    X, y = _small_c1_like(seed=42, n=30, p=80)
    r = orc.enet_path(X, y, 0.5, T=8, delta=1.5, eps_rel=1e-15, K=10_000_000)
    for t, lam in enumerate(r["lambdas"]):
        b = r["beta"][t]
        g = X.T @ (y - X @ b) - 0.5 * lam * b
        on = b != 0
        np.testing.assert_allclose(g[on], 0.5 * lam * np.sign(b[on]), rtol=1e-7, atol=1e-9)
        assert np.all(np.abs(g[~on]) <= 0.5 * lam * (1 + 1e-7))
    lasso = orc.lasso_path(X, y, T=8, delta=1.5, eps_rel=1e-12)
    enet1 = orc.enet_path(X, y, 1.0, T=8, delta=1.5, eps_rel=1e-12)
    np.testing.assert_allclose(enet1["lambdas"], lasso["lambdas"], rtol=1e-14)
    for t in range(8):
        d = X @ (enet1["beta"][t] - lasso["beta"][t])
        assert np.linalg.norm(d) <= (np.sqrt(2 * max(enet1["gap"][t], 0.0)) +
                                     np.sqrt(2 * max(lasso["gap"][t], 0.0)) + 1e-12)


def test_enet_sklearn_cross_check(orc):
    """scikit-learn's ElasticNet minimizes 1/(2n)||y - X b||^2 + a r ||b||_1 +
    a (1 - r)/2 ||b||^2, so a = lambda/n and r = alpha give the same problem."""
    sk = pytest.importorskip("sklearn.linear_model")
    X, y = _small_c1_like(seed=43, n=40, p=60)
    n = X.shape[0]
    lam = 0.2 * np.abs(X.T @ y).max()
    r = orc.enet_path(X, y, 0.6, lambdas=[lam / 0.6 * 5, lam], eps_rel=1e-15, K=10_000_000)
    m = sk.ElasticNet(alpha=lam / n, l1_ratio=0.6, fit_intercept=False, tol=1e-14,
                      max_iter=1_000_000).fit(X, y)
    np.testing.assert_allclose(r["beta"][1], m.coef_, rtol=1e-6, atol=1e-8)


# ---- restricted solve of the learned start ---------------------------------

def test_restricted_solve_orthonormal_closed_form():
    """With orthonormal columns the system is diagonal: b_j = x_j^T y -
    lambda sigma_j (the soft-threshold value on the active side)."""
    import oracle
    rng = np.random.default_rng(41)
    Q, _ = np.linalg.qr(rng.standard_normal((40, 12)))
    y = rng.standard_normal(40)
    W = np.array([0, 3, 4, 9, 11])
    sg = np.array([1.0, -1.0, 1.0, 1.0, -1.0])
    b = oracle.restricted_solve(Q, y, W, sg, 0.3)
    np.testing.assert_allclose(b, Q[:, W].T @ y - 0.3 * sg, rtol=0, atol=1e-13)


def test_restricted_solve_minimizes_smooth_objective():
    """b minimizes 1/2 ||y - X_W b||^2 + lambda sigma^T b (a smooth convex
    function), found here by an independent minimizer (BFGS)."""
    import oracle
    from scipy.optimize import minimize
    rng = np.random.default_rng(42)
    X = rng.standard_normal((30, 20))
    y = rng.standard_normal(30)
    W = np.array([1, 2, 5, 7, 8, 13, 19])
    sg = np.sign(rng.standard_normal(len(W)))
    lam = 0.7
    f = lambda b: 0.5 * np.sum((y - X[:, W] @ b) ** 2) + lam * sg @ b
    g = lambda b: -X[:, W].T @ (y - X[:, W] @ b) + lam * sg
    ref = minimize(f, np.zeros(len(W)), jac=g, method="BFGS", options={"gtol": 1e-12}).x
    np.testing.assert_allclose(oracle.restricted_solve(X, y, W, sg, lam), ref, rtol=1e-7, atol=1e-9)


def test_restricted_solve_on_the_support_is_the_lasso_solution():
    """With W the support of a tight Lasso solution and sigma its signs, b is
    that solution on W (the oracle path's beta, gap <= 1e-13 ||y||^2)."""
    import oracle
    orc = oracle.oracle()
    rng = np.random.default_rng(43)
    n, p = 60, 150
    X = rng.standard_normal((n, p))
    beta = np.zeros(p)
    beta[rng.choice(p, 8, replace=False)] = rng.standard_normal(8) * 2
    y = X @ beta + 0.1 * rng.standard_normal(n)
    lam_max = np.abs(X.T @ y).max()
    r = orc.lasso_path(X, y, lambdas=[0.05 * lam_max], eps_rel=1e-13)
    bh = r["beta"][-1]
    W = np.nonzero(bh)[0]
    b = oracle.restricted_solve(X, y, W, np.sign(bh[W]), 0.05 * lam_max)
    np.testing.assert_allclose(b, bh[W], rtol=1e-6, atol=1e-9)
