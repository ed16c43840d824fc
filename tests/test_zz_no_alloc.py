"""The allocation-free entry point screen_noalloc (static device scratch, no
workspace) against screen() with a workspace: the same kernels on the same
inputs, so every output is equal bit for bit.  Two calls in a row, the
second with a smaller input, so stale contents of the static scratch from
the first call must not leak into the second."""
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
    gs.load_library()
    return torch


def _case(torch, n, p, dt, seed, with_active):
    d = synth.gaussian(seed, n, p, k=8, sigma=0.3)
    X, y = d["X"].astype(dt), d["y"].astype(dt)
    Xd = gs.colmajor_to_device(X)
    yd = torch.from_numpy(np.ascontiguousarray(y)).cuda()
    rng = np.random.default_rng(seed)
    beta = np.zeros(p)
    beta[rng.choice(p, 6, replace=False)] = 0.05 * rng.standard_normal(6)
    bd = torch.from_numpy(beta).cuda()
    lam = 0.3 * float(np.abs(X.astype(np.float64).T @ y.astype(np.float64)).max())
    act = None
    if with_active:
        a = np.sort(rng.choice(p, p // 2, replace=False)).astype(np.int32)
        act = torch.from_numpy(np.union1d(a, np.flatnonzero(beta)).astype(np.int32)).cuda()
    return Xd, yd, bd, lam, act


def _same(torch, a, b):
    q = int(a["q"].cpu()[0])
    assert q == int(b["q"].cpu()[0])
    assert np.array_equal(a["active"].cpu().numpy()[:q], b["active"].cpu().numpy()[:q])
    for k in ("gap", "alpha", "radius", "c"):
        assert np.array_equal(a[k].cpu().numpy(), b[k].cpu().numpy()), k
    return q


def test_noalloc_matches_screen_twice(torch):
    cases = [(1000, 60000, np.float32, 5, False),   # the larger input first
             (203, 3000, np.float32, 6, True),      # then a smaller one
             (50, 500, np.float64, 7, False)]
    for n, p, dt, seed, wa in cases:
        Xd, yd, bd, lam, act = _case(torch, n, p, dt, seed, wa)
        ref = gs.screen(Xd, yd, bd, lam, act)
        got = gs.screen_noalloc(Xd, yd, bd, lam, act)
        torch.cuda.synchronize()
        q = _same(torch, got, ref)
        assert 0 < q <= (p if act is None else act.numel())


def test_noalloc_loop_reuses_outputs(torch):
    """A loop of calls that allocates nothing: outputs preallocated once,
    every call equal to screen() at its own lambda."""
    Xd, yd, bd, lam, act = _case(torch, 500, 8000, np.float32, 9, False)
    out = None
    for f in (1.0, 0.5, 0.8):
        got = gs.screen_noalloc(Xd, yd, bd, f * lam, out=out)
        out = got
        ref = gs.screen(Xd, yd, bd, f * lam)
        torch.cuda.synchronize()
        _same(torch, got, ref)


def test_noalloc_too_large_is_rejected(torch):
    Xd, yd, bd, lam, _ = _case(torch, 8, 600_000, np.float32, 10, False)
    with pytest.raises(gs.GsError) as e:
        gs.screen_noalloc(Xd, yd, bd, lam)
    assert e.value.code == gs.GS_ETOOLARGE
