"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/gapsafe.h declares, and rejects bad arguments before
launching anything."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1505_03410_amd as gs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    txt = open(os.path.join(ROOT, "include", "gapsafe.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w[\w\s\*]*?\b(\w+)\s*\(", txt, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "sizeof")))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(gs.LIB_PATH):
        pytest.fail("libgapsafe.so is not built: run __graft_entry__.build()")
    return gs.load_library()


def test_exports_every_declared_symbol(lib):
    declared = _declared_functions()
    assert set(declared) == set(gs.EXPORTS), declared
    for name in declared:
        assert hasattr(lib, name), name


def test_struct_layout_matches_header():
    # offsets implied by natural alignment of the C structs
    assert ctypes.sizeof(gs.gs_problem) == 160
    assert gs.gs_problem.format.offset == 136 and gs.gs_problem.row_idx.offset == 152
    assert gs.gs_problem.lambda_min_ratio.offset == 72
    assert gs.gs_problem.lambda_out.offset == 128
    assert ctypes.sizeof(gs.gs_opts) == 64
    assert gs.gs_opts.rule.offset == 48
    assert gs.gs_opts.enet_alpha.offset == 56


def test_defaults(lib):
    o = gs.gs_opts()
    lib.gs_opts_default(ctypes.byref(o))
    assert o.eps_rel == 1e-8 and o.screen_every == 10 and o.max_epochs == 100000
    assert o.schedule == 0 and not o.select_counts and not o.timestamps


def _prob(**kw):
    pr = gs.gs_problem()
    pr.n, pr.p, pr.ldx, pr.dtype, pr.T = 8, 20, 8, gs.GS_F32, 3
    fake = 4096
    pr.X = pr.y = pr.beta_out = pr.gap_out = fake
    pr.epochs_out = pr.nactive_out = pr.status_out = fake
    pr.lambda_min_ratio = 0.01
    for k, v in kw.items():
        setattr(pr, k, v)
    return pr


@pytest.mark.parametrize("bad", [
    dict(n=0), dict(p=0), dict(T=0), dict(ldx=4), dict(dtype=7), dict(X=None),
    dict(gap_out=None), dict(lambda_min_ratio=0.0), dict(lambda_min_ratio=2.0),
    dict(lambda_min_ratio=float("nan")),
])
def test_invalid_problem_rejected(lib, bad):
    pr = _prob(**bad)
    o = gs.gs_opts()
    lib.gs_opts_default(ctypes.byref(o))
    assert lib.lasso_workspace_size(ctypes.byref(pr), 1, ctypes.byref(o)) == 0
    rc = lib.lasso_path(ctypes.byref(pr), ctypes.byref(o), ctypes.c_void_p(4096), 1 << 30, None)
    assert rc == gs.GS_EINVAL


def test_invalid_lambdas_rejected(lib):
    o = gs.gs_opts()
    lib.gs_opts_default(ctypes.byref(o))
    for vals in ([1.0, 2.0, 0.5], [1.0, -1.0, -2.0], [1.0, float("inf"), 0.1]):
        lam = np.array(vals)
        pr = _prob(lambdas=lam.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        rc = lib.lasso_path(ctypes.byref(pr), ctypes.byref(o), ctypes.c_void_p(4096), 1 << 30, None)
        assert rc == gs.GS_EINVAL, vals


@pytest.mark.parametrize("field,val", [("eps_rel", 0.0), ("eps_rel", float("nan")),
                                       ("screen_every", 0), ("max_epochs", -1), ("schedule", 9)])
def test_invalid_opts_rejected(lib, field, val):
    pr = _prob()
    o = gs.gs_opts()
    lib.gs_opts_default(ctypes.byref(o))
    setattr(o, field, val)
    rc = lib.lasso_path(ctypes.byref(pr), ctypes.byref(o), ctypes.c_void_p(4096), 1 << 30, None)
    assert rc == gs.GS_EINVAL


def test_workspace_checks(lib):
    pr = _prob()
    o = gs.gs_opts()
    lib.gs_opts_default(ctypes.byref(o))
    need = lib.lasso_workspace_size(ctypes.byref(pr), 1, ctypes.byref(o))
    assert need > 0 and need % 256 == 0
    assert lib.lasso_path(ctypes.byref(pr), ctypes.byref(o), None, need, None) == gs.GS_EWORKSPACE
    assert lib.lasso_path(ctypes.byref(pr), ctypes.byref(o), ctypes.c_void_p(4096), need - 1,
                          None) == gs.GS_EWORKSPACE
    # bigger problems need more
    pr2 = _prob(p=4000, T=100)
    assert lib.lasso_workspace_size(ctypes.byref(pr2), 1, ctypes.byref(o)) > need
    assert lib.screen_workspace_size(8, 20) > 0
    assert lib.screen_workspace_size(0, 20) == 0


def test_unsupported_n(lib):
    pr = _prob(n=5000, ldx=5000)
    o = gs.gs_opts()
    lib.gs_opts_default(ctypes.byref(o))
    rc = lib.lasso_path(ctypes.byref(pr), ctypes.byref(o), ctypes.c_void_p(4096), 1 << 30, None)
    assert rc == gs.GS_EUNSUPPORTED


def test_screen_invalid(lib):
    vp = ctypes.c_void_p(4096)
    args = [8, 20, 8, gs.GS_F32, vp, vp, vp, 0.5, 0, None, 0, vp, vp, vp, vp, vp, None, vp, 1 << 30,
            None]
    for idx, val in [(0, 0), (2, 4), (3, 5), (7, 0.0), (7, float("inf")), (4, None), (8, 5),
                     (8, -1)]:
        a = list(args)
        a[idx] = val
        assert lib.screen(*a) == gs.GS_EINVAL, (idx, val)
    # the comparison rules run on the wide schedule of lasso_path only
    for rule in (2, 3, 4):
        a = list(args)
        a[8] = rule
        assert lib.screen(*a) == gs.GS_EUNSUPPORTED


def test_screen_noalloc_rejects_before_launch(lib):
    """The allocation-free screen() checks its arguments and the size of its
    static scratch on the host, before touching the device: bad arguments
    give GS_EINVAL, a pass larger than GS_NOALLOC_SCRATCH_BYTES gives
    GS_ETOOLARGE (fake device pointers are never dereferenced)."""
    vp = ctypes.c_void_p(4096)
    args = [8, 20, 8, gs.GS_F32, vp, vp, vp, 0.5, 0, None, 0, vp, vp, vp, vp, vp, None, None]
    for idx, val in [(0, 0), (2, 4), (3, 5), (7, 0.0), (7, float("nan")), (4, None), (8, 7)]:
        a = list(args)
        a[idx] = val
        assert lib.screen_noalloc(*a) == gs.GS_EINVAL, (idx, val)
    big = list(args)
    big[1] = 1_000_000
    assert lib.screen_workspace_size(8, 1_000_000) > gs.NOALLOC_SCRATCH_BYTES
    assert lib.screen_noalloc(*big) == gs.GS_ETOOLARGE
    assert "static scratch" in gs.strerror(gs.GS_ETOOLARGE)
    # the largest p that fits at n = 2048 is about 347,000
    assert lib.screen_workspace_size(2048, 340_000) <= gs.NOALLOC_SCRATCH_BYTES
    assert lib.screen_workspace_size(2048, 360_000) > gs.NOALLOC_SCRATCH_BYTES


def test_strerror(lib):
    for c in (0, 1, -1, -2, -3, -4, -5, 99):
        assert isinstance(gs.strerror(c), str) and gs.strerror(c)


def test_plan_and_tuner_argument_checks(lib, tmp_path):
    o = gs.gs_opts()
    lib.gs_opts_default(ctypes.byref(o))
    pr = _prob()
    h = ctypes.c_void_p()
    assert lib.lasso_batch_plan(ctypes.byref(pr), 0, ctypes.byref(o), ctypes.c_void_p(4096),
                                1 << 30, None, ctypes.byref(h)) == gs.GS_EINVAL
    assert lib.lasso_batch_plan(ctypes.byref(pr), 1, ctypes.byref(o), ctypes.c_void_p(4096),
                                1 << 30, None, None) == gs.GS_EINVAL
    assert lib.lasso_batch_run(None, None) == gs.GS_EINVAL
    lib.lasso_batch_plan_free(None)
    ch = (ctypes.c_int32 * 2)()
    assert lib.gs_autotune(ctypes.byref(pr), 0, ctypes.byref(o), ctypes.c_void_p(4096), 1 << 30,
                           None, 3, 2, ch) == gs.GS_EINVAL
    assert lib.gs_autotune(ctypes.byref(pr), 1, ctypes.byref(o), ctypes.c_void_p(4096), 1 << 30,
                           None, 0, 2, ch) == gs.GS_EINVAL
    assert lib.gs_autotune(ctypes.byref(pr), 1, ctypes.byref(o), None, 0, None, 3, 2,
                           ch) == gs.GS_EWORKSPACE
    lib.gs_tune_reset()
    path = str(tmp_path / "tiles.json")
    assert lib.gs_tune_save(path.encode()) == gs.GS_OK
    import json
    thr0 = 16.0 * 1024 * 1024
    assert json.load(open(path)) == {"tiles": [], "schedule": [
        {"sched_dtype": 0, "wide_threshold": thr0}, {"sched_dtype": 1, "wide_threshold": thr0}]}
    with open(path, "w") as f:
        f.write('{"tiles": []}\n')
    assert lib.gs_tune_load(path.encode()) == gs.GS_EINVAL  # no entry
    assert lib.gs_tune_load(str(tmp_path / "missing.json").encode()) == gs.GS_EINVAL
    # schedule thresholds: defaults, a loaded value, reset
    assert lib.gs_wide_threshold(0) == thr0 and lib.gs_wide_threshold(1) == thr0
    assert lib.gs_wide_threshold(7) == -1.0
    with open(path, "w") as f:
        f.write('{"tiles": [], "schedule": [\n  {"sched_dtype": 1, "wide_threshold": 2500000}\n]}\n')
    assert lib.gs_tune_load(path.encode()) == gs.GS_OK
    assert lib.gs_wide_threshold(1) == 2500000.0 and lib.gs_wide_threshold(0) == thr0
    lib.gs_tune_reset()
    assert lib.gs_wide_threshold(1) == thr0
    # the schedule autotuner's argument checks (before any launch)
    c1 = ctypes.c_int32(-1)
    assert lib.gs_autotune_schedule(None, ctypes.byref(o), ctypes.c_void_p(4096), 1 << 30, None,
                                    3, ctypes.byref(c1)) == gs.GS_EINVAL
    assert lib.gs_autotune_schedule(ctypes.byref(pr), ctypes.byref(o), ctypes.c_void_p(4096),
                                    1 << 30, None, 0, ctypes.byref(c1)) == gs.GS_EINVAL
    assert lib.gs_autotune_schedule(ctypes.byref(pr), ctypes.byref(o), None, 0, None, 3,
                                    ctypes.byref(c1)) == gs.GS_EWORKSPACE
    rows = _prob(rows=4096)
    assert lib.gs_autotune_schedule(ctypes.byref(rows), ctypes.byref(o), ctypes.c_void_p(4096),
                                    1 << 30, None, 3, ctypes.byref(c1)) == gs.GS_EUNSUPPORTED
    # a valid entry (dtype 0, 16-byte loads, S=4 NG=5 -> S=16 NG=3) loads and saves back
    with open(path, "w") as f:
        f.write('{"tiles": [\n  {"dtype": 0, "vec": 4, "gather": 0, "S": 4, "NG": 5, '
                '"to_S": 16, "to_NG": 3}\n]}\n')
    assert lib.gs_tune_load(path.encode()) == gs.GS_OK
    out = str(tmp_path / "back.json")
    assert lib.gs_tune_save(out.encode()) == gs.GS_OK
    t = json.load(open(out))["tiles"]
    assert t == [{"dtype": 0, "vec": 4, "gather": 0, "S": 4, "NG": 5, "to_S": 16, "to_NG": 3}]
    lib.gs_tune_reset()


def test_learned_warm_start_argument_checks(lib):
    """The learned-warm-start entry points reject bad arguments before any
    launch (fake device pointers are never dereferenced)."""
    fake = ctypes.c_void_p(4096)
    assert lib.gs_block_corr(8, 20, 8, gs.GS_F32, fake, 0, fake, None) == gs.GS_EINVAL
    assert lib.gs_block_corr(8, 20, 8, gs.GS_F32, fake, 65, fake, None) == gs.GS_EINVAL
    assert lib.gs_block_corr(8, 20, 4, gs.GS_F32, fake, 50, fake, None) == gs.GS_EINVAL
    assert lib.gs_block_corr(8, 20, 8, 7, fake, 50, fake, None) == gs.GS_EINVAL
    assert lib.gs_mlp_forward(fake, fake, -1, fake, None) == gs.GS_EINVAL
    assert lib.gs_mlp_forward(None, fake, 5, fake, None) == gs.GS_EINVAL
    assert lib.gs_mlp_forward(None, None, 0, None, None) == gs.GS_OK  # nothing to do
    assert lib.gs_mlp_train_workspace_size(0) == 0
    # one partial gradient + loss per 64 rows, 256-byte aligned
    assert lib.gs_mlp_train_workspace_size(64) == (4611 * 4 + 255) // 256 * 256
    assert lib.gs_mlp_train_workspace_size(65) == (2 * 4611 * 4 + 255) // 256 * 256
    assert lib.gs_mlp_grad(fake, fake, fake, 64, fake, fake, None, 0, None) == gs.GS_EWORKSPACE
    assert lib.gs_mlp_grad(fake, fake, fake, 64, fake, fake, fake, 100, None) == gs.GS_EWORKSPACE
    assert lib.gs_mlp_grad(fake, fake, None, 64, fake, fake, fake, 1 << 20, None) == gs.GS_EINVAL
    assert lib.gs_mlp_adam(fake, fake, fake, fake, 0, 1e-3, None) == gs.GS_EINVAL
    assert lib.gs_mlp_adam(fake, fake, fake, fake, 1, float("nan"), None) == gs.GS_EINVAL
    assert lib.gs_mlp_train_step(fake, fake, fake, 0, 1e-3, fake, fake, 64, None, fake,
                                 1 << 20, None) == gs.GS_EINVAL
    assert lib.gs_warm_features(10, fake, fake, fake, fake, 0.0, 1.0, 1.0, fake,
                                None) == gs.GS_EINVAL
    assert lib.gs_warm_features(10, fake, fake, fake, fake, 1.0, 1.0, float("inf"), fake,
                                None) == gs.GS_EINVAL
    o = gs.gs_opts()
    lib.gs_opts_default(ctypes.byref(o))
    pr = _prob()
    need = lib.lasso_path_learned_workspace_size(ctypes.byref(pr))
    assert need >= lib.lasso_workspace_size(ctypes.byref(pr), 1, ctypes.byref(o))
    assert lib.lasso_path_learned_workspace_size(None) == 0
    rows = _prob(rows=4096)
    assert lib.lasso_path_learned_workspace_size(ctypes.byref(rows)) == 0
    assert lib.lasso_path_learned(ctypes.byref(rows), ctypes.byref(o), fake, 50, None, fake,
                                  need, None) == gs.GS_EINVAL
    assert lib.lasso_path_learned(ctypes.byref(pr), ctypes.byref(o), fake, 0, None, fake,
                                  need, None) == gs.GS_EINVAL
    assert lib.lasso_path_learned(ctypes.byref(pr), ctypes.byref(o), fake, 50, None, fake,
                                  need - 1, None) == gs.GS_EWORKSPACE
    big = _prob(n=4096, ldx=4096)
    assert lib.lasso_path_learned(ctypes.byref(big), ctypes.byref(o), fake, 50, None, fake,
                                  1 << 40, None) == gs.GS_EUNSUPPORTED


def test_restricted_solve_workspace_size(lib):
    """The restricted solve's workspace: 0 outside 1 <= m <= GS_WS_MAX, at
    least the 8 M (M + 64) bytes of the matrix and its right-hand-side tile
    row (M = m rounded up to 64), at most 15 MB more (the row-split partial
    Gram sums), and never smaller for a
    larger m -- the learned driver sizes one workspace for its largest
    working set and runs every smaller solve in it."""
    hdr = open(os.path.join(ROOT, "include", "gapsafe.h")).read()
    for name in ("GS_WS_ROUNDS", "GS_WS_ADD", "GS_WS_DROPS", "GS_WS_MAX"):
        assert re.search(r"\b%s = (\d+)" % name, hdr).group(1) == str(getattr(gs, name)), name
    assert lib.gs_restricted_solve_workspace_size(0) == 0
    assert lib.gs_restricted_solve_workspace_size(gs.GS_WS_MAX + 1) == 0
    prev = 0
    for m in range(1, gs.GS_WS_MAX + 1):
        need = lib.gs_restricted_solve_workspace_size(m)
        M = (m + 63) // 64 * 64
        assert 8 * M * (M + 64) <= need <= 8 * M * (M + 64) + 15_000_000 + 256, m
        assert need >= prev, m
        prev = need
