"""Python binding of libgapsafe.so, the gfx950 library for the Lasso solved by
cyclic coordinate descent with dynamic GAP SAFE sphere screening
(Fercoq, Gramfort & Salmon, ICML 2015).

The functions here have the names of the C ABI (include/gapsafe.h) and only
marshal arguments: torch tensors supply device memory and the current stream,
every step of the method runs in the library's HIP kernels.  There is no CPU
fallback: importing works without a GPU, calling needs the built library and
a device.

Design matrices are column-major: pass an (n, p) tensor whose strides are
(1, ldx), e.g. ``colmajor_to_device(X)`` or ``Xcm.T[:n]`` for a (p, ldx)
row-major buffer ``Xcm``.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgapsafe.so")

GS_F32, GS_F64 = 0, 1
GS_OK, GS_NOT_CONVERGED = 0, 1
GS_EINVAL, GS_EHIP, GS_EWORKSPACE, GS_EUNSUPPORTED, GS_ETOOLARGE = -1, -2, -3, -4, -5
# the learned start's working-set limits (header enum)
GS_WS_ROUNDS, GS_WS_ADD, GS_WS_DROPS, GS_WS_MAX = 4, 32, 4, 2047
NOALLOC_SCRATCH_BYTES = 16 << 20  # GS_NOALLOC_SCRATCH_BYTES
SCHEDULES = {"auto": 0, "narrow": 1, "wide": 2}
CD_MODES = {"auto": 0, "residual": 1}
RULES = {"sphere": 0, "dome": 1, "static": 2, "dynamic_safe": 3, "st3": 4}


class GsError(RuntimeError):
    def __init__(self, code, text):
        super().__init__(f"gapsafe error {code}: {text}")
        self.code = code


class gs_problem(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32), ("p", ctypes.c_int32), ("ldx", ctypes.c_int64),
        ("dtype", ctypes.c_int32), ("X", ctypes.c_void_p), ("y", ctypes.c_void_p),
        ("rows", ctypes.c_void_p), ("T", ctypes.c_int32),
        ("lambdas", ctypes.POINTER(ctypes.c_double)),
        ("lambda_relative", ctypes.c_int32), ("lambda_min_ratio", ctypes.c_double),
        ("beta_init", ctypes.c_void_p), ("beta_out", ctypes.c_void_p),
        ("gap_out", ctypes.c_void_p), ("epochs_out", ctypes.c_void_p),
        ("nactive_out", ctypes.c_void_p), ("status_out", ctypes.c_void_p),
        ("lambda_out", ctypes.c_void_p), ("format", ctypes.c_int32),
        ("col_ptr", ctypes.c_void_p), ("row_idx", ctypes.c_void_p),
    ]


class gs_opts(ctypes.Structure):
    _fields_ = [
        ("eps_rel", ctypes.c_double), ("screen_every", ctypes.c_int32),
        ("max_epochs", ctypes.c_int32), ("schedule", ctypes.c_int32),
        ("cd_mode", ctypes.c_int32),
        ("select_counts", ctypes.c_void_p), ("timestamps", ctypes.c_void_p),
        ("stats", ctypes.c_void_p), ("rule", ctypes.c_int32),
        ("enet_alpha", ctypes.c_double),
    ]


# Names of the GS_NSTATS counters of gs_opts.stats, in index order.
STAT_NAMES = ["pattern_epochs", "residual_epochs", "rejected", "builds", "setups",
              "support_changes", "passes", "skipped", "exact_checks", "near_checks",
              "wide_visits", "wide_rounds", "wide_stops"]

EXPORTS = ["gs_opts_default", "gs_wallclock_hz", "lasso_workspace_size", "lasso_path",
           "lasso_solve_batch", "lasso_batch_plan", "lasso_batch_run", "lasso_batch_plan_free",
           "gs_autotune", "gs_tune_save", "gs_tune_load", "gs_tune_reset",
           "screen_workspace_size", "screen", "screen_noalloc", "gs_timing_enable",
           "gs_timing_reset", "gs_timing_query", "lasso_strerror",
           "gs_block_corr", "gs_mlp_forward", "gs_mlp_train_workspace_size", "gs_mlp_grad",
           "gs_mlp_adam", "gs_mlp_train_step", "gs_warm_features",
           "lasso_path_learned_workspace_size", "lasso_path_learned",
           "gs_restricted_solve_workspace_size", "gs_restricted_solve",
           "gs_autotune_schedule", "gs_wide_threshold"]

MLP_PARAMS = 4610
# offsets of the parameter array (include/gapsafe.h): name -> (offset, shape)
MLP_LAYOUT = {"W1": (0, (64, 4)), "b1": (256, (64,)), "W2": (320, (64, 64)),
              "b2": (4416, (64,)), "W3": (4480, (2, 64)), "b3": (4608, (2,))}

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libgapsafe.so and declare its C ABI.  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with "
                          "`python -c 'import __graft_entry__ as g; g.build()'`")
    lib = ctypes.CDLL(path)
    P, vp = ctypes.POINTER, ctypes.c_void_p
    lib.gs_opts_default.argtypes = [P(gs_opts)]
    lib.gs_opts_default.restype = None
    lib.gs_wallclock_hz.argtypes = []
    lib.gs_wallclock_hz.restype = ctypes.c_double
    lib.lasso_workspace_size.argtypes = [P(gs_problem), ctypes.c_int32, P(gs_opts)]
    lib.lasso_workspace_size.restype = ctypes.c_size_t
    lib.lasso_path.argtypes = [P(gs_problem), P(gs_opts), vp, ctypes.c_size_t, vp]
    lib.lasso_path.restype = ctypes.c_int
    lib.lasso_solve_batch.argtypes = [P(gs_problem), ctypes.c_int32, P(gs_opts), vp,
                                      ctypes.c_size_t, vp]
    lib.lasso_solve_batch.restype = ctypes.c_int
    lib.lasso_batch_plan.argtypes = [P(gs_problem), ctypes.c_int32, P(gs_opts), vp,
                                     ctypes.c_size_t, vp, P(vp)]
    lib.lasso_batch_plan.restype = ctypes.c_int
    lib.lasso_batch_run.argtypes = [vp, vp]
    lib.lasso_batch_run.restype = ctypes.c_int
    lib.lasso_batch_plan_free.argtypes = [vp]
    lib.lasso_batch_plan_free.restype = None
    lib.gs_autotune.argtypes = [P(gs_problem), ctypes.c_int32, P(gs_opts), vp, ctypes.c_size_t,
                                vp, ctypes.c_int32, ctypes.c_int32, P(ctypes.c_int32)]
    lib.gs_autotune.restype = ctypes.c_int
    lib.gs_tune_save.argtypes = [ctypes.c_char_p]
    lib.gs_tune_save.restype = ctypes.c_int
    lib.gs_tune_load.argtypes = [ctypes.c_char_p]
    lib.gs_tune_load.restype = ctypes.c_int
    lib.gs_tune_reset.argtypes = []
    lib.gs_tune_reset.restype = None
    lib.screen_workspace_size.argtypes = [ctypes.c_int32, ctypes.c_int32]
    lib.screen_workspace_size.restype = ctypes.c_size_t
    lib.screen.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32,
                           vp, vp, vp, ctypes.c_double, ctypes.c_int32, vp, ctypes.c_int32,
                           vp, vp, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
    lib.screen.restype = ctypes.c_int
    lib.screen_noalloc.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                   ctypes.c_int32, vp, vp, vp, ctypes.c_double, ctypes.c_int32,
                                   vp, ctypes.c_int32, vp, vp, vp, vp, vp, vp, vp]
    lib.screen_noalloc.restype = ctypes.c_int
    lib.gs_timing_enable.argtypes = [ctypes.c_int]
    lib.gs_timing_enable.restype = None
    lib.gs_timing_reset.argtypes = []
    lib.gs_timing_reset.restype = None
    lib.gs_timing_query.argtypes = [ctypes.c_char_p, P(ctypes.c_double), P(ctypes.c_int64)]
    lib.gs_timing_query.restype = ctypes.c_int
    lib.lasso_strerror.argtypes = [ctypes.c_int]
    lib.lasso_strerror.restype = ctypes.c_char_p
    i32, i64, sz, f32, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t, ctypes.c_float, ctypes.c_double
    lib.gs_block_corr.argtypes = [i32, i32, i64, i32, vp, i32, vp, vp]
    lib.gs_block_corr.restype = ctypes.c_int
    lib.gs_mlp_forward.argtypes = [vp, vp, i32, vp, vp]
    lib.gs_mlp_forward.restype = ctypes.c_int
    lib.gs_mlp_train_workspace_size.argtypes = [i32]
    lib.gs_mlp_train_workspace_size.restype = sz
    lib.gs_mlp_grad.argtypes = [vp, vp, vp, i32, vp, vp, vp, sz, vp]
    lib.gs_mlp_grad.restype = ctypes.c_int
    lib.gs_mlp_adam.argtypes = [vp, vp, vp, vp, i32, f32, vp]
    lib.gs_mlp_adam.restype = ctypes.c_int
    lib.gs_mlp_train_step.argtypes = [vp, vp, vp, i32, f32, vp, vp, i32, vp, vp, sz, vp]
    lib.gs_mlp_train_step.restype = ctypes.c_int
    lib.gs_warm_features.argtypes = [i32, vp, vp, vp, vp, f64, f64, f64, vp, vp]
    lib.gs_warm_features.restype = ctypes.c_int
    lib.lasso_path_learned_workspace_size.argtypes = [P(gs_problem)]
    lib.lasso_path_learned_workspace_size.restype = sz
    lib.gs_autotune_schedule.argtypes = [P(gs_problem), P(gs_opts), vp, sz, vp, i32, P(i32)]
    lib.gs_autotune_schedule.restype = ctypes.c_int
    lib.gs_wide_threshold.argtypes = [i32]
    lib.gs_wide_threshold.restype = f64
    lib.gs_restricted_solve_workspace_size.argtypes = [i32]
    lib.gs_restricted_solve_workspace_size.restype = sz
    lib.gs_restricted_solve.argtypes = [i32, i32, ctypes.c_int64, i32, vp, vp, vp, vp, i32, f64,
                                        vp, vp, vp, sz, vp]
    lib.gs_restricted_solve.restype = ctypes.c_int
    lib.lasso_path_learned.argtypes = [P(gs_problem), P(gs_opts), vp, i32, vp, vp, sz, vp]
    lib.lasso_path_learned.restype = ctypes.c_int
    _lib = lib
    return lib


def strerror(code: int) -> str:
    return load_library().lasso_strerror(code).decode()


def _check(code: int, allow_not_converged: bool = True):
    if code == GS_OK or (allow_not_converged and code == GS_NOT_CONVERGED):
        return code
    raise GsError(code, strerror(code))


# ------------------------------------------------------------------ helpers

def _torch():
    import torch
    return torch


def _dtype_code(t):
    torch = _torch()
    if t.dtype == torch.float32:
        return GS_F32
    if t.dtype == torch.float64:
        return GS_F64
    raise TypeError(f"unsupported dtype {t.dtype}")


def _stream_ptr(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _active_ptr(active):
    """The active list's pointer: NULL means all p columns in the C ABI, so an
    empty list (whose tensor may have no storage) passes a non-null pointer
    with q_in = 0."""
    if active is None:
        return None, None
    if active.numel() == 0:
        keep = _torch().zeros(1, dtype=_torch().int32, device=active.device)
        return _ptr(keep), keep
    return _ptr(active), active


def colmajor_to_device(X, ld_multiple: int = 4, dtype=None, device="cuda"):
    """numpy (n, p) -> device (n, p) tensor with strides (1, ldx), ldx padded
    to a multiple of ``ld_multiple`` (padding rows are zero)."""
    torch = _torch()
    X = np.asarray(X)
    n, p = X.shape
    ld = ((n + ld_multiple - 1) // ld_multiple) * ld_multiple
    buf = np.zeros((p, ld), dtype=dtype or X.dtype)
    buf[:, :n] = X.T
    t = torch.from_numpy(buf).to(device)
    return t.T[:n]


GS_DENSE, GS_CSC = 0, 1


class CscDesign:
    """A sparse design in compressed sparse column form on the device:
    col_ptr (p+1 int64), row_idx (nnz int32) and values (nnz float32 or
    float64), n rows.  Pass it as X to lasso_path / lasso_solve_batch."""

    def __init__(self, col_ptr, row_idx, values, n):
        torch = _torch()
        if col_ptr.dtype != torch.int64 or row_idx.dtype != torch.int32:
            raise ValueError("col_ptr must be int64 and row_idx int32")
        for t in (col_ptr, row_idx, values):
            if not t.is_cuda or not t.is_contiguous():
                raise ValueError("CSC arrays must be contiguous device tensors")
        self.col_ptr, self.row_idx, self.values, self.n = col_ptr, row_idx, values, int(n)
        self.p = col_ptr.numel() - 1
        self.dtype = values.dtype
        self.device = values.device

    @classmethod
    def from_host(cls, col_ptr, row_idx, values, n, device="cuda"):
        torch = _torch()
        return cls(torch.from_numpy(np.ascontiguousarray(col_ptr, dtype=np.int64)).to(device),
                   torch.from_numpy(np.ascontiguousarray(row_idx, dtype=np.int32)).to(device),
                   torch.from_numpy(np.ascontiguousarray(values)).to(device), n)


def _design(X):
    if X.dim() != 2 or X.stride(0) != 1 or X.stride(1) < X.shape[0]:
        raise ValueError("X must be an (n, p) column-major tensor: strides (1, ldx), ldx >= n")
    if not X.is_cuda:
        raise ValueError("X must be a device tensor")
    return X.shape[0], X.shape[1], X.stride(1)


class PathResult(dict):
    """beta (T, p), gap (T,), epochs (T,), nactive (T,), status (T,), lambdas (T,)."""

    __getattr__ = dict.__getitem__


def _alloc_outputs(n, p, T, dt, device):
    torch = _torch()
    return PathResult(
        beta=torch.empty((T, p), dtype=torch.float64, device=device),
        gap=torch.empty(T, dtype=torch.float64, device=device),
        epochs=torch.empty(T, dtype=torch.int32, device=device),
        nactive=torch.empty(T, dtype=torch.int32, device=device),
        status=torch.empty(T, dtype=torch.int32, device=device),
        lambdas=torch.empty(T, dtype=torch.float64, device=device),
    )


def _problem(X, y, *, T, lambdas, relative, lambda_min_ratio, beta_init, rows, out, n=None):
    torch = _torch()
    csc = isinstance(X, CscDesign)
    ld = 1 if csc else X.stride(1)
    if csc:
        if rows is not None:
            raise ValueError("row subsamples are for dense designs")
        n, p = X.n, X.p
    elif rows is not None:
        if rows.dtype != torch.int32 or not rows.is_cuda or not rows.is_contiguous():
            raise ValueError("rows must be a contiguous int32 device tensor")
        n = rows.numel()
        p = X.shape[1]
    else:
        n, p, ld = _design(X)
    if y.dtype != X.dtype or not y.is_cuda or not y.is_contiguous():
        raise ValueError("y must be a contiguous device tensor of X's dtype")
    host_lam = None
    if lambdas is not None:
        host_lam = np.ascontiguousarray(np.asarray(lambdas, dtype=np.float64))
        T = len(host_lam)
    if beta_init is not None and (beta_init.dtype != torch.float64 or not beta_init.is_contiguous()
                                  or beta_init.numel() != p):
        raise ValueError("beta_init must be p contiguous float64 values")
    if out is None:
        out = _alloc_outputs(n, p, T, X.dtype, X.device)
    pr = gs_problem()
    pr.n, pr.p, pr.ldx = n, p, ld
    if csc:
        pr.dtype = _dtype_code(X.values)
        pr.X, pr.y = X.values.data_ptr(), y.data_ptr()
        pr.format, pr.col_ptr, pr.row_idx = GS_CSC, X.col_ptr.data_ptr(), X.row_idx.data_ptr()
    else:
        pr.dtype = _dtype_code(X)
        pr.X, pr.y = X.data_ptr(), y.data_ptr()
    pr.rows = None if rows is None else rows.data_ptr()
    pr.T = T
    pr.lambdas = None if host_lam is None else host_lam.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    pr.lambda_relative = 1 if relative else 0
    pr.lambda_min_ratio = float(lambda_min_ratio)
    pr.beta_init = None if beta_init is None else beta_init.data_ptr()
    pr.beta_out = out["beta"].data_ptr()
    pr.gap_out = out["gap"].data_ptr()
    pr.epochs_out = out["epochs"].data_ptr()
    pr.nactive_out = out["nactive"].data_ptr()
    pr.status_out = out["status"].data_ptr()
    pr.lambda_out = out["lambdas"].data_ptr()
    return pr, out, host_lam


def _opts(eps_rel, screen_every, max_epochs, schedule, select_counts=None, timestamps=None,
          cd_mode="auto", stats=None, rule="sphere", enet_alpha=1.0):
    o = gs_opts()
    load_library().gs_opts_default(ctypes.byref(o))
    o.rule = RULES[rule] if isinstance(rule, str) else int(rule)
    o.enet_alpha = float(enet_alpha)
    o.eps_rel = float(eps_rel)
    o.screen_every = int(screen_every)
    o.max_epochs = int(max_epochs)
    o.schedule = SCHEDULES[schedule] if isinstance(schedule, str) else int(schedule)
    o.cd_mode = CD_MODES[cd_mode] if isinstance(cd_mode, str) else int(cd_mode)
    o.select_counts = None if select_counts is None else select_counts.data_ptr()
    o.timestamps = None if timestamps is None else timestamps.data_ptr()
    if stats is not None:
        torch = _torch()
        if stats.dtype != torch.int64 or stats.numel() < len(STAT_NAMES) or not stats.is_contiguous():
            raise ValueError("stats must be a contiguous int64 tensor of %d counters" % len(STAT_NAMES))
        o.stats = stats.data_ptr()
    return o


def _workspace(nbytes, device):
    torch = _torch()
    if nbytes == 0:
        raise GsError(GS_EINVAL, "invalid arguments (workspace size query returned 0)")
    return torch.empty(int(nbytes), dtype=torch.uint8, device=device)


# --------------------------------------------------------------------- API

def lasso_path(X, y, *, T: int = 100, lambdas: Optional[Sequence[float]] = None,
               relative: bool = False, lambda_min_ratio: float = 1e-3, beta_init=None,
               rows=None, eps_rel: float = 1e-8, screen_every: int = 10,
               max_epochs: int = 100000, schedule="auto", cd_mode="auto", stream=None,
               out=None, workspace=None, stats=None, rule="sphere", enet_alpha=1.0):
    """Algorithm 1 on the device for one problem; see include/gapsafe.h.
    Returns a PathResult of device tensors (valid after the stream syncs) with
    an extra ``rc`` entry (GS_OK or GS_NOT_CONVERGED).  enet_alpha < 1 solves
    the elastic net through its augmented Lasso."""
    lib = load_library()
    pr, out, _keep = _problem(X, y, T=T, lambdas=lambdas, relative=relative,
                              lambda_min_ratio=lambda_min_ratio, beta_init=beta_init,
                              rows=rows, out=out)
    o = _opts(eps_rel, screen_every, max_epochs, schedule, cd_mode=cd_mode, stats=stats,
              rule=rule, enet_alpha=enet_alpha)
    need = lib.lasso_workspace_size(ctypes.byref(pr), 1, ctypes.byref(o))
    ws = workspace if workspace is not None and workspace.numel() >= need else _workspace(need, X.device)
    rc = lib.lasso_path(ctypes.byref(pr), ctypes.byref(o), _ptr(ws), ws.numel(), _stream_ptr(stream))
    _check(rc)
    out["rc"] = rc
    out["workspace"] = ws
    return out


def _batch_args(problems, eps_rel, screen_every, max_epochs, select_counts, timestamps,
                cd_mode, stats, workspace, rule="sphere"):
    lib = load_library()
    B = len(problems)
    arr = (gs_problem * B)()
    outs, keep = [], []
    for b, pb in enumerate(problems):
        pr, out, hl = _problem(pb["X"], pb["y"], T=pb.get("T", 100), lambdas=pb.get("lambdas"),
                               relative=pb.get("relative", False),
                               lambda_min_ratio=pb.get("lambda_min_ratio", 1e-3),
                               beta_init=pb.get("beta_init"), rows=pb.get("rows"),
                               out=pb.get("out"))
        arr[b] = pr
        outs.append(out)
        keep.append(hl)
    o = _opts(eps_rel, screen_every, max_epochs, "narrow", select_counts, timestamps, cd_mode,
              stats, rule)
    need = lib.lasso_workspace_size(arr, B, ctypes.byref(o))
    X0 = problems[0]["X"]
    dev = X0.device
    ws = workspace if workspace is not None and workspace.numel() >= need else _workspace(need, dev)
    for out in outs:
        out["workspace"] = ws
    return lib, arr, o, outs, keep, ws


def lasso_solve_batch(problems, *, eps_rel: float = 1e-8, screen_every: int = 10,
                      max_epochs: int = 100000, select_counts=None, timestamps=None,
                      cd_mode="auto", stream=None, workspace=None, stats=None, rule="sphere"):
    """Many paths in one persistent launch.  ``problems`` is a list of dicts
    with keys X, y and optionally T, lambdas, relative, lambda_min_ratio,
    beta_init, rows.  Returns the list of PathResults."""
    lib, arr, o, outs, _keep, ws = _batch_args(problems, eps_rel, screen_every, max_epochs,
                                               select_counts, timestamps, cd_mode, stats,
                                               workspace, rule)
    rc = lib.lasso_solve_batch(arr, len(problems), ctypes.byref(o), _ptr(ws), ws.numel(),
                               _stream_ptr(stream))
    _check(rc)
    return outs


class BatchPlan:
    """A batch captured into a HIP graph (lasso_batch_plan); ``run()`` replays
    it.  ``outputs`` are the per-problem result tensors every replay fills."""

    def __init__(self, problems, *, eps_rel=1e-8, screen_every=10, max_epochs=100000,
                 select_counts=None, timestamps=None, cd_mode="auto", stream=None,
                 workspace=None, stats=None):
        lib, arr, o, outs, keep, ws = _batch_args(problems, eps_rel, screen_every, max_epochs,
                                                  select_counts, timestamps, cd_mode, stats,
                                                  workspace)
        self._lib = lib
        self._keep = (arr, o, keep, problems, select_counts, timestamps, stats)
        self.outputs = outs
        self.workspace = ws
        h = ctypes.c_void_p()
        rc = lib.lasso_batch_plan(arr, len(problems), ctypes.byref(o), _ptr(ws), ws.numel(),
                                  _stream_ptr(stream), ctypes.byref(h))
        _check(rc, allow_not_converged=False)
        self._h = h

    def run(self, stream=None):
        rc = self._lib.lasso_batch_run(self._h, _stream_ptr(stream))
        _check(rc, allow_not_converged=False)
        return self.outputs

    def close(self):
        if getattr(self, "_h", None):
            self._lib.lasso_batch_plan_free(self._h)
            self._h = None

    def __del__(self):
        self.close()


def autotune(problems, *, max_lambdas: int = 5, sample: int = 4, eps_rel: float = 1e-8,
             screen_every: int = 10, max_epochs: int = 100000, cd_mode="auto", stream=None,
             workspace=None):
    """Runs the tile autotuner (gs_autotune) on the problem classes present in
    ``problems``; returns the chosen (S, NG) per problem.  The recorded choice
    applies to later calls in this process."""
    lib, arr, o, _outs, _keep, ws = _batch_args(problems, eps_rel, screen_every, max_epochs,
                                                None, None, cd_mode, None, workspace)
    B = len(problems)
    ch = (ctypes.c_int32 * (2 * B))()
    rc = lib.gs_autotune(arr, B, ctypes.byref(o), _ptr(ws), ws.numel(), _stream_ptr(stream),
                         int(max_lambdas), int(sample), ch)
    _check(rc, allow_not_converged=False)
    return [(ch[2 * b], ch[2 * b + 1]) for b in range(B)]


def autotune_schedule(X, y, *, T: int = 100, lambdas: Optional[Sequence[float]] = None,
                      relative: bool = False, lambda_min_ratio: float = 1e-3,
                      max_lambdas: int = 5, eps_rel: float = 1e-8, screen_every: int = 10,
                      max_epochs: int = 100000, cd_mode="auto", stream=None):
    """Times the narrow and the wide schedule on this problem's first
    ``max_lambdas`` lambdas and moves the dtype's auto-schedule threshold
    accordingly (gs_autotune_schedule); returns "wide" or "narrow", the faster."""
    lib = load_library()
    pr, _out, _keep = _problem(X, y, T=T, lambdas=lambdas, relative=relative,
                               lambda_min_ratio=lambda_min_ratio, beta_init=None, rows=None,
                               out=None)
    o = _opts(eps_rel, screen_every, max_epochs, "auto", cd_mode=cd_mode)
    need = lib.lasso_workspace_size(ctypes.byref(pr), 1, ctypes.byref(o))
    ws = _workspace(need, X.device)
    ch = ctypes.c_int32(-1)
    _check(lib.gs_autotune_schedule(ctypes.byref(pr), ctypes.byref(o), _ptr(ws), ws.numel(),
                                    _stream_ptr(stream), int(max_lambdas), ctypes.byref(ch)),
           allow_not_converged=False)
    return "wide" if ch.value == 1 else "narrow"


def wide_threshold(dtype="f32") -> float:
    """The n*p above which the auto schedule is wide, for FP32 ("f32") or
    FP64 ("f64") designs."""
    return float(load_library().gs_wide_threshold(0 if dtype == "f32" else 1))


def tune_save(path: str):
    _check(load_library().gs_tune_save(path.encode()), allow_not_converged=False)


def tune_load(path: str):
    _check(load_library().gs_tune_load(path.encode()), allow_not_converged=False)


def tune_reset():
    load_library().gs_tune_reset()


def screen(X, y, beta, lam: float, active=None, *, want_c: bool = True, stream=None,
           workspace=None, rule="sphere"):
    """One GAP SAFE screening pass at (beta, lam).  Returns device tensors:
    active (kept indices, ascending), q (1,), gap, alpha, radius (1,) and c."""
    torch = _torch()
    lib = load_library()
    n, p, ld = _design(X)
    dev = X.device
    if beta.dtype != torch.float64 or beta.numel() != p or not beta.is_contiguous():
        raise ValueError("beta must be p contiguous float64 values")
    if active is not None:
        if active.dtype != torch.int32 or not active.is_contiguous():
            raise ValueError("active must be a contiguous int32 tensor")
        q = active.numel()
    else:
        q = p
    act_out = torch.empty(max(q, 1), dtype=torch.int32, device=dev)
    q_out = torch.empty(1, dtype=torch.int32, device=dev)
    gap = torch.empty(1, dtype=torch.float64, device=dev)
    alpha = torch.empty(1, dtype=torch.float64, device=dev)
    radius = torch.empty(1, dtype=torch.float64, device=dev)
    c = torch.empty(max(q, 1), dtype=torch.float64, device=dev) if want_c else None
    need = lib.screen_workspace_size(n, p)
    ws = workspace if workspace is not None and workspace.numel() >= need else _workspace(need, dev)
    a_ptr, _a_keep = _active_ptr(active)
    rc = lib.screen(n, p, ld, _dtype_code(X), _ptr(X), _ptr(y), _ptr(beta), float(lam),
                    RULES[rule], a_ptr, q, _ptr(act_out), _ptr(q_out), _ptr(gap), _ptr(alpha),
                    _ptr(radius), _ptr(c), _ptr(ws), ws.numel(), _stream_ptr(stream))
    _check(rc, allow_not_converged=False)
    return dict(active=act_out, q=q_out, gap=gap, alpha=alpha, radius=radius,
                c=c if c is None else c[:q], workspace=ws)


def screen_noalloc(X, y, beta, lam: float, active=None, *, want_c: bool = True, stream=None,
                   out=None, rule="sphere"):
    """screen() through the allocation-free entry point: the library uses its
    static device scratch instead of a workspace.  ``out`` (optional) is a
    dict of preallocated output tensors as returned by a previous call, so a
    loop of calls allocates nothing at all."""
    torch = _torch()
    lib = load_library()
    n, p, ld = _design(X)
    dev = X.device
    if beta.dtype != torch.float64 or beta.numel() != p or not beta.is_contiguous():
        raise ValueError("beta must be p contiguous float64 values")
    if active is not None:
        if active.dtype != torch.int32 or not active.is_contiguous():
            raise ValueError("active must be a contiguous int32 tensor")
        q = active.numel()
    else:
        q = p
    if out is None:
        out = dict(active=torch.empty(max(q, 1), dtype=torch.int32, device=dev),
                   q=torch.empty(1, dtype=torch.int32, device=dev),
                   gap=torch.empty(1, dtype=torch.float64, device=dev),
                   alpha=torch.empty(1, dtype=torch.float64, device=dev),
                   radius=torch.empty(1, dtype=torch.float64, device=dev),
                   c=torch.empty(max(q, 1), dtype=torch.float64, device=dev) if want_c else None)
    elif out["active"].numel() < q or (out.get("c") is not None and out["c"].numel() < q):
        raise ValueError("preallocated outputs are smaller than the active set")
    a_ptr, _a_keep = _active_ptr(active)
    rc = lib.screen_noalloc(n, p, ld, _dtype_code(X), _ptr(X), _ptr(y), _ptr(beta), float(lam),
                            RULES[rule], a_ptr, q, _ptr(out["active"]), _ptr(out["q"]),
                            _ptr(out["gap"]), _ptr(out["alpha"]), _ptr(out["radius"]),
                            _ptr(out.get("c")), _stream_ptr(stream))
    _check(rc, allow_not_converged=False)
    res = dict(out)
    if res.get("c") is not None:
        res["c"] = res["c"][:q]
    return res


def timing_enable(on: bool = True):
    load_library().gs_timing_enable(1 if on else 0)


def timing_reset():
    load_library().gs_timing_reset()


def timing_query(kernel: str):
    """(total milliseconds, launches) of the named kernel since the reset."""
    tot = ctypes.c_double()
    cnt = ctypes.c_int64()
    if load_library().gs_timing_query(kernel.encode(), ctypes.byref(tot), ctypes.byref(cnt)) != 0:
        raise ValueError(f"unknown kernel name {kernel!r}")
    return tot.value, cnt.value


def wallclock_hz() -> float:
    return load_library().gs_wallclock_hz()


# ------------------------------------------------------- learned warm start

def _f32_dev(t, shape_last=None, name="tensor"):
    torch = _torch()
    if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float32 device tensor")
    if shape_last is not None and (t.dim() != 2 or t.shape[1] != shape_last):
        raise ValueError(f"{name} must have shape (m, {shape_last})")
    return t


def mlp_params_to_flat(params, device="cuda"):
    """dict W1, b1, W2, b2, W3, b3 (arrays) -> flat float32 device tensor."""
    torch = _torch()
    flat = np.zeros(MLP_PARAMS, dtype=np.float32)
    for k, (off, shp) in MLP_LAYOUT.items():
        a = np.asarray(params[k], dtype=np.float32)
        if a.shape != shp:
            raise ValueError(f"{k} must have shape {shp}")
        flat[off:off + a.size] = a.reshape(-1)
    return torch.from_numpy(flat).to(device)


def mlp_flat_to_params(flat):
    """flat parameter array (tensor or numpy) -> dict of float64 numpy arrays."""
    a = flat.detach().cpu().numpy() if hasattr(flat, "detach") else np.asarray(flat)
    return {k: a[off:off + int(np.prod(shp))].astype(np.float64).reshape(shp)
            for k, (off, shp) in MLP_LAYOUT.items()}


def block_corr(X, block: int = 50, stream=None):
    """Block max correlation of the columns of X (gs_block_corr): p floats."""
    torch = _torch()
    n, p, ld = _design(X)
    out = torch.empty(p, dtype=torch.float32, device=X.device)
    _check(load_library().gs_block_corr(n, p, ld, _dtype_code(X), _ptr(X), int(block), _ptr(out),
                                        _stream_ptr(stream)), allow_not_converged=False)
    return out


def mlp_forward(params, U, stream=None):
    """Network outputs (m, 2) for inputs U (m, 4) (gs_mlp_forward)."""
    torch = _torch()
    _f32_dev(params, name="params")
    _f32_dev(U, 4, "U")
    out = torch.empty((U.shape[0], 2), dtype=torch.float32, device=U.device)
    _check(load_library().gs_mlp_forward(_ptr(params), _ptr(U), U.shape[0], _ptr(out),
                                         _stream_ptr(stream)), allow_not_converged=False)
    return out


def _train_ws(m, workspace, device):
    need = load_library().gs_mlp_train_workspace_size(m)
    if workspace is not None and workspace.numel() >= need:
        return workspace
    return _workspace(need, device)


def mlp_grad(params, U, targets, stream=None, workspace=None):
    """(gradient (MLP_PARAMS,), loss (1,)) of the training loss (gs_mlp_grad)."""
    torch = _torch()
    _f32_dev(params, name="params")
    _f32_dev(U, 4, "U")
    _f32_dev(targets, 3, "targets")
    m = U.shape[0]
    if targets.shape[0] != m:
        raise ValueError("U and targets must have the same number of rows")
    g = torch.empty(MLP_PARAMS, dtype=torch.float32, device=U.device)
    loss = torch.empty(1, dtype=torch.float32, device=U.device)
    ws = _train_ws(m, workspace, U.device)
    _check(load_library().gs_mlp_grad(_ptr(params), _ptr(U), _ptr(targets), m, _ptr(g),
                                      _ptr(loss), _ptr(ws), ws.numel(), _stream_ptr(stream)),
           allow_not_converged=False)
    return g, loss


def mlp_adam(params, adam_m, adam_v, grad, t: int, lr: float, stream=None):
    """One Adam step in place (gs_mlp_adam)."""
    for a, nm in ((params, "params"), (adam_m, "adam_m"), (adam_v, "adam_v"), (grad, "grad")):
        _f32_dev(a, name=nm)
    _check(load_library().gs_mlp_adam(_ptr(params), _ptr(adam_m), _ptr(adam_v), _ptr(grad),
                                      int(t), float(lr), _stream_ptr(stream)),
           allow_not_converged=False)


def mlp_train_step(params, adam_m, adam_v, t: int, lr: float, U, targets, loss=None,
                   stream=None, workspace=None):
    """Forward, backward and one Adam step in place (gs_mlp_train_step)."""
    for a, nm in ((params, "params"), (adam_m, "adam_m"), (adam_v, "adam_v")):
        _f32_dev(a, name=nm)
    _f32_dev(U, 4, "U")
    _f32_dev(targets, 3, "targets")
    m = U.shape[0]
    ws = _train_ws(m, workspace, U.device)
    _check(load_library().gs_mlp_train_step(_ptr(params), _ptr(adam_m), _ptr(adam_v), int(t),
                                            float(lr), _ptr(U), _ptr(targets), m, _ptr(loss),
                                            _ptr(ws), ws.numel(), _stream_ptr(stream)),
           allow_not_converged=False)
    return ws


def warm_features(c, beta_prev, nrm2, bmc, lam, lam_max, ynorm, stream=None):
    """Network inputs (p, 4) at (beta_prev, lam) (gs_warm_features)."""
    torch = _torch()
    p = c.numel()
    for a, nm in ((c, "c"), (beta_prev, "beta_prev"), (nrm2, "nrm2")):
        if a.dtype != torch.float64 or not a.is_contiguous() or a.numel() != p:
            raise ValueError(f"{nm} must be p contiguous float64 values")
    _f32_dev(bmc, name="bmc")
    U = torch.empty((p, 4), dtype=torch.float32, device=c.device)
    _check(load_library().gs_warm_features(p, _ptr(c), _ptr(beta_prev), _ptr(nrm2), _ptr(bmc),
                                           float(lam), float(lam_max), float(ynorm), _ptr(U),
                                           _stream_ptr(stream)), allow_not_converged=False)
    return U


def restricted_solve(X, y, W, sigma, lam, stream=None):
    """b on the working set W (int32 column indices) with signs sigma
    (float64 +-1): (X_W^T X_W) b = X_W^T y - lam sigma (gs_restricted_solve).
    Returns (b, info) with info the device status (0 = solved)."""
    torch = _torch()
    n, p = X.shape
    m = W.numel()
    if W.dtype != torch.int32 or not W.is_cuda or not W.is_contiguous():
        raise ValueError("W must be a contiguous int32 device tensor")
    if sigma.dtype != torch.float64 or not sigma.is_contiguous() or sigma.numel() != m:
        raise ValueError("sigma must be m contiguous float64 values")
    if y.dtype != X.dtype or not y.is_contiguous():
        raise ValueError("y must be a contiguous device tensor of X's dtype")
    lib = load_library()
    need = lib.gs_restricted_solve_workspace_size(m)
    ws = torch.empty(max(int(need), 1), dtype=torch.uint8, device=X.device)
    b = torch.empty(m, dtype=torch.float64, device=X.device)
    info = torch.zeros(1, dtype=torch.int32, device=X.device)
    _check(lib.gs_restricted_solve(n, p, X.stride(1), _dtype_code(X), _ptr(X), _ptr(y), _ptr(W),
                                   _ptr(sigma), m, float(lam), _ptr(b), _ptr(info), _ptr(ws),
                                   ws.numel(), _stream_ptr(stream)), allow_not_converged=False)
    return b, info


def lasso_path_learned(X, y, params=None, *, block: int = 50, T: int = 100,
                       lambdas: Optional[Sequence[float]] = None, relative: bool = False,
                       lambda_min_ratio: float = 1e-3, beta_init=None, eps_rel: float = 1e-8,
                       screen_every: int = 10, max_epochs: int = 100000, schedule="auto",
                       cd_mode="auto", stream=None, out=None, workspace=None, stats=None):
    """A path whose warm starts come from the network ``params`` (flat
    float32 device tensor; None = plain starts, one lambda at a time); see
    lasso_path_learned in include/gapsafe.h.  Synchronizes the stream.  The
    result has the entries of lasso_path plus ``learned`` (T int32, 1 where
    the network's start was taken)."""
    torch = _torch()
    lib = load_library()
    pr, out, _keep = _problem(X, y, T=T, lambdas=lambdas, relative=relative,
                              lambda_min_ratio=lambda_min_ratio, beta_init=beta_init,
                              rows=None, out=out)
    if params is not None:
        _f32_dev(params, name="params")
        if params.numel() != MLP_PARAMS:
            raise ValueError(f"params must hold {MLP_PARAMS} values")
    o = _opts(eps_rel, screen_every, max_epochs, schedule, cd_mode=cd_mode, stats=stats)
    need = lib.lasso_path_learned_workspace_size(ctypes.byref(pr))
    ws = workspace if workspace is not None and workspace.numel() >= need else _workspace(need, X.device)
    learned = torch.empty(pr.T, dtype=torch.int32, device=X.device)
    rc = lib.lasso_path_learned(ctypes.byref(pr), ctypes.byref(o), _ptr(params), int(block),
                                _ptr(learned), _ptr(ws), ws.numel(), _stream_ptr(stream))
    _check(rc)
    out["rc"] = rc
    out["learned"] = learned
    out["workspace"] = ws
    return out
