"""ctypes binding of libabm (include/abm.h), argument marshalling only.

Device memory and streams come from PyTorch (tensors' data_ptr(), the current
stream's hipStream_t); every step of the method runs in libabm's kernels.  The
binding refuses to work without the built library: there is no fallback.
"""
from __future__ import annotations

import atexit
import ctypes
import sys
import weakref
import os
from typing import List, Optional, Sequence

from .inputs import Problem, RHS_DIM

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libabm.so")

ABM_OK, ABM_EINVAL, ABM_ENOMEM, ABM_EDEVICE, ABM_EAGAIN, ABM_ENOENT, ABM_ECANCELED = \
    0, -1, -2, -3, -4, -5, -6
RHS_ID = {"LINEAR": 0, "DUFFING": 1, "LORENZ": 2, "POLY": 3, "LCR": 4, "DIAG": 5}
PREC_ID = {"fp64": 0, "fp32": 1, "bf16x3": 2, "bf16x6": 3, "fp16x3": 4, "dd": 5, "i8x9": 6}

EXPORTED = ("abm_ctx_create", "abm_ctx_destroy", "abm_plan", "abm_plan_destroy", "abm_plan_check",
            "abm_plan_weights", "abm_plan_timing", "abm_plan_graph", "abm_solve", "abm_solve_batch", "abm_submit", "abm_poll", "abm_cancel",
            "abm_request_bytes", "abm_plan_tuned", "abm_plan_config", "abm_autotune",
            "abm_strerror", "abm_last_error", "abm_solve_noalloc")


class AbmProblem(ctypes.Structure):
    _fields_ = [("rhs", ctypes.c_int32), ("d", ctypes.c_int32), ("alpha", ctypes.c_double),
                ("h", ctypes.c_double), ("N", ctypes.c_int64), ("x0", ctypes.c_double * 4),
                ("p", ctypes.c_double * 8), ("far_prec", ctypes.c_int32),
                ("out_stride", ctypes.c_int32), ("alphas", ctypes.c_double * 4),
                ("x1", ctypes.c_double * 4)]


class AbmStats(ctypes.Structure):
    _fields_ = [("block_L", ctypes.c_int32), ("n_groups", ctypes.c_int32),
                ("history_macs", ctypes.c_int64), ("far_macs", ctypes.c_int64),
                ("far_launches", ctypes.c_int32), ("chain_launches", ctypes.c_int32),
                ("far_ms", ctypes.c_double), ("chain_ms", ctypes.c_double),
                ("narrow_groups", ctypes.c_int32), ("reserved_", ctypes.c_int32)]


class AbmResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("t_submit", ctypes.c_double),
                ("t_start", ctypes.c_double), ("t_done", ctypes.c_double),
                ("max_abs_y", ctypes.c_double)]


class AbmTuning(ctypes.Structure):
    _fields_ = [("block_L", ctypes.c_int32), ("kchunk", ctypes.c_int32),
                ("max_split", ctypes.c_int32), ("column_tiles_only", ctypes.c_int32)]


class AbmTuneTrial(ctypes.Structure):
    _fields_ = [("cfg", AbmTuning), ("status", ctypes.c_int32), ("reserved_", ctypes.c_int32),
                ("ms", ctypes.c_double)]


def _tuning_dict(t: AbmTuning) -> dict:
    return {f: getattr(t, f) for f, _ in AbmTuning._fields_}


# Handles still open when the interpreter exits are released before the HIP
# runtime goes away (plans before their contexts); a finalizer running during
# interpreter shutdown would call into a runtime that no longer exists.
_live_plans = weakref.WeakSet()
_live_contexts = weakref.WeakSet()


def _close_all():
    for group in (_live_plans, _live_contexts):
        for obj in list(group):
            try:
                obj.close()
            except Exception:
                pass


atexit.register(_close_all)


class AbmError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str):
        super().__init__("%s failed with %d: %s" % (where, code, detail))
        self.code = code


_lib = None


def load(path: str = LIB_PATH):
    """Load libabm.so; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libabm.so is not built (%s); run paper_1710_01133_amd/build.py" % path)
    lib = ctypes.CDLL(path)
    vp = ctypes.c_void_p
    lib.abm_ctx_create.argtypes = [ctypes.c_int, vp, ctypes.c_size_t, ctypes.POINTER(vp)]
    lib.abm_ctx_destroy.argtypes = [vp]
    lib.abm_ctx_destroy.restype = None
    lib.abm_plan.argtypes = [vp, ctypes.POINTER(AbmProblem), ctypes.c_int32, ctypes.POINTER(vp)]
    lib.abm_plan_destroy.argtypes = [vp]
    lib.abm_plan_destroy.restype = None
    lib.abm_plan_check.argtypes = [vp]
    dp = ctypes.POINTER(ctypes.c_double)
    lib.abm_plan_weights.argtypes = [vp, ctypes.c_int32, ctypes.c_int64, dp, dp, dp]
    lib.abm_plan_timing.argtypes = [vp, ctypes.c_int32]
    lib.abm_plan_tuned.argtypes = [vp, ctypes.POINTER(AbmProblem), ctypes.c_int32,
                                   ctypes.POINTER(AbmTuning), ctypes.POINTER(vp)]
    lib.abm_plan_config.argtypes = [vp, ctypes.POINTER(AbmTuning)]
    lib.abm_autotune.argtypes = [vp, ctypes.POINTER(AbmProblem), ctypes.c_int32, ctypes.c_double,
                                 ctypes.POINTER(AbmTuning), ctypes.POINTER(AbmTuneTrial),
                                 ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
    lib.abm_plan_graph.argtypes = [vp, ctypes.c_int32]
    lib.abm_solve.argtypes = [vp, ctypes.POINTER(AbmProblem), vp]
    lib.abm_solve_batch.argtypes = [vp, ctypes.POINTER(AbmProblem), ctypes.c_int32,
                                    ctypes.POINTER(vp), ctypes.POINTER(AbmStats)]
    lib.abm_submit.argtypes = [vp, ctypes.POINTER(AbmProblem), vp, ctypes.POINTER(ctypes.c_uint64)]
    lib.abm_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(AbmResult)]
    lib.abm_cancel.argtypes = [vp, ctypes.c_uint64]
    lib.abm_request_bytes.argtypes = [vp, ctypes.POINTER(AbmProblem), ctypes.POINTER(ctypes.c_size_t)]
    lib.abm_solve_noalloc.argtypes = [ctypes.POINTER(AbmProblem), vp, vp]
    for name in ("abm_ctx_create", "abm_plan", "abm_plan_check", "abm_plan_weights",
                 "abm_plan_timing", "abm_plan_graph", "abm_solve", "abm_solve_batch", "abm_submit", "abm_poll",
                 "abm_cancel", "abm_request_bytes", "abm_plan_tuned", "abm_plan_config",
                 "abm_autotune", "abm_solve_noalloc"):
        getattr(lib, name).restype = ctypes.c_int32
    lib.abm_strerror.argtypes = [ctypes.c_int32]
    lib.abm_strerror.restype = ctypes.c_char_p
    lib.abm_last_error.argtypes = []
    lib.abm_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(rc: int, where: str):
    if rc != ABM_OK:
        raise AbmError(rc, where, load().abm_last_error().decode(errors="replace"))


def c_problem(p: Problem, out_stride: int = 0) -> AbmProblem:
    c = AbmProblem()
    c.rhs = RHS_ID[p.rhs]
    c.d = RHS_DIM[p.rhs]
    if isinstance(p.alpha, (tuple, list)):
        # incommensurate orders: one per component
        if len(p.alpha) != c.d:
            raise ValueError("alpha needs one order per component (%d)" % c.d)
        c.alpha = 0.0
        for i, v in enumerate(p.alpha):
            c.alphas[i] = float(v)
    else:
        c.alpha = float(p.alpha)
    if p.x1 is not None:
        for i, v in enumerate(p.x1):
            c.x1[i] = float(v)
    c.h = float(p.h)
    c.N = int(p.N)
    for i, v in enumerate(p.x0):
        c.x0[i] = float(v)
    for i, v in enumerate(p.p):
        c.p[i] = float(v)
    c.far_prec = PREC_ID[p.far_prec]
    c.out_stride = int(out_stride)
    return c


def n_out(N: int, out_stride: int) -> int:
    if out_stride == 0:
        return 1
    return N // out_stride + 1 + (1 if N % out_stride else 0)


def _current_stream_handle() -> int:
    import torch
    return int(torch.cuda.current_stream().cuda_stream)


class Context:
    """abm_ctx on one device, enqueueing on a HIP stream (torch's current one by default)."""

    def __init__(self, device: int = 0, stream: Optional[int] = None, arena_bytes: int = 0):
        lib = load()
        self._h = ctypes.c_void_p()
        if stream is None:
            stream = _current_stream_handle()
        _check(lib.abm_ctx_create(device, ctypes.c_void_p(stream), arena_bytes,
                                  ctypes.byref(self._h)), "abm_ctx_create")
        self._plans = weakref.WeakSet()   # plans made on this context
        _live_contexts.add(self)

    @property
    def handle(self):
        return self._h

    def close(self):
        """Destroy the context; plans still open on it are destroyed first
        (a plan must not outlive its context)."""
        if self._h:
            for plan in list(self._plans):
                plan.close()
            load().abm_ctx_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self, _finalizing=sys.is_finalizing):
        # (bound at definition: module globals may already be gone at exit)
        if not getattr(self, "_h", None) or _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


class Plan:
    """abm_plan over a list of problems (their rhs, alpha, N, precision, stride fixed)."""

    def __init__(self, ctx: Context, problems: Sequence[Problem], out_stride: int = 0,
                 tuning: dict = None):
        lib = load()
        self.ctx = ctx
        self.out_stride = out_stride
        self.problems = list(problems)
        arr = (AbmProblem * len(self.problems))(*[c_problem(p, out_stride) for p in self.problems])
        self._h = ctypes.c_void_p()
        if tuning is None:
            _check(lib.abm_plan(ctx.handle, arr, len(self.problems), ctypes.byref(self._h)), "abm_plan")
        else:
            t = AbmTuning(**tuning)
            _check(lib.abm_plan_tuned(ctx.handle, arr, len(self.problems), ctypes.byref(t),
                                      ctypes.byref(self._h)), "abm_plan_tuned")
        ctx._plans.add(self)
        _live_plans.add(self)

    def config(self) -> dict:
        """The blocking the plan uses (block_L, kchunk, max_split, column_tiles_only)."""
        t = AbmTuning()
        _check(load().abm_plan_config(self._h, ctypes.byref(t)), "abm_plan_config")
        return _tuning_dict(t)

    @property
    def handle(self):
        return self._h

    def check(self):
        _check(load().abm_plan_check(self._h), "abm_plan_check")

    def timing(self, enable: bool):
        """Per-launch device timing of solve_batch (far_ms / chain_ms in its stats)."""
        _check(load().abm_plan_timing(self._h, 1 if enable else 0), "abm_plan_timing")

    def graph(self, enable: bool):
        """Replay solve_batch's launch sequence from a HIP graph captured once."""
        _check(load().abm_plan_graph(self._h, 1 if enable else 0), "abm_plan_graph")

    def weights(self, idx: int, n: int):
        """First n weights b, a, c of problem idx's table, as numpy arrays
        ((n, 2) (hi, lo) pairs for a double-double plan)."""
        import numpy as np
        shape = (n, 2) if self.problems[idx].far_prec == "dd" else (n,)
        b = np.zeros(shape, np.float64)
        a = np.zeros(shape, np.float64)
        c = np.zeros(shape, np.float64)
        dp = ctypes.POINTER(ctypes.c_double)
        _check(load().abm_plan_weights(self._h, idx, n, b.ctypes.data_as(dp), a.ctypes.data_as(dp),
                                       c.ctypes.data_as(dp)), "abm_plan_weights")
        return b, a, c

    def close(self):
        if self._h:
            load().abm_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self, _finalizing=sys.is_finalizing):
        # (bound at definition: module globals may already be gone at exit)
        if not getattr(self, "_h", None) or _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


def alloc_out(problem: Problem, out_stride: int, device: str = "cuda"):
    """Output buffer of a solve: (n_out, d) doubles, or (n_out, d, 2) (hi, lo)
    pairs for a double-double problem."""
    import torch
    shape = (n_out(problem.N, out_stride), problem.d)
    if problem.far_prec == "dd":
        shape = shape + (2,)
    return torch.zeros(shape, dtype=torch.float64, device=device)


def solve(plan: Plan, problem: Problem, y_out) -> None:
    """Plain per-step path (plan over one problem).  y_out: float64 device tensor."""
    c = c_problem(problem, plan.out_stride)
    _check(load().abm_solve(plan.handle, ctypes.byref(c), ctypes.c_void_p(y_out.data_ptr())),
           "abm_solve")


def solve_noalloc(problem: Problem, y_out, out_stride: int = 0, stream: Optional[int] = None) -> None:
    """abm_solve_noalloc: the plain path without a plan or any device
    allocation, on the current device and stream (torch's current one by
    default).  y_out: float64 device tensor of n_out(N, out_stride) x d."""
    c = c_problem(problem, out_stride)
    if stream is None:
        stream = _current_stream_handle()
    _check(load().abm_solve_noalloc(ctypes.byref(c), ctypes.c_void_p(y_out.data_ptr()),
                                    ctypes.c_void_p(stream)), "abm_solve_noalloc")


def solve_batch(plan: Plan, problems: Sequence[Problem], y_outs: List) -> dict:
    """Blocked path over the plan's problems; y_outs: one float64 device tensor each."""
    B = len(problems)
    arr = (AbmProblem * B)(*[c_problem(p, plan.out_stride) for p in problems])
    ptrs = (ctypes.c_void_p * B)(*[y.data_ptr() for y in y_outs])
    st = AbmStats()
    _check(load().abm_solve_batch(plan.handle, arr, B, ptrs, ctypes.byref(st)), "abm_solve_batch")
    return {f: getattr(st, f) for f, _ in AbmStats._fields_}


def submit(ctx: Context, problem: Problem, y_out, out_stride: int = 0) -> int:
    c = c_problem(problem, out_stride)
    t = ctypes.c_uint64()
    _check(load().abm_submit(ctx.handle, ctypes.byref(c), ctypes.c_void_p(y_out.data_ptr()),
                             ctypes.byref(t)), "abm_submit")
    return int(t.value)


def poll(ctx: Context, ticket: int):
    """None while running; a dict once done."""
    r = AbmResult()
    rc = load().abm_poll(ctx.handle, ctypes.c_uint64(ticket), ctypes.byref(r))
    if rc == ABM_EAGAIN:
        return None
    _check(rc, "abm_poll")
    return {f: getattr(r, f) for f, _ in AbmResult._fields_}


def autotune(ctx: Context, problems: Sequence[Problem], out_stride: int = 0,
             budget_s: float = 10.0, max_trials: int = 32):
    """abm_autotune: (best blocking, list of trials as dicts with cfg/status/ms)."""
    arr = (AbmProblem * len(problems))(*[c_problem(p, out_stride) for p in problems])
    best = AbmTuning()
    trials = (AbmTuneTrial * max_trials)()
    n = ctypes.c_int32()
    _check(load().abm_autotune(ctx.handle, arr, len(problems), budget_s, ctypes.byref(best),
                               trials, max_trials, ctypes.byref(n)), "abm_autotune")
    out = [{"cfg": _tuning_dict(t.cfg), "status": t.status, "ms": t.ms}
           for t in trials[:min(n.value, max_trials)]]
    return _tuning_dict(best), out


def request_bytes(ctx: Context, problem: Problem, out_stride: int = 0) -> int:
    """Arena bytes the serving loop takes for this request."""
    c = c_problem(problem, out_stride)
    n = ctypes.c_size_t()
    _check(load().abm_request_bytes(ctx.handle, ctypes.byref(c), ctypes.byref(n)), "abm_request_bytes")
    return int(n.value)


def cancel(ctx: Context, ticket: int) -> None:
    _check(load().abm_cancel(ctx.handle, ctypes.c_uint64(ticket)), "abm_cancel")
