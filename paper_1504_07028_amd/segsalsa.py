"""Python binding of libsegsalsa.so (argument marshalling only).

Every function here has the name of the C entry point it calls (see
include/segsalsa.h) and does nothing but check tensor shapes/dtypes/devices,
pass raw device pointers and the current HIP stream, and translate status
codes into exceptions.  All arithmetic runs in the HIP kernels.  PyTorch
only provides device memory and streams.
"""
from __future__ import annotations

import ctypes
import math
import os
from ctypes import POINTER, c_char_p, c_double, c_int32, c_size_t, c_void_p

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsegsalsa.so")

SEGSALSA_FP32 = 0
SEGSALSA_FP64 = 1
STATUS = {0: "OK", 1: "INVALID_ARG", 2: "UNSUPPORTED", 3: "WORKSPACE", 4: "DEVICE"}
FLAG_NONFINITE_INPUT = 1
FLAG_NEGATIVE_PROB = 2
FLAG_ZERO_PIXEL = 4


class SegsalsaError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"segsalsa {STATUS.get(status, status)}: {msg}")
        self.status = status


class segsalsa_problem(ctypes.Structure):
    _fields_ = [
        ("K", c_int32), ("H", c_int32), ("W", c_int32), ("patch_radius", c_int32),
        ("patch_weights", POINTER(c_double)),
        ("schatten_p", c_double), ("lambda_", c_double), ("mu", c_double),
        ("iters", c_int32), ("input_is_logits", c_int32), ("residual_every", c_int32),
        ("tol", c_double), ("warm_start", c_int32), ("use_graph", c_int32), ("g4_simplex", c_int32),
    ]


class segsalsa_image(ctypes.Structure):
    _fields_ = [("K", c_int32), ("H", c_int32), ("W", c_int32), ("in_offset", ctypes.c_int64),
                ("out_offset", ctypes.c_int64), ("lambda_", c_double), ("mu", c_double)]


class segsalsa_batch_params(ctypes.Structure):
    _fields_ = [("patch_radius", c_int32), ("patch_weights", POINTER(c_double)), ("schatten_p", c_double),
                ("iters", c_int32), ("input_is_logits", c_int32), ("residual_every", c_int32), ("tol", c_double),
                ("warm_start", c_int32), ("use_graph", c_int32), ("g4_simplex", c_int32)]


class segsalsa_tuning(ctypes.Structure):
    _fields_ = [("tile_rows", c_int32), ("tile_cols", c_int32), ("classes_per_wave", c_int32), ("prefetch", c_int32),
                ("generic_fft", c_int32), ("col_dft", c_int32), ("rows_per_block", c_int32), ("row_threads", c_int32),
                ("cols_per_block", c_int32), ("col_threads", c_int32), ("us_per_round", c_double)]


TUNING_FIELDS = ("tile_rows", "tile_cols", "classes_per_wave", "prefetch", "generic_fft", "col_dft", "rows_per_block",
                 "row_threads", "cols_per_block", "col_threads", "us_per_round")
# Launch shapes measured by segsalsa_str_autotune on an MI355X for the shapes
# the benchmark and the tests run (written by `python -m paper_1504_07028_amd.autotune`).
DEFAULT_TUNING_CACHE = os.path.join(_HERE, "tuning", "mi355x_gfx950.json")


class segsalsa_stats(ctypes.Structure):
    _fields_ = [("primal_res", c_double), ("dual_res", c_double), ("objective", c_double),
                ("rounds_done", c_int32), ("flags", c_int32)]


_lib = None


def lib():
    """Load libsegsalsa.so; raise if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1504_07028_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    L.segsalsa_status_string.argtypes = [c_int32]
    L.segsalsa_status_string.restype = c_char_p
    L.segsalsa_last_error.argtypes = []
    L.segsalsa_last_error.restype = c_char_p
    L.segsalsa_str_workspace_size.argtypes = [POINTER(segsalsa_problem), c_int32, POINTER(c_size_t)]
    L.segsalsa_str_workspace_size.restype = c_int32
    L.segsalsa_str_solve.argtypes = [POINTER(segsalsa_problem), c_int32, c_void_p, c_void_p, c_void_p, c_size_t,
                                     POINTER(segsalsa_stats), c_void_p]
    L.segsalsa_str_solve.restype = c_int32
    L.segsalsa_str_labels.argtypes = [c_int32, c_int32, c_int32, c_int32, c_void_p, c_void_p, c_void_p]
    L.segsalsa_str_labels.restype = c_int32
    L.segsalsa_str_state_export.argtypes = [POINTER(segsalsa_problem), c_int32, c_void_p, c_size_t, c_void_p,
                                            c_void_p, c_void_p, c_void_p, c_void_p]
    L.segsalsa_str_state_export.restype = c_int32
    L.segsalsa_str_state_import.argtypes = [POINTER(segsalsa_problem), c_int32, c_void_p, c_size_t, c_void_p,
                                            c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]
    L.segsalsa_str_state_import.restype = c_int32
    L.segsalsa_str_batch_workspace_size.argtypes = [c_int32, POINTER(segsalsa_image), POINTER(segsalsa_batch_params),
                                                    c_int32, POINTER(c_size_t)]
    L.segsalsa_str_batch_workspace_size.restype = c_int32
    L.segsalsa_str_batch_plans.argtypes = [c_int32, POINTER(segsalsa_image), POINTER(segsalsa_batch_params), c_int32,
                                           POINTER(segsalsa_tuning)]
    L.segsalsa_str_batch_plans.restype = c_int32
    L.segsalsa_str_solve_batch.argtypes = [c_int32, POINTER(segsalsa_image), POINTER(segsalsa_batch_params), c_int32,
                                           c_void_p, c_void_p, c_void_p, c_size_t, POINTER(segsalsa_stats), c_void_p]
    L.segsalsa_str_solve_batch.restype = c_int32
    L.segsalsa_str_grad_workspace_size.argtypes = [POINTER(segsalsa_problem), c_int32, c_int32, POINTER(c_size_t)]
    L.segsalsa_str_grad_workspace_size.restype = c_int32
    L.segsalsa_str_grad_checkpoint_interval.argtypes = [POINTER(segsalsa_problem), c_int32, c_int32, POINTER(c_int32)]
    L.segsalsa_str_grad_checkpoint_interval.restype = c_int32
    L.segsalsa_str_solve_ckpt.argtypes = [POINTER(segsalsa_problem), c_int32, c_int32, c_void_p, c_void_p, c_void_p,
                                          c_size_t, c_void_p]
    L.segsalsa_str_solve_ckpt.restype = c_int32
    L.segsalsa_str_backward.argtypes = [POINTER(segsalsa_problem), c_int32, c_int32, c_void_p, c_void_p, c_void_p,
                                        c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]
    L.segsalsa_str_backward.restype = c_int32
    L.segsalsa_profile_enable.argtypes = [c_int32]
    L.segsalsa_profile_enable.restype = c_int32
    L.segsalsa_profile_read.argtypes = [POINTER(c_double), POINTER(ctypes.c_int64), c_int32]
    L.segsalsa_profile_read.restype = c_int32
    L.segsalsa_stream_copy.argtypes = [c_void_p, c_void_p, c_size_t, c_void_p]
    L.segsalsa_stream_copy.restype = c_int32
    shape = [c_int32, c_int32, c_int32, c_int32, c_int32]
    L.segsalsa_tuning_set.argtypes = shape + [POINTER(segsalsa_tuning)]
    L.segsalsa_tuning_set.restype = c_int32
    L.segsalsa_tuning_get.argtypes = shape + [POINTER(segsalsa_tuning), POINTER(c_int32)]
    L.segsalsa_tuning_get.restype = c_int32
    L.segsalsa_tuning_clear.argtypes = []
    L.segsalsa_tuning_clear.restype = c_int32
    L.segsalsa_tuning_load.argtypes = [c_char_p, POINTER(c_int32), POINTER(c_int32)]
    L.segsalsa_tuning_load.restype = c_int32
    L.segsalsa_tuning_save.argtypes = [c_char_p]
    L.segsalsa_tuning_save.restype = c_int32
    L.segsalsa_str_autotune_workspace_size.argtypes = [POINTER(segsalsa_problem), c_int32, POINTER(c_size_t)]
    L.segsalsa_str_autotune_workspace_size.restype = c_int32
    L.segsalsa_str_autotune.argtypes = [POINTER(segsalsa_problem), c_int32, c_void_p, c_void_p, c_void_p, c_size_t,
                                        c_int32, POINTER(segsalsa_tuning), c_void_p]
    L.segsalsa_str_autotune.restype = c_int32
    L.segsalsa_str_solve_noalloc.argtypes = [POINTER(segsalsa_problem), c_int32, c_void_p, c_void_p, c_void_p]
    L.segsalsa_str_solve_noalloc.restype = c_int32
    _lib = L
    if os.path.exists(DEFAULT_TUNING_CACHE) and not os.environ.get("SEGSALSA_NO_TUNING_CACHE"):
        segsalsa_tuning_load(DEFAULT_TUNING_CACHE)
    return L


def _check(status: int):
    if status != 0:
        raise SegsalsaError(status, lib().segsalsa_last_error().decode())


class Problem:
    """Parameters of one SegSALSA-STR problem (mirrors segsalsa_problem)."""

    def __init__(self, K, H, W, patch_radius, patch_weights, schatten_p=1.0, lam=1.0, mu=1.0, iters=100,
                 input_is_logits=False, residual_every=0, tol=0.0, warm_start=False, use_graph=False,
                 g4_simplex=False):
        self.K, self.H, self.W, self.patch_radius = int(K), int(H), int(W), int(patch_radius)
        self.patch_weights = [float(x) for x in patch_weights]
        self.schatten_p = float(schatten_p)
        self.lam, self.mu, self.iters = float(lam), float(mu), int(iters)
        self.input_is_logits = bool(input_is_logits)
        self.residual_every, self.tol, self.warm_start = int(residual_every), float(tol), bool(warm_start)
        self.use_graph = bool(use_graph)
        self.g4_simplex = bool(g4_simplex)

    def c_struct(self):
        w = (c_double * max(1, len(self.patch_weights)))(*self.patch_weights)
        s = segsalsa_problem(self.K, self.H, self.W, self.patch_radius, ctypes.cast(w, POINTER(c_double)),
                             self.schatten_p, self.lam, self.mu, self.iters, int(self.input_is_logits),
                             self.residual_every, self.tol, int(self.warm_start), int(self.use_graph),
                             int(self.g4_simplex))
        s._keep = w  # keep the weights array alive with the struct
        return s


def _prec(dtype) -> int:
    if dtype == torch.float32:
        return SEGSALSA_FP32
    if dtype == torch.float64:
        return SEGSALSA_FP64
    raise TypeError(f"dtype {dtype} not supported (float32 or float64)")


def _dev_ptr(t, name, dtype=None, numel=None):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a device (HIP) tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} has dtype {t.dtype}, expected {dtype}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")
    return c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return c_void_p(stream.cuda_stream)


def segsalsa_str_workspace_size(problem: Problem, precision: int) -> int:
    n = c_size_t(0)
    s = problem.c_struct()
    _check(lib().segsalsa_str_workspace_size(ctypes.byref(s), int(precision), ctypes.byref(n)))
    return int(n.value)


def segsalsa_str_solve(problem: Problem, inp, z_out, workspace, stats: bool = False, stream=None):
    """Run the rounds on the current stream.  Returns a stats dict if stats=True (then waits)."""
    prec = _prec(z_out.dtype)
    nel = problem.K * problem.H * problem.W
    s = problem.c_struct()
    pin = _dev_ptr(inp, "input", z_out.dtype, nel) if inp is not None else None
    pz = _dev_ptr(z_out, "z_out", None, nel)
    pw = _dev_ptr(workspace, "workspace", torch.uint8)
    st = segsalsa_stats() if stats else None
    _check(lib().segsalsa_str_solve(ctypes.byref(s), prec, pin, pz, pw, workspace.numel(),
                                    ctypes.byref(st) if st is not None else None, _stream(stream)))
    if st is None:
        return None
    return dict(primal_res=st.primal_res, dual_res=st.dual_res, objective=st.objective,
                rounds_done=st.rounds_done, flags=st.flags)


NOALLOC_SCRATCH_BYTES = 256 << 20   # SEGSALSA_NOALLOC_SCRATCH_BYTES


def segsalsa_str_solve_noalloc(problem: Problem, inp, z_out, stream=None):
    """segsalsa_str_solve without a workspace: the state lives in the library's per-GPU scratch array."""
    prec = _prec(z_out.dtype)
    nel = problem.K * problem.H * problem.W
    s = problem.c_struct()
    pin = _dev_ptr(inp, "input", z_out.dtype, nel) if inp is not None else None
    _check(lib().segsalsa_str_solve_noalloc(ctypes.byref(s), prec, pin, _dev_ptr(z_out, "z_out", None, nel),
                                            _stream(stream)))


def segsalsa_str_labels(z, labels, stream=None):
    K, H, W = z.shape
    _check(lib().segsalsa_str_labels(K, H, W, _prec(z.dtype), _dev_ptr(z, "z"),
                                     _dev_ptr(labels, "labels", torch.int32, H * W), _stream(stream)))


def segsalsa_str_state_export(problem: Problem, workspace, d1=None, d2=None, d3=None, d4=None, dtype=None,
                              stream=None):
    dtype = dtype or next(t.dtype for t in (d1, d2, d3, d4) if t is not None)
    s = problem.c_struct()
    nel = problem.K * problem.H * problem.W
    L = (2 * problem.patch_radius + 1) ** 2
    _check(lib().segsalsa_str_state_export(
        ctypes.byref(s), _prec(dtype), _dev_ptr(workspace, "workspace", torch.uint8), workspace.numel(),
        _dev_ptr(d1, "d1", dtype, nel), _dev_ptr(d2, "d2", dtype, 2 * L * nel), _dev_ptr(d3, "d3", dtype, nel),
        _dev_ptr(d4, "d4", dtype, nel), _stream(stream)))


def segsalsa_str_state_import(problem: Problem, workspace, p_hat, d1, d2, d3, d4, stream=None):
    dtype = p_hat.dtype
    s = problem.c_struct()
    nel = problem.K * problem.H * problem.W
    L = (2 * problem.patch_radius + 1) ** 2
    _check(lib().segsalsa_str_state_import(
        ctypes.byref(s), _prec(dtype), _dev_ptr(workspace, "workspace", torch.uint8), workspace.numel(),
        _dev_ptr(p_hat, "p_hat", dtype, nel), _dev_ptr(d1, "d1", dtype, nel), _dev_ptr(d2, "d2", dtype, 2 * L * nel),
        _dev_ptr(d3, "d3", dtype, nel), _dev_ptr(d4, "d4", dtype, nel), _stream(stream)))


class BatchParams:
    """Parameters shared by the images of a batch (mirrors segsalsa_batch_params)."""

    def __init__(self, patch_radius, patch_weights, schatten_p=1.0, iters=100, input_is_logits=False,
                 residual_every=0, tol=0.0, warm_start=False, use_graph=False, g4_simplex=False):
        self.patch_radius = int(patch_radius)
        self.patch_weights = [float(x) for x in patch_weights]
        self.schatten_p, self.iters = float(schatten_p), int(iters)
        self.input_is_logits, self.residual_every, self.tol = bool(input_is_logits), int(residual_every), float(tol)
        self.warm_start, self.use_graph = bool(warm_start), bool(use_graph)
        self.g4_simplex = bool(g4_simplex)

    def c_struct(self):
        w = (c_double * max(1, len(self.patch_weights)))(*self.patch_weights)
        s = segsalsa_batch_params(self.patch_radius, ctypes.cast(w, POINTER(c_double)), self.schatten_p, self.iters,
                                  int(self.input_is_logits), self.residual_every, self.tol, int(self.warm_start),
                                  int(self.use_graph), int(self.g4_simplex))
        s._keep = w
        return s


def image_table(shapes, lams, mus):
    """segsalsa_image array for [K][H][W] images packed back to back (same layout in and out)."""
    arr = (segsalsa_image * len(shapes))()
    off = 0
    for i, ((K, H, W), lam, mu) in enumerate(zip(shapes, lams, mus)):
        arr[i] = segsalsa_image(K, H, W, off, off, lam, mu)
        off += K * H * W
    return arr, off


def segsalsa_str_batch_workspace_size(images, params: BatchParams, precision: int) -> int:
    n = c_size_t(0)
    s = params.c_struct()
    _check(lib().segsalsa_str_batch_workspace_size(len(images), images, ctypes.byref(s), int(precision),
                                                   ctypes.byref(n)))
    return int(n.value)


def segsalsa_str_batch_plans(images, params: BatchParams, precision: int):
    """The launch shapes each image of the batch runs with (dicts of TUNING_FIELDS)."""
    s = params.c_struct()
    out = (segsalsa_tuning * len(images))()
    _check(lib().segsalsa_str_batch_plans(len(images), images, ctypes.byref(s), int(precision), out))
    return [_tuning_dict(t) for t in out]


def segsalsa_str_solve_batch(images, params: BatchParams, inp, z_out, workspace, stats: bool = False, stream=None):
    """Solve all images of the packed batch; returns a list of stats dicts if stats=True (then waits)."""
    prec = _prec(z_out.dtype)
    s = params.c_struct()
    st = (segsalsa_stats * len(images))() if stats else None
    _check(lib().segsalsa_str_solve_batch(len(images), images, ctypes.byref(s), prec,
                                          _dev_ptr(inp, "input", z_out.dtype) if inp is not None else None,
                                          _dev_ptr(z_out, "z_out"), _dev_ptr(workspace, "workspace", torch.uint8),
                                          workspace.numel(), st, _stream(stream)))
    if st is None:
        return None
    return [dict(primal_res=x.primal_res, dual_res=x.dual_res, objective=x.objective, rounds_done=x.rounds_done,
                 flags=x.flags) for x in st]


def segsalsa_str_grad_workspace_size(problem: Problem, precision: int, checkpoint_every: int) -> int:
    n = c_size_t(0)
    s = problem.c_struct()
    _check(lib().segsalsa_str_grad_workspace_size(ctypes.byref(s), int(precision), int(checkpoint_every),
                                                  ctypes.byref(n)))
    return int(n.value)


def segsalsa_str_grad_checkpoint_interval(problem: Problem, precision: int, checkpoint_every: int = 0) -> int:
    """The checkpoint interval S that checkpoint_every (0 = automatic) resolves to."""
    n = c_int32(0)
    s = problem.c_struct()
    _check(lib().segsalsa_str_grad_checkpoint_interval(ctypes.byref(s), int(precision), int(checkpoint_every),
                                                       ctypes.byref(n)))
    return int(n.value)


def segsalsa_str_solve_ckpt(problem: Problem, checkpoint_every: int, inp, z_out, workspace, stream=None):
    nel = problem.K * problem.H * problem.W
    s = problem.c_struct()
    _check(lib().segsalsa_str_solve_ckpt(ctypes.byref(s), _prec(z_out.dtype), int(checkpoint_every),
                                         _dev_ptr(inp, "input", z_out.dtype, nel), _dev_ptr(z_out, "z_out", None, nel),
                                         _dev_ptr(workspace, "workspace", torch.uint8), workspace.numel(),
                                         _stream(stream)))


def segsalsa_str_backward(problem: Problem, checkpoint_every: int, inp, grad_z, grad_input, workspace,
                          grad_lambda=None, grad_weights=None, stream=None):
    """Reverse sweep after segsalsa_str_solve_ckpt: writes grad_input and, if given, the FP64 device
    tensors grad_lambda [1] and grad_weights [L]."""
    nel = problem.K * problem.H * problem.W
    L = (2 * problem.patch_radius + 1) ** 2
    dt = grad_z.dtype
    s = problem.c_struct()
    _check(lib().segsalsa_str_backward(
        ctypes.byref(s), _prec(dt), int(checkpoint_every), _dev_ptr(inp, "input", dt, nel),
        _dev_ptr(grad_z, "grad_z", dt, nel), _dev_ptr(grad_input, "grad_input", dt, nel),
        _dev_ptr(grad_lambda, "grad_lambda", torch.float64, 1),
        _dev_ptr(grad_weights, "grad_weights", torch.float64, L),
        _dev_ptr(workspace, "workspace", torch.uint8), workspace.numel(), _stream(stream)))


def _tuning_dict(t):
    return {f: getattr(t, f) for f in TUNING_FIELDS}


def segsalsa_tuning_set(K, H, W, patch_radius, precision, tuning=None):
    """Set the tuned launch shapes of one image shape (a dict of TUNING_FIELDS; None removes the entry)."""
    t = None
    if tuning is not None:
        t = segsalsa_tuning(*[int(tuning.get(f, 0)) for f in TUNING_FIELDS[:-1]],
                            float(tuning.get("us_per_round", 0.0)))
    _check(lib().segsalsa_tuning_set(K, H, W, patch_radius, int(precision), ctypes.byref(t) if t is not None else None))


def segsalsa_tuning_get(K, H, W, patch_radius, precision):
    """(launch shapes the planner uses for this image shape, whether they come from the tuning table)."""
    t = segsalsa_tuning()
    tuned = c_int32(0)
    _check(lib().segsalsa_tuning_get(K, H, W, patch_radius, int(precision), ctypes.byref(t), ctypes.byref(tuned)))
    return _tuning_dict(t), bool(tuned.value)


def segsalsa_tuning_clear():
    _check(lib().segsalsa_tuning_clear())


def segsalsa_tuning_load(path):
    """Add the entries of a JSON tuning cache to the table; returns (loaded, skipped)."""
    a, b = c_int32(0), c_int32(0)
    _check(lib().segsalsa_tuning_load(os.fsencode(path), ctypes.byref(a), ctypes.byref(b)))
    return int(a.value), int(b.value)


def segsalsa_tuning_save(path):
    _check(lib().segsalsa_tuning_save(os.fsencode(path)))


def segsalsa_str_autotune_workspace_size(problem: Problem, precision: int) -> int:
    n = c_size_t(0)
    s = problem.c_struct()
    _check(lib().segsalsa_str_autotune_workspace_size(ctypes.byref(s), int(precision), ctypes.byref(n)))
    return int(n.value)


def segsalsa_str_autotune(problem: Problem, inp, z_scratch, workspace, rounds=5, stream=None):
    """Measure launch shapes for the problem's image shape; stores the fastest in the tuning table and returns it."""
    nel = problem.K * problem.H * problem.W
    s = problem.c_struct()
    t = segsalsa_tuning()
    _check(lib().segsalsa_str_autotune(ctypes.byref(s), _prec(z_scratch.dtype), _dev_ptr(inp, "input", z_scratch.dtype, nel),
                                       _dev_ptr(z_scratch, "z_scratch", None, nel),
                                       _dev_ptr(workspace, "workspace", torch.uint8), workspace.numel(), int(rounds),
                                       ctypes.byref(t), _stream(stream)))
    return _tuning_dict(t)


class SegSalsaSTR(torch.autograd.Function):
    """z = SegSALSA-STR(input; lambda, c) as an autograd function.

    apply(inp, lam, weights, patch_radius, schatten_p, mu, iters, input_is_logits, checkpoint_every)
    inp: device tensor [K][H][W]; lam: 0-d tensor or float; weights: tensor or list of L multipliers.
    The forward keeps checkpoints in a workspace saved for the backward, which calls the reverse sweep;
    checkpoint_every = 0 lets the library pick the interval (every state where they fit in 8 GiB).
    """

    @staticmethod
    def forward(ctx, inp, lam, weights, patch_radius, schatten_p=1.0, mu=1.0, iters=100, input_is_logits=False,
                checkpoint_every=0):
        inp = inp.contiguous()
        K, H, W = inp.shape
        lam_f = float(lam)
        w = [float(x) for x in (weights.tolist() if isinstance(weights, torch.Tensor) else weights)]
        pr = Problem(K, H, W, patch_radius, w, schatten_p, lam_f, mu, iters, input_is_logits)
        need = segsalsa_str_grad_workspace_size(pr, _prec(inp.dtype), checkpoint_every)
        ws = torch.empty(need, dtype=torch.uint8, device=inp.device)
        z = torch.empty_like(inp)
        segsalsa_str_solve_ckpt(pr, checkpoint_every, inp, z, ws)
        ctx.pr, ctx.ck, ctx.ws = pr, checkpoint_every, ws
        ctx.lam_is_tensor = isinstance(lam, torch.Tensor)
        ctx.w_is_tensor = isinstance(weights, torch.Tensor)
        # gradients go back on the device and in the dtype of the tensors given
        ctx.lam_like = (lam.device, lam.dtype) if ctx.lam_is_tensor else None
        ctx.w_like = (weights.device, weights.dtype) if ctx.w_is_tensor else None
        ctx.save_for_backward(inp)
        return z

    @staticmethod
    def backward(ctx, gz):
        (inp,) = ctx.saved_tensors
        pr = ctx.pr
        L = (2 * pr.patch_radius + 1) ** 2
        gi = torch.empty_like(inp)
        gl = torch.empty(1, dtype=torch.float64, device=inp.device)
        gw = torch.empty(L, dtype=torch.float64, device=inp.device)
        segsalsa_str_backward(pr, ctx.ck, inp, gz.contiguous(), gi, ctx.ws, gl, gw)
        ctx.ws = None
        glam = gl[0].to(device=ctx.lam_like[0], dtype=ctx.lam_like[1]) if ctx.lam_is_tensor else None
        gwt = gw.to(device=ctx.w_like[0], dtype=ctx.w_like[1]) if ctx.w_is_tensor else None
        return (gi, glam, gwt, None, None, None, None, None, None)


PHASES = ("prox_rhs", "fold_row_dft", "col_solve", "row_idft", "adjoint_prox")


def segsalsa_stream_copy(src, dst, stream=None):
    """Copy the bytes of src into dst (device tensors of equal byte size, 16-byte multiples) with
    nontemporal 16-byte loads and stores: the reference for the memory system's streaming rate."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("src and dst differ in size")
    _check(lib().segsalsa_stream_copy(_dev_ptr(src, "src"), _dev_ptr(dst, "dst"), nbytes, _stream(stream)))


def segsalsa_profile_enable(on: bool):
    _check(lib().segsalsa_profile_enable(1 if on else 0))


def segsalsa_profile_read(reset: bool = True):
    """Per-phase totals {phase: (milliseconds, launches)} of the event-timed launches."""
    ms = (c_double * len(PHASES))()
    cnt = (ctypes.c_int64 * len(PHASES))()
    _check(lib().segsalsa_profile_read(ms, cnt, 1 if reset else 0))
    return {name: (ms[i], int(cnt[i])) for i, name in enumerate(PHASES)}


def solve(probs, patch_weights, patch_radius, schatten_p=1.0, lam=1.0, mu=1.0, iters=100, input_is_logits=False,
          workspace=None, stats=False):
    """Convenience wrapper: allocate z and the workspace with torch and run segsalsa_str_solve.

    probs: device tensor [K][H][W] (float32 or float64).  Returns z (and stats if asked).
    """
    K, H, W = probs.shape
    pr = Problem(K, H, W, patch_radius, patch_weights, schatten_p, lam, mu, iters, input_is_logits)
    prec = _prec(probs.dtype)
    need = segsalsa_str_workspace_size(pr, prec)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=probs.device)
    z = torch.empty_like(probs)
    st = segsalsa_str_solve(pr, probs, z, workspace, stats=stats)
    return (z, st) if stats else z


def patch_count(M: int) -> int:
    return (2 * M + 1) ** 2


INF = math.inf
