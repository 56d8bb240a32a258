"""Python binding of libfgbd (include/fgbd.h): argument marshalling only.

Every step of the denoising path runs in the HIP library; this module turns
torch device tensors into pointers, allocates outputs and the workspace with
torch, and passes torch's current stream.  Loading fails loudly if the
library has not been built.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref
from typing import Optional

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libfgbd.so")

FGBD_OK = 0
FGBD_E_INVALID = -1
FGBD_E_NOMEM = -2
FGBD_E_HIP = -3
FGBD_E_WORKSPACE = -4
FGBD_E_UNSUPPORTED = -5
FGBD_ST_COORD_RANGE = 1
FGBD_ST_NO_PATCH = 2
FGBD_ST_BAD_OFFSETS = 4
FGBD_ST_SWEEP_STALL = 8
FGBD_ST_RELABELED = 16
FGBD_ST_DIST_CLAMPED = 32
NUM_KERNELS = 11
ABI_VERSION = 9
MAX_BATCH = 64
KERNELS = ("radix_upsweep", "radix_scan", "radix_downsweep", "merge", "weights", "noise", "noise_solve", "sweep",
           "finalize", "relabel", "local_sort")


class FgbdError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"fgbd status {status}: {message}")
        self.status = status


class FgbdStallError(RuntimeError):
    """A result carries FGBD_ST_SWEEP_STALL: the in-launch sweeps gave up
    waiting for each other, so that cloud's output is not the method's."""

    def __init__(self, clouds):
        super().__init__(f"filter sweeps stalled for cloud(s) {clouds}: the output colours of those clouds are "
                         "not the selected filter's (the GPU was shared with work that kept blocks from starting)")
        self.clouds = clouds


class Params(ctypes.Structure):
    _fields_ = [
        ("bits", ctypes.c_int32),
        ("num_dirs", ctypes.c_int32),
        ("window", ctypes.c_int32),
        ("k", ctypes.c_int32),
        ("patch", ctypes.c_int32),
        ("q_max", ctypes.c_int32),
        ("fslr_kappa", ctypes.c_double),
        ("sigma_g", ctypes.c_double),
        ("patch_order", ctypes.c_int32),
        ("pad_", ctypes.c_int32),
    ]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "pad_"}


class Graph(ctypes.Structure):
    _fields_ = [
        ("col", ctypes.c_void_p),
        ("dist2", ctypes.c_void_p),
        ("p", ctypes.c_void_p),
        ("n", ctypes.c_int64),
        ("k", ctypes.c_int32),
        ("pad_", ctypes.c_int32),
    ]


class Transpose(ctypes.Structure):
    """fgbd_transpose: for every point the ids of the edges that point at it."""

    _fields_ = [
        ("off", ctypes.c_void_p),
        ("edge", ctypes.c_void_p),
        ("n", ctypes.c_int64),
        ("k", ctypes.c_int32),
        ("pad_", ctypes.c_int32),
    ]


class Schedule(ctypes.Structure):
    """fgbd_schedule: largest grids of the per-cloud kernels and the number of
    filter sweeps enqueued as launches of their own."""

    _fields_ = [("merge_blocks", ctypes.c_int32), ("noise_blocks", ctypes.c_int32),
                ("sweep_blocks", ctypes.c_int32), ("sweep_launches", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {"merge_blocks": self.merge_blocks, "noise_blocks": self.noise_blocks,
                "sweep_blocks": self.sweep_blocks, "sweep_launches": self.sweep_launches}


RESULT_DTYPE = np.dtype([("sigma_est", "<f8"), ("sigma_g", "<f8"), ("loss", "<f8"), ("q", "<i4"),
                         ("n_fslr", "<i4"), ("n_eff", "<i4"), ("status", "<i4"), ("sweeps", "<i4"), ("m", "<i4")])
RESULT_BYTES = RESULT_DTYPE.itemsize  # 48

_lib = None

_SIGNATURES = {
    "fgbd_abi_version": (ctypes.c_int32, []),
    "fgbd_default_params": (ctypes.c_int, [ctypes.POINTER(Params)]),
    "fgbd_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32]),
    "fgbd_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "fgbd_workspace_size": (ctypes.c_int, [ctypes.POINTER(Params), ctypes.c_int64, ctypes.c_int32,
                                           ctypes.POINTER(ctypes.c_size_t)]),
    "fgbd_set_workspace": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]),
    "fgbd_build_slg": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(Params),
                                      ctypes.POINTER(Graph), ctypes.c_void_p, ctypes.c_void_p]),
    "fgbd_estimate_noise": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Graph), ctypes.c_void_p,
                                           ctypes.POINTER(Params), ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_void_p]),
    "fgbd_estimate_noise_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Graph), ctypes.c_void_p,
                                                   ctypes.POINTER(Params), ctypes.c_void_p, ctypes.c_void_p,
                                                   ctypes.c_void_p, ctypes.c_void_p]),
    "fgbd_filter": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Graph), ctypes.c_void_p, ctypes.POINTER(Params),
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_void_p]),
    "fgbd_denoise": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                    ctypes.POINTER(Params), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "fgbd_denoise_batched": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                            ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(Params), ctypes.c_void_p,
                                            ctypes.c_void_p, ctypes.c_void_p]),
    "fgbd_denoise_batched_fixed_q": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                                    ctypes.c_int64, ctypes.c_void_p, ctypes.c_int32,
                                                    ctypes.POINTER(Params), ctypes.c_int32, ctypes.c_void_p,
                                                    ctypes.c_void_p, ctypes.c_void_p]),
    "fgbd_get_schedule": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Schedule)]),
    "fgbd_set_schedule": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Schedule)]),
    "fgbd_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                     ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(Params), ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(Schedule), ctypes.c_void_p]),
    "fgbd_quantize": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "fgbd_smooth_geometry": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(Params),
                                            ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "fgbd_round_u8": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                     ctypes.c_void_p]),
    "fgbd_poly_filter": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Graph), ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p]),
    "fgbd_poly_saved_floats": (ctypes.c_int64, [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32]),
    "fgbd_graph_transpose": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Graph), ctypes.POINTER(Transpose),
                                            ctypes.c_void_p]),
    "fgbd_poly_filter_backward": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Graph), ctypes.POINTER(Transpose),
                                                 ctypes.c_void_p,
                                                 ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                                 ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "fgbd_set_sweep_wait": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64]),
    "fgbd_last_error": (ctypes.c_char_p, []),
    "fgbd_profile_enable": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "fgbd_profile_read": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_int64), ctypes.c_int32]),
}


def lib() -> ctypes.CDLL:
    """The loaded libfgbd.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2401_09721_amd.build`")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        if handle.fgbd_abi_version() != ABI_VERSION:
            raise ImportError(f"{LIB_PATH} has ABI version {handle.fgbd_abi_version()}, the binding expects "
                              f"{ABI_VERSION}: rebuild it")
        _lib = handle
    return _lib


def _check(status: int) -> None:
    if status != FGBD_OK:
        raise FgbdError(status, lib().fgbd_last_error().decode())


def default_params(**overrides) -> Params:
    p = Params()
    _check(lib().fgbd_default_params(ctypes.byref(p)))
    for k, v in overrides.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def as_params(params) -> Params:
    if params is None:
        return default_params()
    if isinstance(params, Params):
        return params
    return default_params(**dict(params))


def workspace_size(params, n_max: int, batch: int = 1) -> int:
    """Workspace bytes for up to n_max points in `batch` clouds."""
    out = ctypes.c_size_t()
    _check(lib().fgbd_workspace_size(ctypes.byref(as_params(params)), int(n_max), int(batch), ctypes.byref(out)))
    return int(out.value)


# ---------------------------------------------------------------- contexts
def _torch():
    import torch

    return torch


# Contexts still open, closed by an exit hook.  The hook is registered when the
# first context is made, after torch has been imported and has registered its
# own exit work; exit hooks run last-registered first, so every context is
# destroyed (its events synchronised, its own workspace freed) while torch and
# the HIP runtime are still up, never from a finaliser during interpreter
# teardown.
_live_contexts: "weakref.WeakSet" = weakref.WeakSet()
_exit_hook = False
_exiting = False


def _close_all_contexts() -> None:
    global _exiting
    _exiting = True
    for c in list(_live_contexts):
        try:
            c.close()
        except Exception:
            pass
    _contexts.clear()


class Context:
    """A library context bound to one GPU, with a torch-allocated workspace."""

    def __init__(self, device=None):
        global _exit_hook
        torch = _torch()
        dev = torch.device(device if device is not None else "cuda")
        idx = dev.index if dev.index is not None else torch.cuda.current_device()
        self.device = torch.device("cuda", idx)
        h = ctypes.c_void_p()
        _check(lib().fgbd_create(ctypes.byref(h), idx))
        self.handle = h
        self._ws = None
        self._ws_bytes = 0
        _live_contexts.add(self)
        if not _exit_hook:
            atexit.register(_close_all_contexts)
            _exit_hook = True

    def reserve(self, params, n: int, batch: int = 1) -> None:
        """Make sure the workspace covers n points in `batch` clouds (call it
        before capturing a graph: a capture must not allocate)."""
        need = workspace_size(params, n, batch)
        if need > self._ws_bytes:
            torch = _torch()
            ws = torch.empty(need, dtype=torch.uint8, device=self.device)
            if ws.data_ptr() % 256:
                raise RuntimeError("torch returned a workspace that is not 256-byte aligned")
            _check(lib().fgbd_set_workspace(self.handle, ctypes.c_void_p(ws.data_ptr()), need))
            self._ws, self._ws_bytes = ws, need

    def schedule(self) -> dict:
        """The context's launch schedule (largest grid of each per-cloud kernel group)."""
        sc = Schedule()
        _check(lib().fgbd_get_schedule(self.handle, ctypes.byref(sc)))
        return sc.as_dict()

    def set_schedule(self, merge_blocks: int, noise_blocks: int, sweep_blocks: int,
                     sweep_launches: int | None = None) -> None:
        """Set the launch schedule; sweep_launches None keeps the current count."""
        if sweep_launches is None:
            sweep_launches = self.schedule()["sweep_launches"]
        sc = Schedule(int(merge_blocks), int(noise_blocks), int(sweep_blocks), int(sweep_launches))
        _check(lib().fgbd_set_schedule(self.handle, ctypes.byref(sc)))

    def autotune(self, xyz, rgb, offsets, params=None, reps: int = 3, out=None, res=None) -> dict:
        """Time candidate launch schedules on this batch (blocking) and keep
        the fastest in the context.  Returns the chosen schedule."""
        torch = _torch()
        prm = as_params(params)
        xyz, rgb, offsets, batch, n = _batched_args(self, xyz, rgb, offsets)
        _check_outputs(self, rgb, out, res, n, max(batch, 1))
        self.reserve(prm, n, max(batch, 1))
        out = torch.empty_like(rgb) if out is None else out
        res = new_result(self.device, max(batch, 1)) if res is None else res
        sc = Schedule()
        _check(lib().fgbd_autotune(self.handle, _ptr(xyz), _ptr(rgb), n, _ptr(offsets), batch, ctypes.byref(prm),
                                   _ptr(out), _ptr(res), int(reps), ctypes.byref(sc), _stream(self)))
        return sc.as_dict()

    def set_sweep_wait(self, microseconds: int) -> None:
        """Bound of the waits between in-launch sweeps (negative: the default
        half second); 0 makes such a launch give up at once (for tests)."""
        _check(lib().fgbd_set_sweep_wait(self.handle, int(microseconds)))

    def profile(self, enable: bool) -> None:
        _check(lib().fgbd_profile_enable(self.handle, 1 if enable else 0))

    def profile_read(self) -> dict:
        """{kernel kind: (summed ms, launches)} since the last read."""
        ms = (ctypes.c_double * NUM_KERNELS)()
        nl = (ctypes.c_int64 * NUM_KERNELS)()
        _check(lib().fgbd_profile_read(self.handle, ms, nl, NUM_KERNELS))
        return {KERNELS[i]: (ms[i], nl[i]) for i in range(NUM_KERNELS)}

    def close(self) -> None:
        """Destroy the library context (waits for its pending events) and drop
        the workspace.  Idempotent."""
        if self.handle:
            lib().fgbd_destroy(self.handle)
            self.handle = None
        self._ws = None
        self._ws_bytes = 0
        _live_contexts.discard(self)

    def __del__(self):
        # after the exit hook has run, the runtime may be going away: leave it
        if _exiting:
            return
        try:
            self.close()
        except Exception:
            pass


_contexts: dict = {}


def default_context(device=None) -> Context:
    torch = _torch()
    dev = torch.device(device if device is not None else "cuda")
    idx = dev.index if dev.index is not None else torch.cuda.current_device()
    if idx not in _contexts:
        _contexts[idx] = Context(torch.device("cuda", idx))
    return _contexts[idx]


# ---------------------------------------------------------------- helpers
def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(0) if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(ctx: Context, stream=None) -> ctypes.c_void_p:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream(ctx.device)
    return ctypes.c_void_p(s.cuda_stream)


def _need(t, dtype, shape_tail, name, device):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != dtype or t.device != device or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {dtype} tensor on {device}")
    if tuple(t.shape[1:]) != tuple(shape_tail):
        raise ValueError(f"{name} must have shape [n, {', '.join(map(str, shape_tail))}]")


def _need_out(t, dtype, shape, name, device):
    """A caller-supplied output: a contiguous tensor of exactly this dtype,
    shape and device (the library writes shape's bytes through its pointer)."""
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != dtype or t.device != device or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {dtype} tensor on {device}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")


def _need_rows(t, n, name):
    if int(t.shape[0]) != int(n):
        raise ValueError(f"{name} has {int(t.shape[0])} rows, the graph has {int(n)}")


def _need_res(res, count, device, name="res"):
    """A caller-supplied result buffer: contiguous uint8 on the device holding
    at least `count` fgbd_result records."""
    torch = _torch()
    if not isinstance(res, torch.Tensor) or res.dtype != torch.uint8 or res.device != device \
            or not res.is_contiguous():
        raise ValueError(f"{name} must be a contiguous uint8 tensor on {device}")
    if res.numel() < RESULT_BYTES * count:
        raise ValueError(f"{name} holds fewer than {count} results ({RESULT_BYTES} bytes each)")


def _need_graph(graph, device):
    """col, dist2 and p of an SLGraph: contiguous [n, k] int32 / int32 / float32
    tensors on the device."""
    torch = _torch()
    n, k = graph.n, graph.k
    for name, t, dt in (("graph.col", graph.col, torch.int32), ("graph.dist2", graph.dist2, torch.int32),
                        ("graph.p", graph.p, torch.float32)):
        _need_out(t, dt, (n, k), name, device)


def _need_disjoint(a, b, name_a, name_b):
    if a is None or b is None or a.numel() == 0 or b.numel() == 0:
        return
    a0, b0 = a.data_ptr(), b.data_ptr()
    a1, b1 = a0 + a.numel() * a.element_size(), b0 + b.numel() * b.element_size()
    if a0 < b1 and b0 < a1:
        raise ValueError(f"{name_a} and {name_b} must not overlap")


def new_result(device, count: int = 1) -> "object":
    """`count` zeroed device fgbd_result records (48 bytes each, as uint8)."""
    torch = _torch()
    return torch.zeros(RESULT_BYTES * count, dtype=torch.uint8, device=device)


def check_results(records: list) -> None:
    """Raise FgbdStallError when a decoded result carries FGBD_ST_SWEEP_STALL;
    warn on FGBD_ST_COORD_RANGE (coordinates outside the grid: the graph is
    undefined) and FGBD_ST_BAD_OFFSETS (offsets were clamped)."""
    import warnings

    stalled = [i for i, r in enumerate(records) if r["status"] & FGBD_ST_SWEEP_STALL]
    if stalled:
        raise FgbdStallError(stalled)
    rng = [i for i, r in enumerate(records) if r["status"] & FGBD_ST_COORD_RANGE]
    if rng:
        warnings.warn(f"coordinates outside 0..2^bits-1 in cloud(s) {rng}: their graphs are undefined",
                      RuntimeWarning, stacklevel=3)
    bad = [i for i, r in enumerate(records) if r["status"] & FGBD_ST_BAD_OFFSETS]
    if bad:
        warnings.warn("batched offsets were not a valid partition and were clamped into one", RuntimeWarning,
                      stacklevel=3)


def read_results(res, check: bool = True) -> list:
    """Copy device fgbd_result records to the host (synchronises) and decode
    them; with check, raise or warn on device-detected conditions
    (check_results)."""
    raw = res.detach().cpu().numpy().tobytes()
    recs = np.frombuffer(raw, dtype=RESULT_DTYPE)
    out = [{name: rec[name].item() for name in RESULT_DTYPE.names} for rec in recs]
    if check:
        check_results(out)
    return out


def read_result(res, check: bool = True) -> dict:
    """The first fgbd_result of a device buffer, decoded (synchronises)."""
    return read_results(res[:RESULT_BYTES], check)[0]


class SLGraph:
    """Device CSR graph returned by build_slg."""

    def __init__(self, col, dist2, p, result):
        self.col, self.dist2, self.p, self.result = col, dist2, p, result

    @property
    def n(self) -> int:
        return int(self.col.shape[0])

    @property
    def k(self) -> int:
        return int(self.col.shape[1])

    def c_struct(self) -> Graph:
        return Graph(_ptr(self.col).value, _ptr(self.dist2).value, _ptr(self.p).value, self.n, self.k, 0)

    def transpose(self, ctx: Optional["Context"] = None, stream=None):
        """The graph's edge transpose (fgbd_graph_transpose), built on first use
        and kept with the graph: (off int32 [n + 1], edge int32 [n * k]).
        Build it again (rebuild=True) after changing col in place."""
        if getattr(self, "_transpose", None) is None:
            self._transpose = graph_transpose(self, ctx=ctx, stream=stream)
        return self._transpose


# ------------------------------------------------------------- the ABI calls
def build_slg(xyz, params=None, ctx: Optional[Context] = None, stream=None) -> SLGraph:
    """Scan-line graph of int32 [n, 3] device coordinates (Sec. 2.2)."""
    torch = _torch()
    prm = as_params(params)
    ctx = ctx or default_context(xyz.device)
    _need(xyz, torch.int32, (3,), "xyz", ctx.device)
    n = int(xyz.shape[0])
    ctx.reserve(prm, n)
    col = torch.empty((n, prm.k), dtype=torch.int32, device=ctx.device)
    dist2 = torch.empty((n, prm.k), dtype=torch.int32, device=ctx.device)
    p = torch.empty((n, prm.k), dtype=torch.float32, device=ctx.device)
    res = new_result(ctx.device)
    g = SLGraph(col, dist2, p, res)
    gs = g.c_struct()
    _check(lib().fgbd_build_slg(ctx.handle, _ptr(xyz), n, ctypes.byref(prm), ctypes.byref(gs), _ptr(res),
                                _stream(ctx, stream)))
    return g


def estimate_noise(graph: SLGraph, rgb, params=None, ctx: Optional[Context] = None, want_spread: bool = True,
                   want_eig3: bool = False, stream=None):
    """NE-GBP (Sec. 2.3).  Returns (result tensor, spread or None, eig3 or None)."""
    torch = _torch()
    prm = as_params(params)
    ctx = ctx or default_context(rgb.device)
    _need(rgb, torch.float32, (3,), "rgb", ctx.device)
    _need_graph(graph, ctx.device)
    n = graph.n
    _need_rows(rgb, n, "rgb")
    ctx.reserve(prm, n)
    res = new_result(ctx.device)
    spread = torch.empty(n, dtype=torch.float64, device=ctx.device) if want_spread else None
    eig3 = torch.empty((n, 3), dtype=torch.float32, device=ctx.device) if want_eig3 else None
    gs = graph.c_struct()
    _check(lib().fgbd_estimate_noise(ctx.handle, ctypes.byref(gs), _ptr(rgb), ctypes.byref(prm), _ptr(res),
                                     _ptr(spread), _ptr(eig3), _stream(ctx, stream)))
    return res, spread, eig3


def estimate_noise_noalloc(graph: SLGraph, rgb, spread, params=None, ctx: Optional[Context] = None, res=None,
                           eig3=None, stream=None):
    """NE-GBP through the call that allocates nothing on the device: its
    scratch is the library's fixed per-GPU array, so the caller passes every
    output (spread: float64 [n]; res: a result buffer; eig3: optional
    float32 [n, 3]).  Calls that overlap on one GPU race on that array.
    Returns res."""
    torch = _torch()
    prm = as_params(params)
    ctx = ctx or default_context(rgb.device)
    _need(rgb, torch.float32, (3,), "rgb", ctx.device)
    _need_graph(graph, ctx.device)
    n = graph.n
    _need_rows(rgb, n, "rgb")
    _need_out(spread, torch.float64, (n,), "spread", ctx.device)
    if eig3 is not None:
        _need_out(eig3, torch.float32, (n, 3), "eig3", ctx.device)
    if res is None:
        raise ValueError("res is required (the call allocates nothing)")
    _need_res(res, 1, ctx.device)
    gs = graph.c_struct()
    _check(lib().fgbd_estimate_noise_noalloc(ctx.handle, ctypes.byref(gs), _ptr(rgb), ctypes.byref(prm), _ptr(res),
                                             _ptr(spread), _ptr(eig3), _stream(ctx, stream)))
    return res


def filter(graph: SLGraph, rgb, params=None, noise=None, spread=None, q_fixed: int = 0,
           ctx: Optional[Context] = None, stream=None):
    """FSLR selection and the eq. 5 filter (noise given) or q_fixed sweeps.
    Returns (rgb_out, result tensor)."""
    torch = _torch()
    prm = as_params(params)
    ctx = ctx or default_context(rgb.device)
    _need(rgb, torch.float32, (3,), "rgb", ctx.device)
    _need_graph(graph, ctx.device)
    n = graph.n
    _need_rows(rgb, n, "rgb")
    if noise is not None:
        _need_res(noise, 1, ctx.device, "noise")
    if spread is not None:
        _need_out(spread, torch.float64, (n,), "spread", ctx.device)
    ctx.reserve(prm, n)
    out = torch.empty_like(rgb)
    res = new_result(ctx.device)
    gs = graph.c_struct()
    _check(lib().fgbd_filter(ctx.handle, ctypes.byref(gs), _ptr(rgb), ctypes.byref(prm), _ptr(noise), _ptr(spread),
                             int(q_fixed), _ptr(out), _ptr(res), _stream(ctx, stream)))
    return out, res


def denoise(xyz, rgb, params=None, ctx: Optional[Context] = None, out=None, res=None, stream=None):
    """The whole per-frame path (Fig. 1(b)).  Returns (rgb_out, result tensor)."""
    torch = _torch()
    prm = as_params(params)
    ctx = ctx or default_context(xyz.device)
    _need(xyz, torch.int32, (3,), "xyz", ctx.device)
    _need(rgb, torch.float32, (3,), "rgb", ctx.device)
    n = int(xyz.shape[0])
    if rgb.shape[0] != n:
        raise ValueError("xyz and rgb sizes differ")
    _check_outputs(ctx, rgb, out, res, n, 1)
    ctx.reserve(prm, n)
    out = torch.empty_like(rgb) if out is None else out
    res = new_result(ctx.device) if res is None else res
    _check(lib().fgbd_denoise(ctx.handle, _ptr(xyz), _ptr(rgb), n, ctypes.byref(prm), _ptr(out), _ptr(res),
                              _stream(ctx, stream)))
    return out, res


def _check_outputs(ctx, rgb, out, res, n, count):
    """Caller-supplied colour output [n, 3] float32 (not overlapping the
    input) and result buffer of `count` records."""
    torch = _torch()
    if out is not None:
        _need_out(out, torch.float32, (n, 3), "out", ctx.device)
        _need_disjoint(rgb, out, "rgb", "out")
    if res is not None:
        _need_res(res, count, ctx.device)


def _batched_args(ctx, xyz, rgb, offsets):
    torch = _torch()
    _need(xyz, torch.int32, (3,), "xyz", ctx.device)
    _need(rgb, torch.float32, (3,), "rgb", ctx.device)
    if not isinstance(offsets, torch.Tensor) or offsets.dtype != torch.int64 or offsets.device != ctx.device \
            or offsets.dim() != 1 or not offsets.is_contiguous():
        raise ValueError(f"offsets must be a contiguous 1-D int64 tensor on {ctx.device}")
    n = int(xyz.shape[0])
    if rgb.shape[0] != n:
        raise ValueError("xyz and rgb sizes differ")
    return xyz, rgb, offsets, int(offsets.numel()) - 1, n


def denoise_batched(xyz, rgb, offsets, params=None, ctx: Optional[Context] = None, out=None, res=None,
                    stream=None):
    """The per-frame path for B clouds stored back to back (cloud s owns rows
    offsets[s] .. offsets[s+1]-1; offsets: int64 device tensor [B+1]).  The
    sizes stay on the device, so a captured call serves any sizes up to
    xyz.shape[0].  Returns (rgb_out, results: uint8 device tensor [B * 48])."""
    torch = _torch()
    prm = as_params(params)
    ctx = ctx or default_context(xyz.device)
    xyz, rgb, offsets, batch, n = _batched_args(ctx, xyz, rgb, offsets)
    _check_outputs(ctx, rgb, out, res, n, max(batch, 1))
    ctx.reserve(prm, n, max(batch, 1))
    out = torch.empty_like(rgb) if out is None else out
    res = new_result(ctx.device, max(batch, 1)) if res is None else res
    _check(lib().fgbd_denoise_batched(ctx.handle, _ptr(xyz), _ptr(rgb), n, _ptr(offsets), batch,
                                      ctypes.byref(prm), _ptr(out), _ptr(res), _stream(ctx, stream)))
    return out, res


def denoise_batched_fixed_q(xyz, rgb, offsets, q: int, params=None, ctx: Optional[Context] = None, out=None,
                            res=None, stream=None):
    """The periodic mode's in-between frames: like denoise_batched, but no
    noise estimate and no selection; every cloud is filtered with q sweeps on
    its own graph (q: the last full frame's selected q).  Returns (rgb_out,
    results)."""
    torch = _torch()
    prm = as_params(params)
    ctx = ctx or default_context(xyz.device)
    xyz, rgb, offsets, batch, n = _batched_args(ctx, xyz, rgb, offsets)
    _check_outputs(ctx, rgb, out, res, n, max(batch, 1))
    ctx.reserve(prm, n, max(batch, 1))
    out = torch.empty_like(rgb) if out is None else out
    res = new_result(ctx.device, max(batch, 1)) if res is None else res
    _check(lib().fgbd_denoise_batched_fixed_q(ctx.handle, _ptr(xyz), _ptr(rgb), n, _ptr(offsets), batch,
                                              ctypes.byref(prm), int(q), _ptr(out), _ptr(res),
                                              _stream(ctx, stream)))
    return out, res


# ------------------------------------------------------- polynomial filter
def quantize(xyz, bits: int = 10, ctx: Optional[Context] = None, out=None, frame=None, stream=None):
    """Float32 [n, 3] device coordinates onto the 2^bits grid with one scale for
    the three axes (Sec. 2.2 takes voxel coordinates).  Returns (int32 [n, 3],
    float64 [4] frame = lo_x, lo_y, lo_z, s)."""
    torch = _torch()
    ctx = ctx or default_context(xyz.device)
    _need(xyz, torch.float32, (3,), "xyz", ctx.device)
    n = int(xyz.shape[0])
    if out is not None:
        _need_out(out, torch.int32, (n, 3), "out", ctx.device)
        _need_disjoint(xyz, out, "xyz", "out")
    if frame is not None:
        _need_out(frame, torch.float64, (4,), "frame", ctx.device)
    out = torch.empty((n, 3), dtype=torch.int32, device=ctx.device) if out is None else out
    frame = torch.empty(4, dtype=torch.float64, device=ctx.device) if frame is None else frame
    _check(lib().fgbd_quantize(ctx.handle, _ptr(xyz), n, int(bits), _ptr(out), _ptr(frame), _stream(ctx, stream)))
    return out, frame


def smooth_geometry(xyz, q: int, params=None, ctx: Optional[Context] = None, out=None, res=None, stream=None):
    """The scan-line graph and q eq. 5 sweeps applied to the int32 [n, 3] device
    coordinates themselves.  Returns (float32 [n, 3], result tensor)."""
    torch = _torch()
    prm = as_params(params)
    ctx = ctx or default_context(xyz.device)
    _need(xyz, torch.int32, (3,), "xyz", ctx.device)
    n = int(xyz.shape[0])
    if out is not None:
        _need_out(out, torch.float32, (n, 3), "out", ctx.device)
        _need_disjoint(xyz, out, "xyz", "out")
    if res is not None:
        _need_res(res, 1, ctx.device)
    ctx.reserve(prm, n)
    out = torch.empty((n, 3), dtype=torch.float32, device=ctx.device) if out is None else out
    res = new_result(ctx.device) if res is None else res
    _check(lib().fgbd_smooth_geometry(ctx.handle, _ptr(xyz), n, ctypes.byref(prm), int(q), _ptr(out), _ptr(res),
                                      _stream(ctx, stream)))
    return out, res


def round_u8(rgb, ctx: Optional[Context] = None, out=None, stream=None):
    """Filtered float32 [n, 3] colours to uint8: round half to even, clip to 0..255."""
    torch = _torch()
    ctx = ctx or default_context(rgb.device)
    _need(rgb, torch.float32, (3,), "rgb", ctx.device)
    n = int(rgb.shape[0])
    if out is not None:
        _need_out(out, torch.uint8, (n, 3), "out", ctx.device)
        _need_disjoint(rgb, out, "rgb", "out")
    out = torch.empty((n, 3), dtype=torch.uint8, device=ctx.device) if out is None else out
    _check(lib().fgbd_round_u8(ctx.handle, _ptr(rgb), n, _ptr(out), _stream(ctx, stream)))
    return out


def saved_floats(n: int, k: int, ncoef: int) -> int:
    """Length of poly_filter's saved buffer (fgbd_poly_saved_floats)."""
    v = int(lib().fgbd_poly_saved_floats(int(n), int(k), int(ncoef)))
    if v < 0:
        raise ValueError(f"no saved buffer for n={n}, k={k}, ncoef={ncoef}")
    return v


def poly_filter(graph: SLGraph, x, coef, sigma_g, ctx: Optional[Context] = None, stream=None):
    """out = sum_k coef[k] T^k x with eq. 4 weights at the device bandwidth
    sigma_g (float64 scalar tensor).  Returns (out, saved): saved is a flat
    float32 buffer of what the backward call needs (the iterates and the
    bandwidth derivatives u_m, [2 ncoef - 1][n][3], then the forward's weights
    and T's diagonal)."""
    torch = _torch()
    ctx = ctx or default_context(x.device)
    _need(x, torch.float32, (3,), "x", ctx.device)
    if coef.dtype != torch.float32 or coef.device != ctx.device or coef.dim() != 1:
        raise ValueError("coef must be a 1-D float32 device tensor")
    if sigma_g.dtype != torch.float64 or sigma_g.device != ctx.device or sigma_g.numel() != 1:
        raise ValueError("sigma_g must be a float64 device scalar")
    _need_graph(graph, ctx.device)
    n, nc = graph.n, int(coef.numel())
    _need_rows(x, n, "x")
    coef = coef.contiguous()
    sigma_g = sigma_g.contiguous()
    out = torch.empty_like(x)
    saved = torch.empty(saved_floats(n, graph.k, nc), dtype=torch.float32, device=ctx.device)
    gs = graph.c_struct()
    _check(lib().fgbd_poly_filter(ctx.handle, ctypes.byref(gs), _ptr(x), _ptr(coef), nc, _ptr(sigma_g), _ptr(out),
                                  _ptr(saved), _stream(ctx, stream)))
    return out, saved


def graph_transpose(graph: SLGraph, ctx: Optional[Context] = None, stream=None):
    """Edge transpose of a graph: (off int32 [n + 1], edge int32 [n * k]) with
    edge[off[j]:off[j + 1]] the ids i * k + slot of the edges pointing at j,
    ascending."""
    torch = _torch()
    ctx = ctx or default_context(graph.col.device)
    _need_out(graph.col, torch.int32, (graph.n, graph.k), "graph.col", ctx.device)
    n, k = graph.n, graph.k
    off = torch.empty(n + 1, dtype=torch.int32, device=ctx.device)
    edge = torch.empty(max(n * k, 1), dtype=torch.int32, device=ctx.device)
    gs = graph.c_struct()
    ts = Transpose(_ptr(off).value, _ptr(edge).value, n, k, 0)
    _check(lib().fgbd_graph_transpose(ctx.handle, ctypes.byref(gs), ctypes.byref(ts), _stream(ctx, stream)))
    return off, edge


def poly_filter_backward(graph: SLGraph, saved, coef, sigma_g, grad_out, ctx: Optional[Context] = None,
                         stream=None, transpose=True):
    """Adjoint of poly_filter.  transpose: True uses the graph's cached edge
    transpose (built on first use), False builds one inside the call, or an
    (off, edge) pair from graph_transpose.  Returns (grad_x, grad_coef,
    grad_sigma_g)."""
    torch = _torch()
    ctx = ctx or default_context(grad_out.device)
    grad_out = grad_out.contiguous()
    _need(grad_out, torch.float32, (3,), "grad_out", ctx.device)
    _need_graph(graph, ctx.device)
    _need_rows(grad_out, graph.n, "grad_out")
    if coef.dtype != torch.float32 or coef.device != ctx.device or coef.dim() != 1:
        raise ValueError("coef must be a 1-D float32 device tensor")
    if sigma_g.dtype != torch.float64 or sigma_g.device != ctx.device or sigma_g.numel() != 1:
        raise ValueError("sigma_g must be a float64 device scalar")
    nc = int(coef.numel())
    _need_out(saved, torch.float32, (saved_floats(graph.n, graph.k, nc),), "saved", ctx.device)
    ts = None
    if transpose is True:
        transpose = graph.transpose(ctx=ctx, stream=stream)
    if transpose is not None and transpose is not False:
        off, edge = transpose
        _need_out(off, torch.int32, (graph.n + 1,), "transpose off", ctx.device)
        if edge.dtype != torch.int32 or edge.device != ctx.device or not edge.is_contiguous() \
                or edge.numel() < graph.n * graph.k:
            raise ValueError(f"transpose edge must be a contiguous int32 tensor on {ctx.device} "
                             f"with at least n * k entries")
        ts = Transpose(_ptr(off).value, _ptr(edge).value, graph.n, graph.k, 0)
    gx = torch.empty_like(grad_out)
    gc = torch.empty(nc, dtype=torch.float32, device=ctx.device)
    gsig = torch.empty((), dtype=torch.float64, device=ctx.device)
    gs = graph.c_struct()
    _check(lib().fgbd_poly_filter_backward(ctx.handle, ctypes.byref(gs), ctypes.byref(ts) if ts is not None else None,
                                           _ptr(saved), _ptr(coef.contiguous()), nc, _ptr(sigma_g.contiguous()),
                                           _ptr(grad_out), _ptr(gx), _ptr(gc), _ptr(gsig), _stream(ctx, stream)))
    return gx, gc, gsig


def _make_autograd():
    torch = _torch()

    class FgbdPolyFilter(torch.autograd.Function):
        """Differentiable polynomial graph filter: gradients with respect to the
        colours, the coefficients and the bandwidth come from the library's
        hand-written adjoint."""

        @staticmethod
        def forward(fctx, x, coef, sigma_g, graph, ctx=None):
            out, saved = poly_filter(graph, x.detach().contiguous(), coef.detach(), sigma_g.detach(), ctx=ctx)
            fctx.graph, fctx.lib_ctx = graph, ctx
            fctx.save_for_backward(saved, coef.detach(), sigma_g.detach())
            return out

        @staticmethod
        def backward(fctx, grad_out):
            saved, coef, sigma_g = fctx.saved_tensors
            gx, gc, gs = poly_filter_backward(fctx.graph, saved, coef, sigma_g, grad_out, ctx=fctx.lib_ctx)
            return gx, gc, gs.reshape(sigma_g.shape), None, None

    return FgbdPolyFilter


_poly_fn = None


def poly_filter_autograd(x, coef, sigma_g, graph: SLGraph, ctx: Optional[Context] = None):
    """FgbdPolyFilter.apply: differentiable in x, coef and sigma_g."""
    global _poly_fn
    if _poly_fn is None:
        _poly_fn = _make_autograd()
    return _poly_fn.apply(x, coef, sigma_g, graph, ctx)
