"""ctypes binding of the C ABI in include/kdt.h.

Argument marshalling only: every step of the build runs in the gfx950
kernels of ``libkdt.so``.  PyTorch supplies device memory and the current
stream.  If the library has not been built, every call raises; there is no
fallback.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# KDT_LIB selects another build of the same library (e.g. a tuning variant).
LIB_PATH = os.environ.get("KDT_LIB") or os.path.join(_HERE, "libkdt.so")

OK = 0
EINVAL = 1
ENOMEM = 2
EDEVICE = 3
ENONFINITE = 4
EBUSY = 5
ENOTFOUND = 6

STATUS_INTERNAL_BIT = 0x100   # device status: an internal check failed (include/kdt.h)

ROUND_ROBIN = 0
WIDEST = 1
STATIC_WS_BYTES = 64 << 20    # workspace of kdt_build_static (include/kdt.h)
MAX_POINTS = (1 << 30) - 1

_lib = None

_SIGS = {
    "kdt_workspace_bytes": (ctypes.c_size_t, [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int]),
    "kdt_build_ws": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int,
                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "kdt_build": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int,
                                 ctypes.c_void_p]),
    "kdt_build_ws_i32": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "kdt_build_batched_i32": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32,
                                             ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "kdt_permute_payload": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_uint32,
                                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "kdt_build_static": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p]),
    "kdt_inplace_workspace_bytes": (ctypes.c_size_t, [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int]),
    "kdt_build_inplace": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int,
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_size_t, ctypes.c_void_p]),
    "kdt_build_inplace_i32": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_size_t, ctypes.c_void_p]),
    "kdt_batched_workspace_bytes": (ctypes.c_size_t, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32,
                                                      ctypes.c_int]),
    "kdt_build_batched": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32,
                                         ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "kdt_release_cached": (None, []),
    "kdt_server_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "kdt_server_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "kdt_server_poll": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p]),
    "kdt_server_wait": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p]),
    "kdt_server_release": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64]),
    "kdt_server_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "kdt_server_copy_out": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_void_p]),
    "kdt_clock": (ctypes.c_double, []),
    "kdt_tune_batched": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32,
                                        ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_uint32,
                                        ctypes.c_void_p, ctypes.c_void_p]),
    "kdt_tuning_get": (ctypes.c_int, [ctypes.c_uint32, ctypes.c_int, ctypes.c_uint32, ctypes.c_void_p]),
    "kdt_tuning_set": (ctypes.c_int, [ctypes.c_uint32, ctypes.c_int, ctypes.c_uint32, ctypes.c_void_p]),
    "kdt_tuning_save": (ctypes.c_int, [ctypes.c_char_p]),
    "kdt_tuning_load": (ctypes.c_int, [ctypes.c_char_p]),
    "kdt_tuning_clear": (None, []),
    "kdt_profile_enable": (ctypes.c_int, [ctypes.c_int]),
    "kdt_profile_collect": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "kdt_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "kdt_last_error": (ctypes.c_char_p, []),
}


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_uint64),
                ("total_ms", ctypes.c_double), ("alg_bytes", ctypes.c_double),
                ("method_bytes", ctypes.c_double)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("max_inflight", ctypes.c_uint32),
                ("max_batch_requests", ctypes.c_uint32), ("max_batch_points", ctypes.c_uint64)]


class Request(ctypes.Structure):
    _fields_ = [("h_points", ctypes.c_void_p), ("n", ctypes.c_uint32), ("k", ctypes.c_uint32),
                ("dim_mode", ctypes.c_int)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("n", ctypes.c_uint32), ("k", ctypes.c_uint32),
                ("d_tree", ctypes.c_void_p), ("d_perm", ctypes.c_void_p), ("d_dim", ctypes.c_void_p),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double),
                ("device_ms", ctypes.c_double), ("batch_requests", ctypes.c_uint32)]


class Tuning(ctypes.Structure):
    _fields_ = [("radix_bits", ctypes.c_uint32), ("level_items", ctypes.c_uint32), ("rank_layout", ctypes.c_uint32),
                ("presort_dims", ctypes.c_uint32), ("ms", ctypes.c_double)]


class KdtError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {status_string(status)} ({last_error()})")


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
        h = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(h, name)
            f.restype = res
            f.argtypes = args
        _lib = h
    return _lib


def status_string(status: int) -> str:
    return lib().kdt_status_string(int(status)).decode()


def last_error() -> str:
    return lib().kdt_last_error().decode()


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def workspace_bytes(n: int, k: int, mode: int = ROUND_ROBIN) -> int:
    return int(lib().kdt_workspace_bytes(n, k, mode))


def _check_points(points):
    """The points' entry-point suffix: "" for float32, "_i32" for int32."""
    import torch
    if points.dtype not in (torch.float32, torch.int32) or points.dim() != 2 or not points.is_contiguous():
        raise ValueError("points must be a contiguous (N, k) float32 or int32 tensor")
    if not points.is_cuda:
        raise ValueError("points must live on the GPU")
    return "_i32" if points.dtype == torch.int32 else ""


def build_ws(points, mode: int = ROUND_ROBIN, *, tree=None, perm=None, dim=None, status=None,
             workspace=None, stream=None, want_tree=True, want_perm=True, want_dim=True):
    """kdt_build_ws (float32 points) or kdt_build_ws_i32 (int32 points) over
    torch tensors.  Missing outputs are allocated (unless want_* is False);
    returns (tree, perm, dim, status) with status a 1-element int32 device
    tensor holding KDT_OK or KDT_ENONFINITE."""
    import torch
    suffix = _check_points(points)
    n, k = points.shape
    dev = points.device
    if tree is None and want_tree:
        tree = torch.empty((n, k), dtype=points.dtype, device=dev)
    if perm is None and want_perm:
        perm = torch.empty(n, dtype=torch.int32, device=dev)
    if dim is None and want_dim:
        dim = torch.empty(n, dtype=torch.uint8, device=dev)
    if status is None:
        status = torch.zeros(1, dtype=torch.int32, device=dev)
    nbytes = workspace_bytes(n, k, mode)
    if workspace is None:
        workspace = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=dev)
    rc = getattr(lib(), "kdt_build_ws" + suffix)(_ptr(points), n, k, mode, _ptr(tree), _ptr(perm), _ptr(dim),
                                                _ptr(status), _ptr(workspace),
                                                workspace.numel() * workspace.element_size(), _stream(stream))
    if rc != OK:
        raise KdtError(rc, "kdt_build_ws" + suffix)
    return tree, perm, dim, status


def permute_payload(perm, payload, out=None, status=None, stream=None):
    """kdt_permute_payload: out[s] = payload[perm[s]] for a device tensor
    whose first dimension indexes the points (any dtype, any trailing shape,
    contiguous)."""
    import torch
    if not payload.is_contiguous() or not payload.is_cuda or payload.shape[0] != perm.shape[0]:
        raise ValueError("payload must be a contiguous device tensor with one row per point")
    n = payload.shape[0]
    stride = payload.element_size() * (payload.numel() // max(n, 1))
    if out is None:
        out = torch.empty_like(payload)
    rc = lib().kdt_permute_payload(_ptr(perm), n, _ptr(payload), stride, _ptr(out), _ptr(status), _stream(stream))
    if rc != OK:
        raise KdtError(rc, "kdt_permute_payload")
    return out


def build_static(points, mode: int = ROUND_ROBIN, *, tree=None, perm=None, dim=None, status=None, stream=None):
    """kdt_build_static over torch tensors: kdt_build_ws with the library's
    fixed per-device workspace (no device allocation by the library).
    Outputs not given are allocated here by torch; pass them all in to keep
    the call allocation-free.  Returns (tree, perm, dim, status)."""
    import torch
    if _check_points(points):
        raise ValueError("this entry point takes float32 points")
    n, k = points.shape
    dev = points.device
    if tree is None:
        tree = torch.empty((n, k), dtype=torch.float32, device=dev)
    if perm is None:
        perm = torch.empty(n, dtype=torch.int32, device=dev)
    if dim is None:
        dim = torch.empty(n, dtype=torch.uint8, device=dev)
    if status is None:
        status = torch.zeros(1, dtype=torch.int32, device=dev)
    rc = lib().kdt_build_static(_ptr(points), n, k, mode, _ptr(tree), _ptr(perm), _ptr(dim), _ptr(status),
                                _stream(stream))
    if rc != OK:
        raise KdtError(rc, "kdt_build_static")
    return tree, perm, dim, status


def build(points, mode: int = ROUND_ROBIN, stream=None):
    """kdt_build: replace `points` by its tree in level order (in place)."""
    if _check_points(points):
        raise ValueError("this entry point takes float32 points")
    n, k = points.shape
    rc = lib().kdt_build(_ptr(points), n, k, mode, _stream(stream))
    if rc != OK:
        raise KdtError(rc, "kdt_build")
    return points


def inplace_workspace_bytes(n: int, k: int, mode: int = ROUND_ROBIN) -> int:
    return int(lib().kdt_inplace_workspace_bytes(n, k, mode))


def build_inplace(points, mode: int = ROUND_ROBIN, *, perm=None, dim=None, status=None, workspace=None,
                  stream=None, want_dim=True):
    """kdt_build_inplace (float32) or kdt_build_inplace_i32 (int32): replace
    `points` by its tree in level order, with perm (one int32 per point, the
    build's only per-point storage) receiving the original indices.  Missing
    outputs and the (small) workspace are allocated here.  Returns
    (points, perm, dim, status)."""
    import torch
    suffix = _check_points(points)
    n, k = points.shape
    dev = points.device
    if perm is None:
        perm = torch.empty(n, dtype=torch.int32, device=dev)
    if dim is None and want_dim:
        dim = torch.empty(n, dtype=torch.uint8, device=dev)
    if status is None:
        status = torch.zeros(1, dtype=torch.int32, device=dev)
    nbytes = inplace_workspace_bytes(n, k, mode)
    if workspace is None:
        workspace = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=dev)
    rc = getattr(lib(), "kdt_build_inplace" + suffix)(_ptr(points), n, k, mode, _ptr(perm), _ptr(dim),
                                                     _ptr(status), _ptr(workspace),
                                                     workspace.numel() * workspace.element_size(), _stream(stream))
    if rc != OK:
        raise KdtError(rc, "kdt_build_inplace" + suffix)
    return points, perm, dim, status


def _offsets(offsets):
    """Host uint32 copy of the C+1 cloud offsets (kept alive by the caller)."""
    import numpy as np
    o = np.asarray(offsets)
    if o.ndim != 1 or o.size < 2:
        raise ValueError("offsets must be a 1-D array of C+1 entries")
    if int(o[-1]) > MAX_POINTS or int(o.min()) < 0:
        raise ValueError("offsets out of range")
    return np.ascontiguousarray(o, dtype=np.uint32)


def batched_workspace_bytes(offsets, k: int, mode: int = ROUND_ROBIN) -> int:
    o = _offsets(offsets)
    return int(lib().kdt_batched_workspace_bytes(o.ctypes.data_as(ctypes.c_void_p), o.size - 1, k, mode))


def build_batched(points, offsets, mode: int = ROUND_ROBIN, *, tree=None, perm=None, dim=None, status=None,
                  workspace=None, stream=None, want_tree=True, want_perm=True, want_dim=True):
    """kdt_build_batched over torch tensors: points is the (sum N_c, k)
    concatenation of the clouds, offsets the host array of C+1 row offsets.
    Missing outputs are allocated (unless want_* is False); returns
    (tree, perm, dim, status), with perm local to each cloud."""
    import torch
    suffix = _check_points(points)
    n, k = points.shape
    o = _offsets(offsets)
    if int(o[-1]) != n:
        raise ValueError(f"offsets end at {int(o[-1])} but points has {n} rows")
    dev = points.device
    if tree is None and want_tree:
        tree = torch.empty((n, k), dtype=points.dtype, device=dev)
    if perm is None and want_perm:
        perm = torch.empty(n, dtype=torch.int32, device=dev)
    if dim is None and want_dim:
        dim = torch.empty(n, dtype=torch.uint8, device=dev)
    if status is None:
        status = torch.zeros(1, dtype=torch.int32, device=dev)
    if workspace is None:
        nbytes = batched_workspace_bytes(o, k, mode)
        workspace = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=dev)
    rc = getattr(lib(), "kdt_build_batched" + suffix)(_ptr(points), o.ctypes.data_as(ctypes.c_void_p), o.size - 1,
                                                     k, mode, _ptr(tree), _ptr(perm), _ptr(dim), _ptr(status),
                                                     _ptr(workspace), workspace.numel() * workspace.element_size(),
                                                     _stream(stream))
    if rc != OK:
        raise KdtError(rc, "kdt_build_batched" + suffix)
    return tree, perm, dim, status


def tune_batched(points, offsets, mode: int = ROUND_ROBIN, reps: int = 3, workspace=None, stream=None):
    """kdt_tune_batched: time every digit-width / tile / presort-grouping
    choice on this batch and record the fastest; returns (radix_bits,
    level_items, presort_dims, ms)."""
    import torch
    if _check_points(points):
        raise ValueError("this entry point takes float32 points")
    n, k = points.shape
    o = _offsets(offsets)
    if workspace is None:
        workspace = torch.empty(max(batched_workspace_bytes(o, k, mode), 1), dtype=torch.uint8,
                                device=points.device)
    best = Tuning()
    rc = lib().kdt_tune_batched(_ptr(points), o.ctypes.data_as(ctypes.c_void_p), o.size - 1, k, mode,
                                _ptr(workspace), workspace.numel() * workspace.element_size(), reps,
                                _stream(stream), ctypes.byref(best))
    if rc != OK:
        raise KdtError(rc, "kdt_tune_batched")
    return best.radix_bits, best.level_items, best.presort_dims, best.ms


def tuning_get(k: int, mode: int, rank_bits: int):
    t = Tuning()
    rc = lib().kdt_tuning_get(k, mode, rank_bits, ctypes.byref(t))
    if rc != OK:
        raise KdtError(rc, "kdt_tuning_get")
    return t.radix_bits, t.level_items, t.rank_layout, t.presort_dims


def tuning_set(k: int, mode: int, rank_bits: int, radix_bits: int, level_items: int, rank_layout: int = 0,
               presort_dims: int = 0):
    t = Tuning(radix_bits, level_items, rank_layout, presort_dims, 0.0)
    rc = lib().kdt_tuning_set(k, mode, rank_bits, ctypes.byref(t))
    if rc != OK:
        raise KdtError(rc, "kdt_tuning_set")


def tuning_save(path: str):
    rc = lib().kdt_tuning_save(path.encode())
    if rc != OK:
        raise KdtError(rc, "kdt_tuning_save")


def tuning_load(path: str):
    rc = lib().kdt_tuning_load(path.encode())
    if rc != OK:
        raise KdtError(rc, "kdt_tuning_load")


def tuning_clear():
    lib().kdt_tuning_clear()


def release_cached():
    lib().kdt_release_cached()


def profile_enable(on: bool = True):
    """Bracket every kernel of subsequent builds with hipEvents on the build's
    stream (kdt_profile_enable)."""
    lib().kdt_profile_enable(1 if on else 0)


def profile_collect():
    """Per-kernel {launches, total_ms, alg_bytes, method_bytes} recorded since
    the last call."""
    arr = (KernelStat * 32)()
    m = lib().kdt_profile_collect(ctypes.cast(arr, ctypes.c_void_p), 32)
    if m < 0:
        raise RuntimeError(f"kdt_profile_collect failed: {last_error()}")
    return {arr[i].name.decode(): {"launches": int(arr[i].launches), "total_ms": float(arr[i].total_ms),
                                   "alg_bytes": float(arr[i].alg_bytes),
                                   "method_bytes": float(arr[i].method_bytes)} for i in range(m)}


def clock() -> float:
    """Seconds on the monotonic clock of the server's timestamps."""
    return float(lib().kdt_clock())


class Server:
    """kdt_server_*: a request loop that builds trees for submitted host point
    arrays, batching queued requests of the same shape and running up to
    `max_inflight` batches at once inside an HBM budget."""

    def __init__(self, hbm_budget_bytes: int, max_inflight: int = 4, max_batch_requests: int = 64,
                 max_batch_points: int = 1 << 26):
        cfg = ServerConfig(hbm_budget_bytes, max_inflight, max_batch_requests, max_batch_points)
        h = ctypes.c_void_p()
        rc = lib().kdt_server_create(ctypes.byref(cfg), ctypes.byref(h))
        if rc != OK:
            raise KdtError(rc, "kdt_server_create")
        self._h = h
        self._keep = {}      # ticket -> host array kept alive until done

    def submit(self, points, mode: int = ROUND_ROBIN) -> int:
        """Queue a build of `points` (an (n, k) float32 C-contiguous host array:
        numpy, or a torch CPU tensor, ideally pinned); returns the ticket."""
        import numpy as np
        if hasattr(points, "data_ptr"):
            n, k = points.shape
            if points.dtype.__str__() != "torch.float32" or not points.is_contiguous() or points.is_cuda:
                raise ValueError("points must be a contiguous float32 CPU tensor")
            ptr = points.data_ptr()
        else:
            points = np.ascontiguousarray(points, dtype=np.float32)
            n, k = points.shape
            ptr = points.ctypes.data
        req = Request(ctypes.c_void_p(ptr), n, k, mode)
        t = ctypes.c_uint64()
        rc = lib().kdt_server_submit(self._h, ctypes.byref(req), ctypes.byref(t))
        if rc != OK:
            raise KdtError(rc, "kdt_server_submit")
        self._keep[t.value] = points
        return t.value

    def poll(self, ticket: int):
        """The Result once the request is done, else None."""
        r = Result()
        rc = lib().kdt_server_poll(self._h, ticket, ctypes.byref(r))
        if rc == EBUSY:
            return None
        if rc != OK:
            raise KdtError(rc, "kdt_server_poll")
        return r

    def wait(self, ticket: int):
        r = Result()
        rc = lib().kdt_server_wait(self._h, ticket, ctypes.byref(r))
        if rc != OK:
            raise KdtError(rc, "kdt_server_wait")
        return r

    def release(self, ticket: int):
        rc = lib().kdt_server_release(self._h, ticket)
        if rc != OK:
            raise KdtError(rc, "kdt_server_release")
        self._keep.pop(ticket, None)

    def fetch(self, ticket: int):
        """Copy a done request's (tree, perm, dim) from the server's pool into
        new device tensors (on torch's current stream)."""
        import torch
        r = self.wait(ticket)
        n, k = r.n, r.k
        tree = torch.empty((n, k), dtype=torch.float32, device="cuda")
        perm = torch.empty(n, dtype=torch.int32, device="cuda")
        dim = torch.empty(n, dtype=torch.uint8, device="cuda")
        rc = lib().kdt_server_copy_out(self._h, ticket, _ptr(tree), _ptr(perm), _ptr(dim), _stream(None))
        if rc != OK:
            raise KdtError(rc, "kdt_server_copy_out")
        return tree, perm, dim

    def close(self):
        if self._h:
            lib().kdt_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
