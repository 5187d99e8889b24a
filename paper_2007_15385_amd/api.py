"""torch-facing wrappers with the C ABI's names (argument marshalling only)."""
from __future__ import annotations

import ctypes
import threading

import torch

from ._lib import PIP_F32, PIP_F64, PipError, load_library, num_label_words

_ctx_lock = threading.Lock()
_ctx: dict[int, int] = {}


def _lib():
    return load_library()


def context(device: int) -> int:
    """The library context of HIP device ``device`` (created once)."""
    with _ctx_lock:
        h = _ctx.get(device)
        if h is None:
            out = ctypes.c_void_p()
            s = _lib().pip_create(int(device), ctypes.byref(out))
            _check(s, "pip_create", None)
            h = _ctx[device] = out.value
        return h


def _check(s: int, where: str, ctx) -> None:
    if s != 0:
        detail = _lib().pip_last_error(ctx).decode()
        raise PipError(s, where, detail)


def _dev(t: torch.Tensor) -> int:
    if not t.is_cuda:
        raise ValueError("tensors must live on a ROCm GPU device (no CPU fallback)")
    return t.device.index if t.device.index is not None else torch.cuda.current_device()


def _stream(device: int) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _polygon(V: torch.Tensor) -> torch.Tensor:
    if V.dtype != torch.float64 or V.dim() != 2 or V.shape[1] != 2 or not V.is_contiguous():
        raise ValueError("V must be a contiguous float64 tensor of shape [n, 2]")
    return V


def _points(Q: torch.Tensor) -> tuple[torch.Tensor, int]:
    if Q.dim() != 2 or Q.shape[1] != 2 or not Q.is_contiguous():
        raise ValueError("Q must be a contiguous tensor of shape [m, 2]")
    if Q.dtype == torch.float32:
        return Q, PIP_F32
    if Q.dtype == torch.float64:
        return Q, PIP_F64
    raise ValueError("Q must be float32 or float64")


def _status_buf(status, device):
    if status is None:
        return None
    if status.dtype != torch.int32 or status.numel() < 1 or _dev(status) != device:
        raise ValueError("status must be an int32 tensor with >= 1 element on the same device")
    return status


def polygon_to_generators(V: torch.Tensor, out: torch.Tensor | None = None,
                          status: torch.Tensor | None = None) -> torch.Tensor:
    """[n+1, 2] float64 generators: row 0 the centroid, row 1+i edge i's."""
    V = _polygon(V)
    d = _dev(V)
    n = V.shape[0]
    if out is None:
        out = torch.empty((n + 1, 2), dtype=torch.float64, device=V.device)
    elif out.dtype != torch.float64 or out.numel() < 2 * (n + 1) or not out.is_contiguous():
        raise ValueError("out must be a contiguous float64 tensor with 2(n+1) elements")
    status = _status_buf(status, d)
    ctx = context(d)
    s = _lib().polygon_to_generators(ctx, V.data_ptr(), n, out.data_ptr(),
                                     status.data_ptr() if status is not None else None,
                                     _stream(d))
    _check(s, "polygon_to_generators", ctx)
    return out


def _run_labels(fn_name: str, V, Q, labels, status):
    V = _polygon(V)
    Q, qdt = _points(Q)
    d = _dev(V)
    if _dev(Q) != d:
        raise ValueError("V and Q must be on the same device")
    m = Q.shape[0]
    words = num_label_words(m)
    if labels is None:
        labels = torch.empty(max(words, 1), dtype=torch.int32, device=V.device)
    elif labels.dtype not in (torch.int32, torch.uint32) or labels.numel() < words or \
            not labels.is_contiguous() or _dev(labels) != d:
        raise ValueError("labels must be a contiguous int32 tensor with ceil(m/32) elements")
    status = _status_buf(status, d)
    ctx = context(d)
    fn = getattr(_lib(), fn_name)
    s = fn(ctx, V.data_ptr(), V.shape[0], Q.data_ptr() if m else None, qdt, m,
           labels.data_ptr(), status.data_ptr() if status is not None else None, _stream(d))
    _check(s, fn_name, ctx)
    return labels[:words] if labels.numel() != words else labels


def pip_voronoi(V, Q, labels=None, status=None):
    """Packed labels (int32 words, bit k%32 of word k//32 = point k)."""
    return _run_labels("pip_voronoi", V, Q, labels, status)


def pip_sign_of_offset(V, Q, labels=None, status=None):
    return _run_labels("pip_sign_of_offset", V, Q, labels, status)


def pip_ray_crossing(V, Q, labels=None, status=None):
    return _run_labels("pip_ray_crossing", V, Q, labels, status)


def pip_voronoi_fp32_plain(V, Q, labels=None, status=None):
    return _run_labels("pip_voronoi_fp32_plain", V, Q, labels, status)


def pip_voronoi_max_margin(V, Q, out=None, status=None):
    V = _polygon(V)
    Q, qdt = _points(Q)
    d = _dev(V)
    m = Q.shape[0]
    if out is None:
        out = torch.empty(max(m, 1), dtype=torch.float32, device=V.device)
    elif out.dtype != torch.float32 or out.numel() < m or not out.is_contiguous():
        raise ValueError("out must be a contiguous float32 tensor with m elements")
    status = _status_buf(status, d)
    ctx = context(d)
    s = _lib().pip_voronoi_max_margin(ctx, V.data_ptr(), V.shape[0],
                                      Q.data_ptr() if m else None, qdt, m, out.data_ptr(),
                                      status.data_ptr() if status is not None else None,
                                      _stream(d))
    _check(s, "pip_voronoi_max_margin", ctx)
    return out[:m]


def unpack_labels(words: torch.Tensor, m: int) -> torch.Tensor:
    """Packed int32 words -> bool tensor of m labels (same device)."""
    w = words.contiguous().view(torch.uint8)
    bits = (w.unsqueeze(-1) >> torch.arange(8, device=w.device, dtype=torch.uint8)) & 1
    return bits.reshape(-1)[:m].bool()
