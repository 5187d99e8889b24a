"""torch-facing wrappers with the C ABI's names (argument marshalling only)."""
from __future__ import annotations

import ctypes
import threading

import torch

from ._lib import (PIP_F32, PIP_F64, VariantConfig, BatchedConfig, PipError, load_library,
                   num_label_words)

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


def set_option(option: int, value: int, device: int | None = None) -> None:
    d = torch.cuda.current_device() if device is None else device
    ctx = context(d)
    _check(_lib().pip_set_option(ctx, int(option), int(value)), "pip_set_option", ctx)


def get_option(option: int, device: int | None = None) -> int:
    d = torch.cuda.current_device() if device is None else device
    ctx = context(d)
    v = ctypes.c_int64()
    _check(_lib().pip_get_option(ctx, int(option), ctypes.byref(v)), "pip_get_option", ctx)
    return int(v.value)


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


def pip_voronoi_radial_bounds(V):
    """Thresholds of pip_voronoi's radial pre-screen: float32 tensor [17] =
    T_in[8], T_out[8] (octant o = 4 s(X) + 2 s(Y) + (|Y| > |X|), s = sign
    bit of the float32 local coordinate) and T_far."""
    V = _polygon(V)
    d = _dev(V)
    out = torch.empty(17, dtype=torch.float32, device=V.device)
    ctx = context(d)
    s = _lib().pip_voronoi_radial_bounds(ctx, V.data_ptr(), V.shape[0], out.data_ptr(), _stream(d))
    _check(s, "pip_voronoi_radial_bounds", ctx)
    return out


def pip_screen_table(V, test: int = 0, matrix: int = 0):
    """The float32 screen table (float32 tensor [12 + 4 n4]): o_x, o_y, KQ,
    KA, KB, KC, n4, status, RQ (the band's fold radius), SO (sign of offset:
    the one-sided screen's bound on fl32(|X| + |Y|); 0 for Voronoi), 0, 0,
    then n4 rows (A, B, -C, 0) for the Voronoi test (test 0) or the
    sign-of-offset rows, oriented so that the inner side is positive (test
    1), as the vector (matrix 0) or matrix-core (matrix 1) screen derives
    them."""
    V = _polygon(V)
    d = _dev(V)
    n4 = (V.shape[0] + 3) // 4 * 4
    out = torch.empty(12 + 4 * n4, dtype=torch.float32, device=V.device)
    ctx = context(d)
    s = _lib().pip_screen_table(ctx, int(test), int(matrix), V.data_ptr(), V.shape[0],
                                out.data_ptr(), _stream(d))
    _check(s, "pip_screen_table", ctx)
    return out


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


def pip_voronoi_raster(V, x0, y0, dx, dy, width, height, labels=None, status=None):
    """Coverage raster of one convex polygon: pixel (i, j) is the binary64
    point (x0 + i dx, y0 + j dy).  Returns labels [height, ceil(width/32)]
    int32, bit i % 32 of word i // 32 of row j = pixel (i, j) inside."""
    V = _polygon(V)
    d = _dev(V)
    width, height = int(width), int(height)
    rw = num_label_words(width)
    if labels is None:
        labels = torch.empty((max(height, 1), max(rw, 1)), dtype=torch.int32, device=V.device)
    elif labels.numel() < height * rw or not labels.is_contiguous():
        raise ValueError(f"labels must be a contiguous int32 tensor of >= {height * rw} words")
    st = _status_buf(status, d)
    ctx = context(d)
    s = _lib().pip_voronoi_raster(ctx, V.data_ptr(), V.shape[0], float(x0), float(y0), float(dx),
                                  float(dy), width, height, labels.data_ptr(),
                                  st.data_ptr() if st is not None else None, _stream(d))
    _check(s, "pip_voronoi_raster", ctx)
    return labels[:height, :rw] if labels.dim() == 2 else labels


def unpack_labels(words: torch.Tensor, m: int) -> torch.Tensor:
    """Packed int32 words -> bool tensor of m labels (same device)."""
    w = words.contiguous().view(torch.uint8)
    bits = (w.unsqueeze(-1) >> torch.arange(8, device=w.device, dtype=torch.uint8)) & 1
    return bits.reshape(-1)[:m].bool()


# ---------------------------------------------------------------------------
# batched
# ---------------------------------------------------------------------------
def _i64(t, name):
    if t.dtype != torch.int64 or t.dim() != 1 or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous 1-D int64 tensor")
    return t


def label_word_offsets(pt_off: torch.Tensor) -> torch.Tensor:
    """Word offsets that start every set on a fresh 32-bit word."""
    sizes = pt_off[1:] - pt_off[:-1]
    words = (sizes + 31) // 32
    return torch.cat([torch.zeros(1, dtype=torch.int64, device=pt_off.device),
                      torch.cumsum(words, 0)])


def batched_workspace_bytes(P: int, total_vertices: int, total_points: int) -> int:
    return int(_lib().pip_voronoi_batched_workspace_bytes(int(P), int(total_vertices),
                                                          int(total_points)))


class _BatchedArgs:
    def __init__(self, vtx_off, V, pt_off, Q, lbl_word_off, labels, status):
        self.vtx_off = _i64(vtx_off, "vtx_off")
        self.pt_off = _i64(pt_off, "pt_off")
        self.V = _polygon(V)
        if Q.dtype != torch.float32 or Q.dim() != 2 or Q.shape[1] != 2 or not Q.is_contiguous():
            raise ValueError("Q must be a contiguous float32 tensor of shape [m, 2]")
        self.Q = Q
        self.P = self.vtx_off.numel() - 1
        if self.pt_off.numel() != self.P + 1:
            raise ValueError("vtx_off and pt_off must both have P+1 entries")
        self.device = _dev(self.V)
        self.lbl = _i64(lbl_word_off, "lbl_word_off") if lbl_word_off is not None else \
            label_word_offsets(self.pt_off)
        nwords = int(self.lbl[-1].item()) if self.P > 0 else 0
        if labels is None:
            labels = torch.zeros(max(nwords, 1), dtype=torch.int32, device=self.V.device)
        self.labels = labels
        self.status = status if status is not None else \
            torch.zeros(max(self.P, 1), dtype=torch.int32, device=self.V.device)
        self.TV = self.V.shape[0]
        self.TP = self.Q.shape[0]

    def ptrs(self):
        return (self.P, self.vtx_off.data_ptr(), self.V.data_ptr() if self.TV else None, self.TV,
                self.pt_off.data_ptr(), self.Q.data_ptr() if self.TP else None, self.TP,
                self.lbl.data_ptr(), self.labels.data_ptr(), self.status.data_ptr())


def pip_voronoi_batched(vtx_off, V, pt_off, Q, lbl_word_off=None, labels=None, status=None,
                        workspace=None, config=None):
    """Labels of P polygons against their own point sets; returns
    (labels, lbl_word_off, status)."""
    a = _BatchedArgs(vtx_off, V, pt_off, Q, lbl_word_off, labels, status)
    need = batched_workspace_bytes(a.P, a.TV, a.TP)
    if workspace is None:
        workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=a.V.device)
    cfg = None
    if config is not None:
        cfg = BatchedConfig(int(config[0]), int(config[1]))
    ctx = context(a.device)
    s = _lib().pip_voronoi_batched(ctx, *a.ptrs(), workspace.data_ptr(), workspace.numel(),
                                   ctypes.byref(cfg) if cfg is not None else None,
                                   _stream(a.device))
    _check(s, "pip_voronoi_batched", ctx)
    return a.labels, a.lbl, a.status


def pip_voronoi_batched_noalloc(vtx_off, V, pt_off, Q, lbl_word_off=None, labels=None,
                                status=None, config=None):
    """pip_voronoi_batched on the library's static scratch array (no
    workspace; the library call allocates nothing).  Pass ``labels`` and
    ``status`` (and ``lbl_word_off``) to keep this wrapper from allocating
    them.  Returns (labels, lbl_word_off, status)."""
    a = _BatchedArgs(vtx_off, V, pt_off, Q, lbl_word_off, labels, status)
    cfg = None
    if config is not None:
        cfg = BatchedConfig(int(config[0]), int(config[1]))
    ctx = context(a.device)
    s = _lib().pip_voronoi_batched_noalloc(ctx, *a.ptrs(),
                                           ctypes.byref(cfg) if cfg is not None else None,
                                           _stream(a.device))
    _check(s, "pip_voronoi_batched_noalloc", ctx)
    return a.labels, a.lbl, a.status


def pip_plan_create(kind: int, desc, device: int = 0) -> int:
    """The plan handle of pip_plan_create (kind PIP_PLAN_*, desc the kind's
    descriptor structure from ._lib); destroy it with pip_plan_destroy."""
    ctx = context(device)
    h = ctypes.c_void_p()
    s = _lib().pip_plan_create(ctx, int(kind), ctypes.byref(desc), ctypes.byref(h))
    _check(s, "pip_plan_create", ctx)
    return h.value


class BatchedPlan:
    """Autotuned, graph-captured batched launch bound to fixed buffers."""

    def __init__(self, vtx_off, V, pt_off, Q, lbl_word_off=None, labels=None, status=None):
        self.args = _BatchedArgs(vtx_off, V, pt_off, Q, lbl_word_off, labels, status)
        self.ctx = context(self.args.device)
        h = ctypes.c_void_p()
        s = _lib().pip_plan_create_batched(self.ctx, *self.args.ptrs(), ctypes.byref(h))
        _check(s, "pip_plan_create_batched", self.ctx)
        self.handle = h.value

    @property
    def labels(self):
        return self.args.labels

    @property
    def status(self):
        return self.args.status

    @property
    def lbl_word_off(self):
        return self.args.lbl

    def autotune(self, reps: int = 3):
        s = _lib().pip_plan_autotune(self.handle, int(reps), _stream(self.args.device))
        _check(s, "pip_plan_autotune", self.ctx)
        return self.config()

    def launch(self):
        s = _lib().pip_plan_launch(self.handle, _stream(self.args.device))
        _check(s, "pip_plan_launch", self.ctx)
        return self.args.labels

    def config(self):
        cfg = BatchedConfig()
        ms = ctypes.c_float()
        s = _lib().pip_plan_config(self.handle, ctypes.byref(cfg), ctypes.byref(ms))
        _check(s, "pip_plan_config", self.ctx)
        return (cfg.chunks_per_tile, cfg.blocks_per_cu), float(ms.value)

    def set_config(self, chunks_per_tile: int, blocks_per_cu: int):
        cfg = BatchedConfig(int(chunks_per_tile), int(blocks_per_cu))
        s = _lib().pip_plan_set_config(self.handle, ctypes.byref(cfg))
        _check(s, "pip_plan_set_config", self.ctx)

    def close(self):
        if getattr(self, "handle", None):
            _lib().pip_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class LocateIndex:
    """Point-location index over a stored set of convex polygons
    (vtx_off [P+1] int64 and V [total, 2] float64 on the GPU).  locate(Q)
    returns, per float32 point, the smallest index of a polygon containing
    it, or -1."""

    def __init__(self, vtx_off, V, cells: int = 0, status=None):
        vtx_off = _i64(vtx_off, "vtx_off")
        if V.dtype != torch.float64 or V.dim() != 2 or V.shape[1] != 2 or not V.is_contiguous():
            raise ValueError("V must be a contiguous float64 tensor of shape [total, 2]")
        self.device = _dev(vtx_off)
        self.P = vtx_off.numel() - 1
        if status is not None and (status.dtype != torch.int32 or status.numel() < self.P):
            raise ValueError("status must be an int32 tensor with >= P elements")
        self.ctx = context(self.device)
        self._keep = (vtx_off, V)
        h = ctypes.c_void_p()
        s = _lib().pip_index_create(self.ctx, self.P, vtx_off.data_ptr(),
                                    V.data_ptr() if V.numel() else None, V.shape[0], int(cells),
                                    status.data_ptr() if status is not None else None,
                                    _stream(self.device), ctypes.byref(h))
        _check(s, "pip_index_create", self.ctx)
        self.handle = h.value

    def info(self):
        c, e = ctypes.c_int64(), ctypes.c_int64()
        s = _lib().pip_index_info(self.handle, ctypes.byref(c), ctypes.byref(e))
        _check(s, "pip_index_info", self.ctx)
        return int(c.value), int(e.value)

    def workspace_bytes(self, m: int) -> int:
        return int(_lib().pip_index_locate_workspace_bytes(self.handle, int(m)))

    def locate(self, Q, ids=None, binned: bool = True, workspace=None):
        """ids of the points Q; binned=True sorts the points by super-cell
        first (needs a workspace, allocated here unless given)."""
        if Q.dtype != torch.float32 or Q.dim() != 2 or Q.shape[1] != 2 or not Q.is_contiguous():
            raise ValueError("Q must be a contiguous float32 tensor of shape [m, 2]")
        m = Q.shape[0]
        if ids is None:
            ids = torch.empty(max(m, 1), dtype=torch.int32, device=Q.device)
        if binned and m > 0:
            need = self.workspace_bytes(m)
            if workspace is None:
                workspace = torch.empty(need, dtype=torch.uint8, device=Q.device)
            s = _lib().pip_index_locate_binned(self.handle, Q.data_ptr(), m, ids.data_ptr(),
                                               workspace.data_ptr(), workspace.numel(),
                                               _stream(self.device))
            _check(s, "pip_index_locate_binned", self.ctx)
        else:
            s = _lib().pip_index_locate(self.handle, Q.data_ptr() if m else None, m,
                                        ids.data_ptr(), _stream(self.device))
            _check(s, "pip_index_locate", self.ctx)
        return ids[:m]

    def close(self):
        if getattr(self, "handle", None):
            _lib().pip_index_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# poses, all pairs
# ---------------------------------------------------------------------------
def pip_poses_to_polygons(footprint, pose, cs, out=None):
    """[K, n, 2] float64 world vertices of `footprint` at `pose` ([K,3]
    float32) with cos/sin `cs` ([K,2] float64)."""
    F = _polygon(footprint)
    d = _dev(F)
    if pose.dtype != torch.float32 or pose.dim() != 2 or pose.shape[1] != 3 or \
            not pose.is_contiguous():
        raise ValueError("pose must be a contiguous float32 tensor of shape [K, 3]")
    if cs.dtype != torch.float64 or tuple(cs.shape) != (pose.shape[0], 2) or not cs.is_contiguous():
        raise ValueError("cs must be a contiguous float64 tensor of shape [K, 2]")
    K, n = pose.shape[0], F.shape[0]
    if out is None:
        out = torch.empty((K, n, 2), dtype=torch.float64, device=F.device)
    ctx = context(d)
    s = _lib().pip_poses_to_polygons(ctx, F.data_ptr(), n, pose.data_ptr(), cs.data_ptr(), K,
                                     out.data_ptr(), _stream(d))
    _check(s, "pip_poses_to_polygons", ctx)
    return out


class AllpairsPlan:
    """pip_voronoi_allpairs bound to its buffers: autotune() times the exact
    variants (dense, culled, antipodal pairs, both) on the bound data,
    checks that they agree word for word and captures the fastest in a
    hipGraph; launch() replays it."""

    def __init__(self, V, Q, labels=None, counts=None, status=None):
        if V.dtype != torch.float64 or V.dim() != 3 or V.shape[2] != 2 or not V.is_contiguous():
            raise ValueError("V must be a contiguous float64 tensor of shape [P, n, 2]")
        if Q.dtype != torch.float32 or Q.dim() != 2 or Q.shape[1] != 2 or not Q.is_contiguous():
            raise ValueError("Q must be a contiguous float32 tensor of shape [m, 2]")
        self.device = _dev(V)
        Pn, n, m = V.shape[0], V.shape[1], Q.shape[0]
        words = num_label_words(m)
        if labels is None:
            labels = torch.zeros((Pn, max(words, 1)), dtype=torch.int32, device=V.device)
        if counts is None:
            counts = torch.zeros(max(Pn, 1), dtype=torch.int32, device=V.device)
        self.V, self.Q, self.labels, self.counts, self.status = V, Q, labels, counts, status
        self.ctx = context(self.device)
        h = ctypes.c_void_p()
        s = _lib().pip_plan_create_allpairs(self.ctx, Pn, n, V.data_ptr(),
                                            Q.data_ptr() if m else None, m, labels.data_ptr(),
                                            counts.data_ptr(),
                                            status.data_ptr() if status is not None else None,
                                            ctypes.byref(h))
        _check(s, "pip_plan_create_allpairs", self.ctx)
        self.handle = h.value

    def autotune(self, reps: int = 3):
        s = _lib().pip_plan_autotune(self.handle, int(reps), _stream(self.device))
        _check(s, "pip_plan_autotune", self.ctx)
        return self.config()

    def launch(self):
        s = _lib().pip_plan_launch(self.handle, _stream(self.device))
        _check(s, "pip_plan_launch", self.ctx)
        return self.labels, self.counts

    def config(self):
        cfg = VariantConfig()
        ms = ctypes.c_float()
        s = _lib().pip_plan_variant(self.handle, ctypes.byref(cfg), ctypes.byref(ms))
        _check(s, "pip_plan_variant", self.ctx)
        return (cfg.cull, cfg.pair), float(ms.value)

    def set_config(self, cull: int, pair: int):
        cfg = VariantConfig(int(cull), int(pair))
        s = _lib().pip_plan_set_variant(self.handle, ctypes.byref(cfg))
        _check(s, "pip_plan_set_variant", self.ctx)

    def close(self):
        if getattr(self, "handle", None):
            _lib().pip_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def allpairs_workspace_bytes(P: int, n: int) -> int:
    """Bytes of the pip_voronoi_allpairs workspace for P polygons of n edges."""
    return int(_lib().pip_voronoi_allpairs_workspace_bytes(P, n))


def pip_voronoi_allpairs(V, Q, labels=None, counts=None, status=None, workspace=None):
    """V [P, n, 2] float64, Q [m, 2] float32 -> (labels [P, ceil(m/32)] int32,
    counts [P] int32, status [P] int32)."""
    if V.dtype != torch.float64 or V.dim() != 3 or V.shape[2] != 2 or not V.is_contiguous():
        raise ValueError("V must be a contiguous float64 tensor of shape [P, n, 2]")
    if Q.dtype != torch.float32 or Q.dim() != 2 or Q.shape[1] != 2 or not Q.is_contiguous():
        raise ValueError("Q must be a contiguous float32 tensor of shape [m, 2]")
    d = _dev(V)
    Pn, n = V.shape[0], V.shape[1]
    m = Q.shape[0]
    words = num_label_words(m)
    if labels is None:
        labels = torch.empty((Pn, max(words, 1)), dtype=torch.int32, device=V.device)
    if counts is None:
        counts = torch.empty(max(Pn, 1), dtype=torch.int32, device=V.device)
    if status is None:
        status = torch.empty(max(Pn, 1), dtype=torch.int32, device=V.device)
    need = allpairs_workspace_bytes(Pn, n)
    if workspace is None:
        workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=V.device)
    ctx = context(d)
    s = _lib().pip_voronoi_allpairs(ctx, Pn, n, V.data_ptr(), Q.data_ptr() if m else None, m,
                                    labels.data_ptr(), counts.data_ptr(), status.data_ptr(),
                                    workspace.data_ptr(), workspace.numel(), _stream(d))
    _check(s, "pip_voronoi_allpairs", ctx)
    return labels, counts[:Pn], status[:Pn]


def pip_mfma_margin_probe(entries):
    """entries [count, 5] float32 (A, B, c, X, Y) -> [count] float32: A X +
    B Y + c as the matrix-core screen's multiply-add forms it (diagnostic)."""
    if entries.dtype != torch.float32 or entries.dim() != 2 or entries.shape[1] != 5 or \
            not entries.is_contiguous():
        raise ValueError("entries must be a contiguous float32 tensor of shape [count, 5]")
    d = _dev(entries)
    count = entries.shape[0]
    out = torch.empty(max(count, 1), dtype=torch.float32, device=entries.device)
    ctx = context(d)
    s = _lib().pip_mfma_margin_probe(ctx, entries.data_ptr() if count else None, count,
                                     out.data_ptr(), _stream(d))
    _check(s, "pip_mfma_margin_probe", ctx)
    return out[:count]

def allpairs_csr_workspace_bytes(P: int, total_vertices: int) -> int:
    return int(_lib().pip_voronoi_allpairs_csr_workspace_bytes(int(P), int(total_vertices)))


def pip_voronoi_allpairs_csr(vtx_off, V, Q, labels=None, counts=None, status=None,
                             workspace=None):
    """Polygons of uneven vertex counts (vtx_off [P+1] int64, V [total, 2]
    float64) against all points Q [m, 2] float32 -> (labels [P, ceil(m/32)]
    int32, counts [P] int32, status [P] int32)."""
    vtx_off = _i64(vtx_off, "vtx_off")
    V = _polygon(V) if V.shape[0] else V
    if V.dtype != torch.float64 or V.dim() != 2 or V.shape[1] != 2 or not V.is_contiguous():
        raise ValueError("V must be a contiguous float64 tensor of shape [total_vertices, 2]")
    if Q.dtype != torch.float32 or Q.dim() != 2 or Q.shape[1] != 2 or not Q.is_contiguous():
        raise ValueError("Q must be a contiguous float32 tensor of shape [m, 2]")
    d = _dev(Q)
    Pn = vtx_off.numel() - 1
    m = Q.shape[0]
    words = num_label_words(m)
    if labels is None:
        labels = torch.empty((max(Pn, 1), max(words, 1)), dtype=torch.int32, device=Q.device)
    if counts is None:
        counts = torch.empty(max(Pn, 1), dtype=torch.int32, device=Q.device)
    if status is None:
        status = torch.empty(max(Pn, 1), dtype=torch.int32, device=Q.device)
    need = allpairs_csr_workspace_bytes(Pn, V.shape[0])
    if workspace is None:
        workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=Q.device)
    ctx = context(d)
    s = _lib().pip_voronoi_allpairs_csr(ctx, Pn, vtx_off.data_ptr(),
                                        V.data_ptr() if V.shape[0] else None, V.shape[0],
                                        Q.data_ptr() if m else None, m, labels.data_ptr(),
                                        counts.data_ptr(), status.data_ptr(),
                                        workspace.data_ptr(), workspace.numel(), _stream(d))
    _check(s, "pip_voronoi_allpairs_csr", ctx)
    return labels[:Pn], counts[:Pn], status[:Pn]

# -- non-convex polygons: union of convex pieces ------------------------------
def convex_decompose(V, max_piece_vertices: int = 64):
    """Convex pieces of a simple polygon (the library's host routine):
    ``V`` is a host float64 array [n, 2]; returns (piece_off, piece_idx) as
    int32 numpy arrays (K + 1 offsets, vertex indices of each piece)."""
    import numpy as np
    Vn = np.ascontiguousarray(np.asarray(V, dtype=np.float64).reshape(-1, 2))
    n = Vn.shape[0]
    if n < 3:
        raise ValueError("a polygon needs at least 3 vertices")
    off = np.zeros(max(n - 1, 1), dtype=np.int32)
    idx = np.zeros(max(3 * (n - 2), 1), dtype=np.int32)
    K = ctypes.c_int32()
    cnt = ctypes.c_int64()
    s = _lib().pip_convex_decompose(Vn.ctypes.data, n, int(max_piece_vertices), off.ctypes.data,
                                    idx.ctypes.data, ctypes.byref(K), ctypes.byref(cnt))
    _check(s, "pip_convex_decompose", None)
    return off[:K.value + 1].copy(), idx[:cnt.value].copy()


def pieces_workspace_bytes(K: int, idx_count: int) -> int:
    return int(_lib().pip_voronoi_pieces_workspace_bytes(int(K), int(idx_count)))


def pip_voronoi_pieces(V, piece_off, piece_idx, Q, labels=None, status=None, workspace=None):
    """Labels of Q against the union of the convex pieces (device int32
    piece_off [K+1] and piece_idx) of polygon V; returns (labels, status)."""
    V = _polygon(V)
    Q, qdt = _points(Q)
    d = _dev(V)
    for t, name in ((piece_off, "piece_off"), (piece_idx, "piece_idx")):
        if t.dtype != torch.int32 or t.dim() != 1 or not t.is_contiguous() or _dev(t) != d:
            raise ValueError(f"{name} must be a contiguous int32 vector on V's device")
    K = piece_off.numel() - 1
    cnt = piece_idx.numel()
    m = Q.shape[0]
    if labels is None:
        labels = torch.zeros(max(num_label_words(m), 1), dtype=torch.int32, device=V.device)
    if status is None:
        status = torch.zeros(max(K, 1), dtype=torch.int32, device=V.device)
    need = pieces_workspace_bytes(K, cnt)
    if workspace is None:
        workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=V.device)
    ctx = context(d)
    s = _lib().pip_voronoi_pieces(ctx, V.data_ptr(), V.shape[0], K, piece_off.data_ptr(),
                                  piece_idx.data_ptr() if cnt else None, cnt,
                                  Q.data_ptr() if m else None, qdt, m, labels.data_ptr(),
                                  status.data_ptr(), workspace.data_ptr(), workspace.numel(),
                                  _stream(d))
    _check(s, "pip_voronoi_pieces", ctx)
    return labels, status
