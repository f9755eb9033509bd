"""MI355X shell fill of Guidefill (arXiv 1611.05319): Python binding.

Argument marshalling only: every step of the fill runs in the HIP library
`libguidefill.so` (built from `csrc/guidefill.hip`, C ABI in
`include/guidefill.h`).  PyTorch supplies device memory and the stream.  There
is no CPU fallback: without the built library or a HIP device every call
raises.

    fill(img, label, guide, eps=3, mu=50)          one frame  (H x W x C)
    fill_batched(img, label, guide, ...)           B frames   (B x H x W x C)
    fill_backward(...)                             reverse-mode derivative
    GuidefillFn.apply(img, theta, label, ...)      autograd w.r.t. the image and
                                                   the guide angle, g = (cos, sin)
"""

from __future__ import annotations

import ctypes
import os
import threading
from dataclasses import dataclass

import torch

__all__ = [
    "Params", "FillResult", "FillPlan", "BackwardPlan", "fill", "fill_batched", "fill_batched_noalloc",
    "guide_field", "fill_coherence", "CoherenceResult",
    "fill_backward", "GuidefillFn",
    "library_path", "load", "stats_fields", "tile_geometry", "ENGINE_TILED", "ENGINE_FRONT",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libguidefill.so")
_lib = None
_lock = threading.Lock()

GF_F32, GF_F16 = 0, 1
SCRATCH_BYTES = 16 << 20  # GF_SCRATCH_BYTES: the static workspace of gf_fill_batched_noalloc
_STATUS = {0: "ok", -1: "invalid argument", -2: "HIP device error", -3: "unsupported request"}
(STAT_SHELLS, STAT_FILLED, STAT_HOLE, STAT_MAX_FRONT, STAT_LABEL_ERR, STAT_ORDER_TRUNC,
 STAT_SYNC_TIMEOUT, STAT_WORKGROUPS) = range(8)
STAT_FRAME0, STAT_PER_FRAME = 8, 4


ENGINE_TILED, ENGINE_FRONT = 0, 1


class _Params(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("mu", ctypes.c_double), ("c", ctypes.c_double),
                ("ghost", ctypes.c_int32), ("tracking", ctypes.c_int32),
                ("max_shells", ctypes.c_int32), ("engine", ctypes.c_int32),
                ("group", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32),
                ("pass_shells", ctypes.c_int32), ("tile_threads", ctypes.c_int32),
                ("c2", ctypes.c_double)]


@dataclass
class Params:
    """Fill parameters (gf_params).  c < 0: onion order; c >= 0: smart order;
    c2 >= 0: the data term of eqn:ready2 (|g| > c2) until it leaves nothing ready.
    engine 0: tiled (LDS windows, pass_shells shells per grid sync);
    engine 1: one grid sync per shell with a global front list."""

    eps: float = 3.0
    mu: float = 50.0
    c: float = -1.0
    ghost: bool = True
    tracking: bool = True
    max_shells: int = 0
    engine: int = ENGINE_TILED
    group: int = 0
    blocks_per_cu: int = 0
    tile_w: int = 0
    tile_h: int = 0
    pass_shells: int = 0
    tile_threads: int = 0
    c2: float = -1.0

    def c_struct(self) -> _Params:
        return _Params(float(self.eps), float(self.mu), float(self.c), int(bool(self.ghost)),
                       int(bool(self.tracking)), int(self.max_shells), int(self.engine),
                       int(self.group), int(self.blocks_per_cu), int(self.tile_w),
                       int(self.tile_h), int(self.pass_shells), int(self.tile_threads),
                       float(self.c2))


def library_path() -> str:
    return _LIB_PATH


def load():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(
                f"{_LIB_PATH} is missing: build it with `python -m paper_1611_05319_amd.build`")
        lib = ctypes.CDLL(_LIB_PATH)
        P, I, Z = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t
        PP = ctypes.POINTER(_Params)
        lib.gf_workspace_size.argtypes = [I, I, I, I, I, PP]
        lib.gf_workspace_size.restype = Z
        lib.gf_backward_workspace_size.argtypes = [I, I, I, I, I, PP]
        lib.gf_backward_workspace_size.restype = Z
        lib.gf_fill_batched.argtypes = [P, P, I, I, I, I, I, P, P, PP, P, P, P, P, P, I, P, Z, P]
        lib.gf_fill_batched.restype = I
        lib.gf_fill_batched_noalloc.argtypes = [P, P, I, I, I, I, I, P, P, PP, P, P, P, P, P, I, P]
        lib.gf_fill_batched_noalloc.restype = I
        lib.gf_coherence_workspace_size.argtypes = [I, I, I, I, I, P]
        lib.gf_coherence_workspace_size.restype = Z
        D = ctypes.c_double
        lib.gf_fill_coherence.argtypes = [P, P, I, I, I, I, I, P, P, D, D, D, P, P, P, P, Z, P]
        lib.gf_fill_coherence.restype = I
        lib.gf_guide_field.argtypes = [I, I, I, P, P, P, ctypes.c_double, ctypes.c_double, P, P]
        lib.gf_guide_field.restype = I
        lib.gf_fill.argtypes = [P, P, I, I, I, I, P, P, PP, P, P, P, Z, P]
        lib.gf_fill.restype = I
        lib.gf_fill_backward.argtypes = [P, P, I, I, I, I, I, P, P, P, I, PP, P, P, P, Z, P]
        lib.gf_fill_backward.restype = I
        lib.gf_status_string.argtypes = [I]
        lib.gf_status_string.restype = ctypes.c_char_p
        lib.gf_last_error.argtypes = []
        lib.gf_last_error.restype = ctypes.c_char_p
        lib.gf_version.argtypes = []
        lib.gf_version.restype = I
        lib.gf_tile_geometry.argtypes = [I, I, I, I, PP, P]
        lib.gf_tile_geometry.restype = I
        _lib = lib
        return lib


def _check(rc: int, what: str):
    if rc != 0:
        lib = load()
        msg = lib.gf_status_string(rc).decode()
        detail = lib.gf_last_error().decode()
        raise RuntimeError(f"{what} failed: {msg} ({rc}) {detail}")


def _ptr(t: torch.Tensor | None):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream_ptr(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float32:
        return GF_F32
    if t.dtype == torch.float16:
        return GF_F16
    raise TypeError("image must be float32 or float16")


def _require_device(*ts):
    dev = None
    for t in ts:
        if t is None:
            continue
        if not t.is_cuda:
            raise ValueError("all tensors must be on the HIP device")
        if not t.is_contiguous():
            raise ValueError("all tensors must be contiguous")
        dev = t.device if dev is None else dev
        if t.device != dev:
            raise ValueError("all tensors must be on the same device")
    return dev


@dataclass
class FillResult:
    out: torch.Tensor          # filled image(s)
    shell: torch.Tensor        # int32 shell map(s)
    stats: torch.Tensor        # int32 device stats (layout in include/guidefill.h)
    order: torch.Tensor | None = None
    shell_offsets: torch.Tensor | None = None
    front_hist: torch.Tensor | None = None

    def host_stats(self) -> dict:
        return stats_fields(self.stats)


def tile_geometry(H: int, W: int, C: int, dtype=torch.float32, params: Params | None = None):
    """(tile_w, tile_h, pass_shells, halo, window LDS bytes, lanes per pixel) the
    tiled engine uses for these parameters on the current device."""
    lib = load()
    p = (params or Params()).c_struct()
    out = (ctypes.c_int32 * 6)()
    rc = lib.gf_tile_geometry(H, W, C, GF_F16 if dtype == torch.float16 else GF_F32,
                              ctypes.byref(p), out)
    _check(rc, "gf_tile_geometry")
    return tuple(out)


def stats_fields(stats: torch.Tensor) -> dict:
    s = stats.cpu().tolist()
    B = (len(s) - STAT_FRAME0) // STAT_PER_FRAME
    frames = [s[STAT_FRAME0 + STAT_PER_FRAME * f:STAT_FRAME0 + STAT_PER_FRAME * (f + 1)]
              for f in range(B)]
    return {
        "K": s[STAT_SHELLS], "filled": s[STAT_FILLED], "hole": s[STAT_HOLE],
        "unfilled": s[STAT_HOLE] - s[STAT_FILLED], "max_front": s[STAT_MAX_FRONT],
        "label_errors": s[STAT_LABEL_ERR], "order_truncated": bool(s[STAT_ORDER_TRUNC]),
        "sync_timeout": bool(s[STAT_SYNC_TIMEOUT]),
        "workgroups": s[STAT_WORKGROUPS],
        "frame_K": [fr[0] for fr in frames], "frame_filled": [fr[1] for fr in frames],
        "frame_hole": [fr[2] for fr in frames],
    }


class Workspace:
    """Reusable device workspace (grows on demand)."""

    def __init__(self):
        self.buf = None

    def get(self, nbytes: int, device) -> torch.Tensor:
        if self.buf is None or self.buf.numel() < nbytes or self.buf.device != device:
            self.buf = torch.zeros(max(nbytes, 256), dtype=torch.uint8, device=device)
        return self.buf


_default_ws = threading.local()


def _workspace(nbytes: int, device) -> torch.Tensor:
    ws = getattr(_default_ws, "ws", None)
    if ws is None:
        ws = Workspace()
        _default_ws.ws = ws
    return ws.get(nbytes, device)


def fill_batched(img: torch.Tensor, label: torch.Tensor, guide: torch.Tensor,
                 params: Params | None = None, out: torch.Tensor | None = None,
                 shell: torch.Tensor | None = None, record_order: bool = False,
                 record_fronts: bool = False, kcap: int | None = None,
                 workspace: torch.Tensor | None = None, **kw) -> FillResult:
    """Fill B frames in one launch.  img: B x H x W x C (float32 or float16),
    label: B x H x W uint8, guide: B x H x W x 2 float32.  `out` may be `img`
    (in place).  Keyword arguments override fields of `params`."""
    p = params or Params()
    if kw:
        p = Params(**{**p.__dict__, **kw})
    dev = _require_device(img, label, guide, out, shell)
    if img.dim() != 4 or label.dim() != 3 or guide.dim() != 4:
        raise ValueError("expected img B x H x W x C, label B x H x W, guide B x H x W x 2")
    B, H, W, C = img.shape
    if tuple(label.shape) != (B, H, W) or tuple(guide.shape) != (B, H, W, 2):
        raise ValueError("shape mismatch between img, label and guide")
    if label.dtype != torch.uint8 or guide.dtype != torch.float32:
        raise TypeError("label must be uint8 and guide float32")
    lib = load()
    if record_order and p.engine != ENGINE_FRONT:
        p = Params(**{**p.__dict__, "engine": ENGINE_FRONT})  # the fill order comes from that engine
    if out is None:
        out = torch.empty_like(img)
    if shell is None:
        shell = torch.empty((B, H, W), dtype=torch.int32, device=dev)
    stats = torch.empty(STAT_FRAME0 + STAT_PER_FRAME * B, dtype=torch.int32, device=dev)
    cp = p.c_struct()
    dt = _dtype_code(img)
    if kcap is None:
        kcap = min(H * W, 1 << 16) + 1
    order = offs = hist = None
    if record_order:
        order = torch.empty(B * H * W, dtype=torch.int32, device=dev)
        offs = torch.zeros(kcap, dtype=torch.int32, device=dev)
    if record_fronts:
        hist = torch.zeros(kcap, dtype=torch.int32, device=dev)
    nbytes = lib.gf_workspace_size(B, H, W, C, dt, ctypes.byref(cp))
    ws = workspace if workspace is not None else _workspace(nbytes, dev)
    rc = lib.gf_fill_batched(_ptr(img), _ptr(out), B, H, W, C, dt, _ptr(label), _ptr(guide),
                             ctypes.byref(cp), _ptr(shell), _ptr(stats), _ptr(order), _ptr(offs),
                             _ptr(hist), int(kcap), _ptr(ws), ws.numel(), _stream_ptr(dev))
    _check(rc, "gf_fill_batched")
    return FillResult(out, shell, stats, order, offs, hist)


def fill_batched_noalloc(img: torch.Tensor, label: torch.Tensor, guide: torch.Tensor,
                         params: Params, out: torch.Tensor, shell: torch.Tensor,
                         stats: torch.Tensor, stream: torch.cuda.Stream | None = None) -> FillResult:
    """gf_fill_batched_noalloc: fill_batched into caller-provided `out`, `shell`
    and `stats` (int32, 8 + 4 B entries) with the library's static scratch as
    the workspace; neither this function nor the library allocates."""
    dev = _require_device(img, label, guide, out, shell, stats)
    B, H, W, C = img.shape
    if tuple(label.shape) != (B, H, W) or tuple(guide.shape) != (B, H, W, 2):
        raise ValueError("shape mismatch between img, label and guide")
    if tuple(out.shape) != tuple(img.shape) or tuple(shell.shape) != (B, H, W):
        raise ValueError("shape mismatch of out or shell")
    if stats.dtype != torch.int32 or stats.numel() < STAT_FRAME0 + STAT_PER_FRAME * B:
        raise ValueError("stats must be int32 with 8 + 4 B entries")
    lib = load()
    cp = params.c_struct()
    s = stream if stream is not None else torch.cuda.current_stream(dev)
    rc = lib.gf_fill_batched_noalloc(_ptr(img), _ptr(out), B, H, W, C, _dtype_code(img), _ptr(label),
                                     _ptr(guide), ctypes.byref(cp), _ptr(shell), _ptr(stats), None,
                                     None, None, 0, ctypes.c_void_p(s.cuda_stream))
    _check(rc, "gf_fill_batched_noalloc")
    return FillResult(out, shell, stats)


@dataclass
class CoherenceResult:
    out: torch.Tensor          # (B x) H x W x C filled image
    shell: torch.Tensor        # (B x) H x W int32 shell map
    stats: torch.Tensor        # int32 stats (gf_fill_batched layout)
    guide_used: torch.Tensor | None  # (B x) H x W x 2: the guide each pixel was filled with


def fill_coherence(img: torch.Tensor, label: torch.Tensor, params: Params | None = None,
                   sigma: float = 2.0, rho: float = 4.0, Lambda: float = 1e-5,
                   out: torch.Tensor | None = None, want_guide: bool = True,
                   workspace: Workspace | None = None) -> CoherenceResult:
    """gf_fill_coherence: the coherence-transport comparison mode (the guide
    re-estimated before every shell from the modified structure tensor of the
    known pixels).  params default to the lattice ball (ghost off).  The call
    returns when the fill has finished (one host read-back per shell)."""
    squeeze = img.dim() == 3
    im = img.unsqueeze(0) if squeeze else img
    lab = label.unsqueeze(0) if squeeze else label
    dev = _require_device(im, lab)
    B, H, W, C = im.shape
    if lab.shape != (B, H, W) or lab.dtype != torch.uint8:
        raise ValueError("label must be (B x) H x W uint8")
    p = params if params is not None else Params(ghost=False)
    pc = p.c_struct()
    dt = _dtype_code(im)
    lib = load()
    need = lib.gf_coherence_workspace_size(B, H, W, C, dt, ctypes.byref(pc))
    if need == 0:
        raise RuntimeError(f"gf_coherence_workspace_size rejected the request: {lib.gf_last_error().decode()}")
    ws = workspace if workspace is not None else Workspace()
    buf = ws.get(need, dev)
    o = out if out is not None else torch.empty_like(im)
    shell = torch.empty((B, H, W), dtype=torch.int32, device=dev)
    stats = torch.empty(STAT_FRAME0 + STAT_PER_FRAME * B, dtype=torch.int32, device=dev)
    gu = torch.empty((B, H, W, 2), dtype=torch.float32, device=dev) if want_guide else None
    rc = lib.gf_fill_coherence(_ptr(im), _ptr(o), B, H, W, C, dt, _ptr(lab), ctypes.byref(pc),
                               float(sigma), float(rho), float(Lambda), _ptr(shell), _ptr(stats),
                               _ptr(gu), _ptr(buf), need, _stream_ptr(dev))
    _check(rc, "gf_fill_coherence")
    if squeeze:
        return CoherenceResult(o[0], shell[0], stats, gu[0] if gu is not None else None)
    return CoherenceResult(o, shell, stats, gu)


def guide_field(label: torch.Tensor, seg: torch.Tensor, seg_off: torch.Tensor, eta: float = 3.0,
                cutoff: float | None = None, out: torch.Tensor | None = None,
                check_offsets: bool = True) -> torch.Tensor:
    """gf_guide_field: the guide field of Sec. 3.2 from polyline splines.
    label: (B x) H x W uint8; seg: n x 6 float32 (x0, y0, x1, y1, gx, gy);
    seg_off: B + 1 int32 offsets of each frame's segments; cutoff defaults to
    3 eta.  Returns (B x) H x W x 2 float32.  check_offsets reads seg_off back
    to the host to validate it before the launch."""
    squeeze = label.dim() == 2
    lab = label.unsqueeze(0) if squeeze else label
    dev = _require_device(lab, seg, seg_off)
    if seg.dtype != torch.float32 or seg_off.dtype != torch.int32 or lab.dtype != torch.uint8:
        raise TypeError("seg float32, seg_off int32, label uint8")
    B, H, W = lab.shape
    if seg_off.numel() != B + 1 or seg.dim() != 2 or seg.shape[1] != 6:
        raise ValueError("seg must be n x 6 and seg_off hold B + 1 offsets")
    if check_offsets:  # one device-to-host copy of B + 1 integers
        so = seg_off.cpu()
        if int(so[0]) < 0 or bool((so[1:] < so[:-1]).any()) or int(so[-1]) > seg.shape[0]:
            raise ValueError("seg_off must be non-decreasing offsets into seg")
    if out is None:
        out = torch.empty((B, H, W, 2), dtype=torch.float32, device=dev)
    lib = load()
    rc = lib.gf_guide_field(B, H, W, _ptr(lab), _ptr(seg) if seg.numel() else None, _ptr(seg_off),
                            float(eta), float(3.0 * eta if cutoff is None else cutoff), _ptr(out),
                            _stream_ptr(dev))
    _check(rc, "gf_guide_field")
    return out[0] if squeeze else out


def fill(img: torch.Tensor, label: torch.Tensor, guide: torch.Tensor,
         params: Params | None = None, out: torch.Tensor | None = None, **kw) -> FillResult:
    """Fill one frame: img H x W x C, label H x W, guide H x W x 2."""
    if out is not None:
        out = out.unsqueeze(0)
    r = fill_batched(img.unsqueeze(0), label.unsqueeze(0), guide.unsqueeze(0), params, out=out, **kw)
    r.out = r.out[0]
    r.shell = r.shell[0]
    return r


def fill_backward(grad_out: torch.Tensor, fwd: FillResult, label: torch.Tensor,
                  guide: torch.Tensor, params: Params | None = None,
                  K: int | None = None, workspace: torch.Tensor | None = None, **kw):
    """dL/d img_in and dL/d guide of a completed fill (any engine).  Shapes
    B x H x W x C / B x H x W x 2.  K: shells to replay (default: taken from
    the shell map on the device).  Returns (grad_img, grad_guide)."""
    p = params or Params()
    if kw:
        p = Params(**{**p.__dict__, **kw})
    img_out = fwd.out
    if img_out.dim() == 3:
        img_out = img_out.unsqueeze(0)
    shell = fwd.shell if fwd.shell.dim() == 3 else fwd.shell.unsqueeze(0)
    if label.dim() == 2:
        label, guide, grad_out = label.unsqueeze(0), guide.unsqueeze(0), grad_out.unsqueeze(0)
    dev = _require_device(grad_out, img_out, label, guide, shell)
    if grad_out.dtype != torch.float32:
        raise TypeError("grad_out must be float32")
    B, H, W, C = img_out.shape
    lib = load()
    grad_img = torch.empty_like(grad_out)
    grad_guide = torch.empty((B, H, W, 2), dtype=torch.float32, device=dev)
    cp = p.c_struct()
    dt = _dtype_code(img_out)
    nbytes = lib.gf_backward_workspace_size(B, H, W, C, dt, ctypes.byref(cp))
    ws = workspace if workspace is not None else torch.zeros(max(nbytes, 256), dtype=torch.uint8, device=dev)
    rc = lib.gf_fill_backward(_ptr(grad_out), _ptr(img_out), B, H, W, C, dt, _ptr(label),
                              _ptr(guide), _ptr(shell), -1 if K is None else int(K), ctypes.byref(cp),
                              _ptr(grad_img), _ptr(grad_guide), _ptr(ws), ws.numel(), _stream_ptr(dev))
    _check(rc, "gf_fill_backward")
    return grad_img, grad_guide


class FillPlan:
    """Preallocated outputs and workspace for repeated fills of one shape:
    `run()` is a single call into the library (no allocation, no sync)."""

    def __init__(self, img: torch.Tensor, label: torch.Tensor, guide: torch.Tensor,
                 params: Params | None = None, inplace: bool = False, record_order: bool = False,
                 kcap: int | None = None):
        self.params = params or Params()
        if record_order and self.params.engine != ENGINE_FRONT:
            self.params = Params(**{**self.params.__dict__, "engine": ENGINE_FRONT})
        dev = _require_device(img, label, guide)
        if img.dim() == 3:
            img, label, guide = img.unsqueeze(0), label.unsqueeze(0), guide.unsqueeze(0)
        B, H, W, C = img.shape
        self.shape = (B, H, W, C)
        self.img, self.label, self.guide = img, label, guide
        self.out = img if inplace else torch.empty_like(img)
        self.shell = torch.empty((B, H, W), dtype=torch.int32, device=dev)
        self.stats = torch.empty(STAT_FRAME0 + STAT_PER_FRAME * B, dtype=torch.int32, device=dev)
        self.kcap = kcap or (min(H * W, 1 << 16) + 1)
        self.order = self.offsets = None
        if record_order:
            self.order = torch.empty(B * H * W, dtype=torch.int32, device=dev)
            self.offsets = torch.zeros(self.kcap, dtype=torch.int32, device=dev)
        self._cp = self.params.c_struct()
        self._dt = _dtype_code(img)
        lib = load()
        nbytes = lib.gf_workspace_size(B, H, W, C, self._dt, ctypes.byref(self._cp))
        self.ws = torch.zeros(max(nbytes, 256), dtype=torch.uint8, device=dev)
        self._lib = lib
        self._args = (_ptr(img), _ptr(self.out), B, H, W, C, self._dt, _ptr(label), _ptr(guide),
                      ctypes.byref(self._cp), _ptr(self.shell), _ptr(self.stats),
                      _ptr(self.order), _ptr(self.offsets), None, int(self.kcap),
                      _ptr(self.ws), self.ws.numel())
        self.device = dev

    def run(self, stream: torch.cuda.Stream | None = None):
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        rc = self._lib.gf_fill_batched(*self._args, ctypes.c_void_p(s.cuda_stream))
        if rc != 0:
            _check(rc, "gf_fill_batched")

    def result(self) -> FillResult:
        return FillResult(self.out, self.shell, self.stats, self.order, self.offsets, None)


class BackwardPlan:
    """Preallocated reverse-shell call for a FillPlan (any engine):
    grad_out -> (grad_img, grad_guide).  K: shells to replay (default: taken
    from the shell map on the device)."""

    def __init__(self, fwd: FillPlan, grad_out: torch.Tensor, grad_img: torch.Tensor,
                 grad_guide: torch.Tensor, K: int = -1):
        _require_device(grad_out, grad_img, grad_guide)
        B, H, W, C = fwd.shape
        lib = load()
        self._cp = fwd.params.c_struct()
        nbytes = lib.gf_backward_workspace_size(B, H, W, C, fwd._dt, ctypes.byref(self._cp))
        self.ws = torch.zeros(max(nbytes, 256), dtype=torch.uint8, device=fwd.device)
        self._lib = lib
        self._args = (_ptr(grad_out), _ptr(fwd.out), B, H, W, C, fwd._dt, _ptr(fwd.label),
                      _ptr(fwd.guide), _ptr(fwd.shell), int(K), ctypes.byref(self._cp),
                      _ptr(grad_img), _ptr(grad_guide), _ptr(self.ws), self.ws.numel())
        self.device = fwd.device

    def run(self, stream: torch.cuda.Stream | None = None):
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        rc = self._lib.gf_fill_backward(*self._args, ctypes.c_void_p(s.cuda_stream))
        if rc != 0:
            _check(rc, "gf_fill_backward")


class GuidefillFn(torch.autograd.Function):
    """u_out = fill(img, g = (cos theta, sin theta) on the hole); differentiable
    w.r.t. img (float32) and theta (float32, B x H x W).  The shell order is
    fixed by the forward and never altered by the backward."""

    @staticmethod
    def forward(ctx, img, theta, label, params: Params):
        g = torch.stack([torch.cos(theta), torch.sin(theta)], dim=-1)
        g = torch.where((label == 1).unsqueeze(-1), g, torch.zeros_like(g)).contiguous()
        r = fill_batched(img.contiguous(), label, g, params)
        ctx.save_for_backward(theta, label, g)
        ctx.fwd = r
        ctx.params = params
        ctx.mark_non_differentiable(r.shell)
        return r.out, r.shell

    @staticmethod
    def backward(ctx, grad_out, grad_shell):
        theta, label, g = ctx.saved_tensors
        gi, gg = fill_backward(grad_out.contiguous().float(), ctx.fwd, label, g, ctx.params)
        gtheta = -torch.sin(theta) * gg[..., 0] + torch.cos(theta) * gg[..., 1]
        return gi, gtheta, None, None
