"""FP64 CPU oracle of the Guidefill shell fill (arXiv 1611.05319).

TEST INFRASTRUCTURE ONLY: the reference the HIP path is checked against.
Only `tests/`, `__graft_entry__.smoke()` and the benchmark's `cpu_baseline`
leg may import this package; the product path never does.  It shares no code
with the HIP path (see `gf_oracle.c` for what is computed and the readings of
the paper it takes).

`fill` runs Algorithm 1 (Sec. 3) with the Guidefill neighbourhood (rotated
ball of ghost pixels, Sec. 3.1 and 3.3) or the coherence-transport lattice
ball, the weights of eqn:weight and onion or smart order (eqn:confidence,
eqn:ready).  `adjoint` is the reverse-mode derivative of that fill.
`guide_field` builds g from polyline splines (Sec. 3.2); `coherence_fill`
is the coherence-transport comparison mode, g re-estimated before every
shell from the modified structure tensor (eqn:modStructureTensor).
`tiny` holds an independent pure-Python transcription for small domains.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np
from dataclasses import dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gf_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libgforacle.so")
_lock = threading.Lock()
_lib = None

STORAGE = {"f64": 0, "f32": 1, "f16": 2}


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (no fused multiply-add, OpenMP)."""
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-shared", "-fPIC", _SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        lib.gfo_fill.argtypes = [ctypes.c_int] * 4 + [P, P, P, ctypes.c_double, ctypes.c_double,
                                                      ctypes.c_double, ctypes.c_double,
                                                      ctypes.c_int, ctypes.c_int,
                                                      ctypes.c_int, P, P, P, P, P, ctypes.c_int,
                                                      ctypes.c_int]
        lib.gfo_fill.restype = ctypes.c_int
        lib.gfo_guide_field.argtypes = [ctypes.c_int] * 3 + [P, P, P, ctypes.c_double,
                                                          ctypes.c_double, P]
        lib.gfo_guide_field.restype = ctypes.c_int
        lib.gfo_adjoint.argtypes = [ctypes.c_int] * 4 + [P, P, ctypes.c_double, ctypes.c_double,
                                                         ctypes.c_int, P, P, P, P, P]
        lib.gfo_adjoint.restype = ctypes.c_int
        lib.gfo_mod_structure_tensor.argtypes = [ctypes.c_int] * 3 + [P, P, P, ctypes.c_double,
                                                                      ctypes.c_double, P]
        lib.gfo_mod_structure_tensor.restype = ctypes.c_int
        lib.gfo_tensor_guide.argtypes = [P, ctypes.c_double, P]
        lib.gfo_tensor_guide.restype = None
        lib.gfo_coherence_guide.argtypes = [ctypes.c_int] * 4 + [P, P] + [ctypes.c_double] * 3 + [P]
        lib.gfo_coherence_guide.restype = ctypes.c_int
        lib.gfo_offsets.argtypes = [ctypes.c_double, P, P, ctypes.c_int]
        lib.gfo_offsets.restype = ctypes.c_int
        lib.gfo_round_f16.argtypes = [ctypes.c_double]
        lib.gfo_round_f16.restype = ctypes.c_double
        _lib = lib
        return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _as_batch(img, label, guide):
    img = np.asarray(img)
    label = np.asarray(label)
    guide = np.asarray(guide)
    squeeze = False
    if label.ndim == 2:
        img, label, guide = img[None], label[None], guide[None]
        squeeze = True
    if img.ndim == 3:
        raise ValueError("img must be H x W x C (or B x H x W x C)")
    return img, label, guide, squeeze


class Result:
    """Outputs of `fill`: colours (FP64), shell map (int32), per-frame stats,
    per-shell active-front and fill counts."""

    def __init__(self, u, s, stats, front_hist, fill_hist, squeeze):
        self.u = u[0] if squeeze else u
        self.shell = s[0] if squeeze else s
        self.stats = stats
        K = int(stats[:, 0].max()) if len(stats) else 0
        self.front_hist = front_hist[:, :K + 1]
        self.fill_hist = fill_hist[:, :K + 1]

    @property
    def K(self):
        return int(self.stats[0, 0]) if self.stats.shape[0] == 1 else self.stats[:, 0].copy()

    @property
    def n_filled(self):
        return int(self.stats[:, 1].sum())

    @property
    def n_unfilled(self):
        return int(self.stats[:, 2].sum())

    @property
    def max_front(self):
        return int(self.stats[:, 3].max())

    @property
    def n_ties(self):
        return int(self.stats[:, 5].sum())


def fill(img, label, guide, eps: float = 3.0, mu: float = 50.0, c: float = -1.0,
         ghost: bool = True, max_shells: int = 0, storage: str = "f64",
         threads: int | None = None, hist_cap: int = 4096, c2: float = -1.0) -> Result:
    """Run the FP64 oracle.  img: (B x) H x W x C; label: (B x) H x W uint8
    (0 readable, 1 inpaint, 2 bystander); guide: (B x) H x W x 2 (gx, gy).
    `c < 0` selects onion order; `c2 >= 0` adds eqn:ready2's data term
    |g| > c2; `storage` rounds stored values ('f32', 'f16')."""
    lib = _load()
    img, label, guide, squeeze = _as_batch(img, label, guide)
    B, H, W, C = img.shape
    u_in = np.ascontiguousarray(img, dtype=np.float64)
    lab = np.ascontiguousarray(label, dtype=np.uint8)
    g = np.ascontiguousarray(guide, dtype=np.float64)
    if lab.shape != (B, H, W) or g.shape != (B, H, W, 2):
        raise ValueError("shape mismatch")
    u = np.empty_like(u_in)
    s = np.empty((B, H, W), dtype=np.int32)
    stats = np.zeros((B, 8), dtype=np.int64)
    fh = np.zeros((B, hist_cap), dtype=np.int64)
    ph = np.zeros((B, hist_cap), dtype=np.int64)
    if threads is None:
        threads = int(os.environ.get("GFO_THREADS", os.cpu_count() or 1))
    rc = lib.gfo_fill(B, H, W, C, _ptr(u_in), _ptr(lab), _ptr(g), float(eps), float(mu), float(c),
                      float(c2), int(bool(ghost)), int(max_shells), STORAGE[storage], _ptr(u), _ptr(s),
                      _ptr(stats), _ptr(fh), _ptr(ph), hist_cap, int(threads))
    if rc != 0:
        raise ValueError(f"oracle fill failed with code {rc}")
    return Result(u, s, stats, fh, ph, squeeze)


def adjoint(label, guide, u_out, shell, grad_out, eps: float = 3.0, mu: float = 50.0,
            ghost: bool = True):
    """dL/du_in and dL/dg of the fill, given dL/du_out and the forward's
    outputs (colours and shell map).  Shapes as in `fill`."""
    lib = _load()
    label = np.asarray(label)
    squeeze = label.ndim == 2
    if squeeze:
        label, guide, u_out, shell, grad_out = (a[None] for a in
                                                (label, np.asarray(guide), np.asarray(u_out),
                                                 np.asarray(shell), np.asarray(grad_out)))
    B, H, W, C = u_out.shape
    lab = np.ascontiguousarray(label, dtype=np.uint8)
    g = np.ascontiguousarray(guide, dtype=np.float64)
    uo = np.ascontiguousarray(u_out, dtype=np.float64)
    s = np.ascontiguousarray(shell, dtype=np.int32)
    go = np.ascontiguousarray(grad_out, dtype=np.float64)
    gi = np.empty_like(go)
    gg = np.empty((B, H, W, 2), dtype=np.float64)
    rc = lib.gfo_adjoint(B, H, W, C, _ptr(lab), _ptr(g), float(eps), float(mu), int(bool(ghost)),
                         _ptr(uo), _ptr(s), _ptr(go), _ptr(gi), _ptr(gg))
    if rc != 0:
        raise ValueError(f"oracle adjoint failed with code {rc}")
    if squeeze:
        return gi[0], gg[0]
    return gi, gg


def guide_field(label, seg, seg_off, eta: float = 3.0, cutoff: float | None = None):
    """The guide field of Sec. 3.2 from polyline splines: label (B x) H x W;
    seg: n x 6 (x0, y0, x1, y1, gx, gy) per segment; seg_off: B + 1 offsets of
    each frame's segments; cutoff defaults to 3 eta.  Returns (B x) H x W x 2."""
    lib = _load()
    label = np.asarray(label)
    squeeze = label.ndim == 2
    lab = np.ascontiguousarray(label[None] if squeeze else label, dtype=np.uint8)
    B, H, W = lab.shape
    sg = np.ascontiguousarray(np.asarray(seg, dtype=np.float64).reshape(-1, 6))
    so = np.ascontiguousarray(np.asarray(seg_off, dtype=np.int32))
    if so.shape != (B + 1,) or so[-1] > sg.shape[0]:
        raise ValueError("seg_off must hold B + 1 offsets into seg")
    g = np.empty((B, H, W, 2), dtype=np.float64)
    rc = lib.gfo_guide_field(B, H, W, _ptr(lab), _ptr(sg), _ptr(so), float(eta),
                             float(3.0 * eta if cutoff is None else cutoff), _ptr(g))
    if rc != 0:
        raise ValueError(f"oracle guide field failed with code {rc}")
    return g[0] if squeeze else g


def mod_structure_tensor(u, known, sigma: float = 2.0, rho: float = 4.0):
    """The modified structure tensor of eqn:modStructureTensor over the known
    set `known` (H x W bool) of u (H x W x C): H x W x 3 (Jxx, Jxy, Jyy), NaN
    where no known pixel lies within the rho window."""
    lib = _load()
    u = np.asarray(u, dtype=np.float64)
    if u.ndim == 2:
        u = u[..., None]
    H, W, C = u.shape
    uu = np.ascontiguousarray(u)
    kn = np.ascontiguousarray(np.asarray(known, dtype=bool).astype(np.uint8))
    if kn.shape != (H, W):
        raise ValueError("known must be H x W")
    J = np.empty((H, W, 3), dtype=np.float64)
    rc = lib.gfo_mod_structure_tensor(H, W, C, _ptr(uu), _ptr(kn), None, float(sigma), float(rho),
                                      _ptr(J))
    if rc != 0:
        raise ValueError(f"oracle structure tensor failed with code {rc}")
    return J


def tensor_guide(J, Lambda: float = 1e-5):
    """tanh((l+ - l-) / Lambda) v- of each tensor in J (... x 3), sign fixed
    so that gx > 0 (or gx == 0 and gy > 0); 0 for NaN tensors."""
    lib = _load()
    J = np.asarray(J, dtype=np.float64)
    flat = np.ascontiguousarray(J.reshape(-1, 3))
    g = np.zeros((flat.shape[0], 2), dtype=np.float64)
    one = np.empty(2, dtype=np.float64)
    for e in range(flat.shape[0]):
        row = np.ascontiguousarray(flat[e])
        lib.gfo_tensor_guide(_ptr(row), float(Lambda), _ptr(one))
        g[e] = one
    return g.reshape(J.shape[:-1] + (2,))


def coherence_guide(u, label, sigma: float = 2.0, rho: float = 4.0, Lambda: float = 1e-5):
    """The comparison mode's guide for the current state: on every label-1
    pixel the coherence direction of the modified structure tensor over the
    label-0 pixels; 0 elsewhere.  u: (B x) H x W x C; label: (B x) H x W."""
    lib = _load()
    label = np.asarray(label)
    squeeze = label.ndim == 2
    lab = np.ascontiguousarray(label[None] if squeeze else label, dtype=np.uint8)
    uu = np.asarray(u, dtype=np.float64)
    uu = np.ascontiguousarray(uu[None] if squeeze else uu)
    B, H, W = lab.shape
    C = uu.shape[-1]
    if uu.shape != (B, H, W, C):
        raise ValueError("shape mismatch")
    g = np.empty((B, H, W, 2), dtype=np.float64)
    rc = lib.gfo_coherence_guide(B, H, W, C, _ptr(uu), _ptr(lab), float(sigma), float(rho),
                                 float(Lambda), _ptr(g))
    if rc != 0:
        raise ValueError(f"oracle coherence guide failed with code {rc}")
    return g[0] if squeeze else g


@dataclass
class CoherenceResult:
    u: np.ndarray        # B x H x W x C
    shell: np.ndarray    # B x H x W: -1 readable, -2 bystander, k filled at shell k, -3 never
    guide: np.ndarray    # B x H x W x 2: the guide each pixel was filled with (0 elsewhere)
    K: int               # shells that filled at least one pixel
    frame_K: list


def coherence_fill(img, label, eps: float = 3.0, mu: float = 50.0, sigma: float = 2.0,
                   rho: float = 4.0, Lambda: float = 1e-5, c: float = -1.0, ghost: bool = False,
                   max_shells: int = 0, storage: str = "f64", guide_f32: bool = False,
                   threads: int | None = None):
    """The coherence-transport comparison mode (Sec. 3.2): before every shell
    the guide of each inpaint pixel is re-estimated from the modified
    structure tensor of the current known set, then one shell of Algorithm 1
    runs with it (lattice ball by default).  `guide_f32` rounds each guide to
    binary32 before the fill uses it (the fill's guide input type).
    Returns a CoherenceResult."""
    img = np.asarray(img)
    label = np.asarray(label)
    squeeze = label.ndim == 2
    u = np.array(img[None] if squeeze else img, dtype=np.float64)
    lab = np.array(label[None] if squeeze else label, dtype=np.uint8)
    B, H, W = lab.shape
    shell = np.where(lab == 0, -1, np.where(lab == 2, -2, -3)).astype(np.int32)
    used = np.zeros((B, H, W, 2), dtype=np.float64)
    frame_K = [0] * B
    k = 0
    while max_shells <= 0 or k < max_shells:
        if not (lab == 1).any():
            break
        g = coherence_guide(u, lab, sigma, rho, Lambda)
        if guide_f32:
            g = g.astype(np.float32).astype(np.float64)
        r = fill(u, lab, g, eps=eps, mu=mu, c=c, ghost=ghost, max_shells=1, storage=storage,
                 threads=threads)
        rs = r.shell if r.shell.ndim == 3 else r.shell[None]
        new = (lab == 1) & (rs == 0)
        if not new.any():
            break
        ru = r.u if r.u.ndim == 4 else r.u[None]
        u = np.array(ru)
        shell[new] = k
        used[new] = g[new]
        lab[new] = 0
        for f in range(B):
            if new[f].any():
                frame_K[f] += 1
        k += 1
    res = CoherenceResult(u, shell, used, k, frame_K)
    if squeeze:
        res = CoherenceResult(u[0], shell[0], used[0], k, frame_K)
    return res


def offsets(eps: float):
    """The lattice ball {(n, m): 0 < n^2 + m^2 <= eps^2}, m ascending then n."""
    lib = _load()
    on = np.zeros(4096, dtype=np.int32)
    om = np.zeros(4096, dtype=np.int32)
    T = lib.gfo_offsets(float(eps), _ptr(on), _ptr(om), 4096)
    return list(zip(on[:T].tolist(), om[:T].tolist()))


def round_f16(v: float) -> float:
    return float(_load().gfo_round_f16(float(v)))
