"""FP64 CPU oracle for the recursive multidimensional prediction-error filter.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the GPU library (``paper_1408_3526_amd``) and never imports it.

Two independent routes to the same quantities live here:

* ``liborc.so`` (``rmdf_oracle.c``): the recursive pipeline in the paper's
  order -- row and column sliding DFTs, the temporal deadbeat observer
  (Sec. 1, eq. 6-7), the flow part (Sec. 2, eq. 9-10) and the velocity-tuned
  filter (eq. 4, 8) -- in double precision.
* ``brute.py``: the plain definitions (eq. 1, 2, 5, 6, 10) evaluated directly
  on one window at a time, used to pin the recursive route.

``pixel_series`` combines the direct window spectrum with the library's flow
and filter steps, so single pixels of full-size frames can be checked without
running the whole frame.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rmdf_oracle.c")
_SO = os.path.join(_HERE, "liborc.so")
_LIB = None


def build(force: bool = True) -> str:
    """Compile liborc.so with gcc (-O2, OpenMP).  Returns the path."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-shared", "-fPIC",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < max(os.path.getmtime(_SRC), os.path.getmtime(
                os.path.join(_HERE, "rmdf_oracle.h"))):
            build(force=True)
        L = ctypes.CDLL(_SO)
        dp = ctypes.POINTER(ctypes.c_double)
        L.orc_dirichlet.restype = ctypes.c_double
        L.orc_dirichlet.argtypes = [ctypes.c_int, ctypes.c_double]
        L.orc_coeffs.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_double, ctypes.c_void_p]
        L.orc_observer_series.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_void_p]
        L.orc_flow_R.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                 ctypes.c_void_p]
        L.orc_background.restype = ctypes.c_double
        L.orc_background.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.orc_run.restype = ctypes.c_int
        L.orc_run.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p] + [ctypes.c_void_p] * 9
        L.orc_threads.restype = ctypes.c_int
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_set_threads.restype = None
        L.orc_peak_vertex.restype = ctypes.c_double
        L.orc_peak_vertex.argtypes = [ctypes.c_double] * 6
        L.orc_refine.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
        _LIB = L
        del dp
    return _LIB


class _CCfg(ctypes.Structure):
    _fields_ = [("H", ctypes.c_int), ("W", ctypes.c_int),
                ("Mx", ctypes.c_int), ("My", ctypes.c_int), ("Mz", ctypes.c_int),
                ("Bx", ctypes.c_int), ("By", ctypes.c_int),
                ("dx", ctypes.c_int), ("dy", ctypes.c_int), ("dt", ctypes.c_int),
                ("alpha", ctypes.c_double),
                ("nvx", ctypes.c_int), ("nvy", ctypes.c_int),
                ("gx", ctypes.c_void_p), ("gy", ctypes.c_void_p),
                ("vmode", ctypes.c_int), ("fvx", ctypes.c_double), ("fvy", ctypes.c_double)]


@dataclass
class Cfg:
    """Oracle configuration.  Mx, My, Mz are window lengths (DFT sizes)."""
    H: int
    W: int
    Mx: int
    My: int
    Mz: int
    gx: np.ndarray
    gy: np.ndarray
    Bx: int | None = None
    By: int | None = None
    dx: int | None = None
    dy: int | None = None
    dt: int | None = None
    alpha: float = float(np.exp(-0.1))
    vmode: int = 0
    fvx: float = 0.0
    fvy: float = 0.0
    _keep: list = field(default_factory=list, repr=False)

    def __post_init__(self):
        # Defaults (readings of Sec. 3 for window lengths the paper does not
        # list): B = floor(3M/8), m' = floor(M/2).  For M = 9 these give the
        # paper's B = 3 and m' = K = 4.  Parity unpinned: they are parameter
        # choices, and every pin passes B and m' explicitly or holds for any.
        if self.Bx is None:
            self.Bx = (3 * self.Mx) // 8
        if self.By is None:
            self.By = (3 * self.My) // 8
        if self.dx is None:
            self.dx = self.Mx // 2
        if self.dy is None:
            self.dy = self.My // 2
        if self.dt is None:
            self.dt = self.Mz // 2
        self.gx = np.ascontiguousarray(self.gx, dtype=np.float64)
        self.gy = np.ascontiguousarray(self.gy, dtype=np.float64)

    @property
    def nv(self) -> int:
        return len(self.gx) * len(self.gy)

    @property
    def N(self) -> int:
        return self.Mx * self.My * self.Mz

    def c(self) -> _CCfg:
        s = _CCfg(self.H, self.W, self.Mx, self.My, self.Mz, self.Bx, self.By,
                  self.dx, self.dy, self.dt, float(self.alpha), len(self.gx), len(self.gy),
                  self.gx.ctypes.data, self.gy.ctypes.data, int(self.vmode),
                  float(self.fvx), float(self.fvy))
        self._keep = [s, self.gx, self.gy]
        return s


def _p(a):
    return None if a is None else a.ctypes.data


def dirichlet(W: int, w: float) -> float:
    """Eq. (3)."""
    return lib().orc_dirichlet(int(W), float(w))


def peak_vertex(x0, r0, x1, r1, x2, r2) -> float:
    """Vertex of the parabola through three points (velocity mode 3)."""
    return lib().orc_peak_vertex(*(float(v) for v in (x0, r0, x1, r1, x2, r2)))


def refine(cfg: Cfg, rsp: np.ndarray, best: int) -> tuple:
    """Sub-grid velocity from the smoothed R of one anchor (velocity mode 3)."""
    rsp = np.ascontiguousarray(rsp, np.float64)
    vx, vy = ctypes.c_double(), ctypes.c_double()
    c = cfg.c()
    lib().orc_refine(ctypes.byref(c), rsp.ctypes.data, int(best), ctypes.byref(vx), ctypes.byref(vy))
    return vx.value, vy.value


def coeffs(cfg: Cfg, vx: float, vy: float) -> np.ndarray:
    """Eq. (8) at the DFT bins; array [Mx, My, Mz] complex."""
    out = np.zeros((cfg.Mx, cfg.My, cfg.Mz), np.complex128)
    c = cfg.c()
    lib().orc_coeffs(ctypes.byref(c), float(vx), float(vy), out.ctypes.data)
    return out


def observer_series(Mz: int, s2: np.ndarray, a0: np.ndarray | None = None) -> np.ndarray:
    """Temporal deadbeat observer on one bin's input series; returns [T, Mz]."""
    s2 = np.ascontiguousarray(s2, np.complex128)
    T = s2.shape[0]
    out = np.zeros((T, Mz), np.complex128)
    a0c = None if a0 is None else np.ascontiguousarray(a0, np.complex128)
    lib().orc_observer_series(int(Mz), int(T), s2.ctypes.data, _p(a0c), out.ctypes.data)
    return out


def flow_R(cfg: Cfg, S: np.ndarray, want_P: bool = False):
    """Eq. (9)-(10) (+ high-pass, Hann) for spectra S[..., Mx, My, Mz]."""
    S = np.ascontiguousarray(S, np.complex128)
    lead = S.shape[:-3]
    n = int(np.prod(lead)) if lead else 1
    R = np.zeros(lead + (cfg.nv,), np.float64)
    P = np.zeros(lead + (cfg.Mx, cfg.My, cfg.Mz), np.float64) if want_P else None
    c = cfg.c()
    lib().orc_flow_R(ctypes.byref(c), n, S.ctypes.data, R.ctypes.data, _p(P))
    return (R, P) if want_P else R


def background(cfg: Cfg, Hk: np.ndarray, S: np.ndarray) -> float:
    """Eq. (4)."""
    Hk = np.ascontiguousarray(Hk, np.complex128)
    S = np.ascontiguousarray(S, np.complex128)
    c = cfg.c()
    return lib().orc_background(ctypes.byref(c), Hk.ctypes.data, S.ctypes.data)


def run(cfg: Cfg, frames: np.ndarray, want_r: bool = False, want_rs: bool = False,
        want_spec: bool = False) -> dict:
    """Whole recursive pipeline over frames [T, H, W] (float32)."""
    frames = np.ascontiguousarray(frames, np.float32)
    T, H, W = frames.shape
    assert (H, W) == (cfg.H, cfg.W)
    HW = H * W
    out = np.zeros((T, H, W), np.float64)
    vxy = np.zeros((T, H, W, 2), np.float64)
    idx = np.zeros((T, H, W), np.int32)
    rs_last = np.zeros((H, W, cfg.nv), np.float64)
    r_all = np.zeros((T, H, W, cfg.nv), np.float64) if want_r else None
    rs_all = np.zeros((T, H, W, cfg.nv), np.float64) if want_rs else None
    en_all = np.zeros((T, H, W), np.float64) if want_rs else None
    spec = np.zeros((H, W, cfg.Mx, cfg.My, cfg.Mz), np.complex128) if want_spec else None
    nbad = ctypes.c_longlong(0)
    c = cfg.c()
    rc = lib().orc_run(ctypes.byref(c), T, frames.ctypes.data, out.ctypes.data, vxy.ctypes.data,
                       idx.ctypes.data, rs_last.ctypes.data, _p(r_all), _p(rs_all), _p(en_all), _p(spec),
                       ctypes.addressof(nbad))
    if rc != 0:
        raise ValueError("orc_run failed with code %d" % rc)
    del HW
    return {"out": out, "vxy": vxy, "idx": idx, "rs_last": rs_last, "r_all": r_all,
            "rs_all": rs_all, "en_all": en_all, "spec": spec, "n_nonfinite": nbad.value}


def pixel_series(cfg: Cfg, frames: np.ndarray, x: int, y: int, T: int | None = None) -> dict:
    """Oracle outputs at one anchor (x, y) for frames 0..T-1, from the direct
    window DFT (eq. 6) instead of the recursion: instantaneous and smoothed R,
    velocity index, velocity, background estimate and output per frame."""
    from . import brute
    frames = np.asarray(frames)
    if T is None:
        T = frames.shape[0]
    clean = np.where(np.isfinite(frames[:T]), frames[:T], 0.0).astype(np.float64)
    S = np.stack([brute.spectrum(clean, x, y, t, (cfg.Mx, cfg.My, cfg.Mz)) for t in range(T)])
    R, P = flow_R(cfg, S, want_P=True)
    rs = np.zeros_like(R)
    en = np.zeros(T)
    acc = np.zeros(cfg.nv)
    eacc = 0.0
    for t in range(T):
        acc = (1.0 - cfg.alpha) * R[t] + cfg.alpha * acc
        eacc = (1.0 - cfg.alpha) * P[t].sum() + cfg.alpha * eacc
        rs[t] = acc
        en[t] = eacc
    idx = np.argmax(rs, axis=1).astype(np.int32)        # first maximum
    nvx = len(cfg.gx)
    cache = {}
    ihat = np.zeros(T)
    out = np.zeros(T)
    vxy = np.zeros((T, 2))
    for t in range(T):
        if cfg.vmode == 2:
            key = (cfg.fvx, cfg.fvy)
            idx[t] = -1
        elif cfg.vmode == 3:
            key = refine(cfg, rs[t], idx[t])
        else:
            key = (cfg.gx[idx[t] % nvx], cfg.gy[idx[t] // nvx])
        if key not in cache:
            cache[key] = coeffs(cfg, *key)
        vxy[t] = key
        ihat[t] = background(cfg, cache[key], S[t])
        ts, xs, ys = t - cfg.dt, x - cfg.dx, y - cfg.dy
        ides = clean[ts, ys, xs] if (ts >= 0 and xs >= 0 and ys >= 0) else 0.0
        out[t] = ides - ihat[t]
    return {"S": S, "R": R, "rs": rs, "en": en, "idx": idx, "vxy": vxy, "ihat": ihat, "out": out}


def threads() -> int:
    return lib().orc_threads()


def set_threads(n: int) -> None:
    """Thread count of the oracle's OpenMP loops (timing runs only)."""
    lib().orc_set_threads(int(n))
