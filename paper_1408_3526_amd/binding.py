"""ctypes binding of librmdf.so (C ABI in include/rmdf.h).

Argument marshalling only: every step of the filter runs in the HIP library.
Device buffers are torch tensors on a HIP device (their ``data_ptr()`` is
passed through); torch supplies memory and streams and nothing else.  There is
no CPU fallback: if librmdf.so is missing, ``lib()`` raises.

The module-level functions carry the C names; ``Filter`` wraps a context.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SO_PATH = os.path.join(_HERE, "librmdf.so")
_LIB = None

RMDF_OK, RMDF_E_INVAL, RMDF_E_NOMEM, RMDF_E_DEVICE, RMDF_E_STATE, RMDF_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5
VEL_SEARCH, VEL_LEARNED, VEL_FIXED, VEL_REFINED = 0, 1, 2, 3
TEMPORAL_OBSERVER, TEMPORAL_RING, TEMPORAL_DIRECT = 0, 1, 2

_STATUS = {0: "RMDF_OK", -1: "RMDF_E_INVAL", -2: "RMDF_E_NOMEM", -3: "RMDF_E_DEVICE",
           -4: "RMDF_E_STATE", -5: "RMDF_E_UNSUPPORTED"}


class RmdfError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (_STATUS.get(status, str(status)), msg))
        self.status = status


class rmdf_params(ctypes.Structure):
    _fields_ = [("Bx", ctypes.c_int), ("By", ctypes.c_int),
                ("delay_x", ctypes.c_int), ("delay_y", ctypes.c_int), ("delay_t", ctypes.c_int),
                ("alpha", ctypes.c_float), ("velocity_mode", ctypes.c_int),
                ("fixed_vx", ctypes.c_float), ("fixed_vy", ctypes.c_float),
                ("conf_threshold", ctypes.c_float), ("tile_rows", ctypes.c_int),
                ("kernel_variant", ctypes.c_int), ("write_features", ctypes.c_int), ("temporal", ctypes.c_int)]


# rmdf_spectrum_noalloc: most anchors per call (include/rmdf.h)
SPECTRUM_NOALLOC_MAX = 65536

# C signatures: name -> (restype, argtypes)
_VP, _I, _LL, _D, _SZ = ctypes.c_void_p, ctypes.c_int, ctypes.c_longlong, ctypes.c_double, ctypes.c_size_t
_SIGS = {
    "rmdf_params_default": (None, [ctypes.POINTER(rmdf_params)]),
    "rmdf_create": (_I, [_I, _I, _I, _I, _I, _VP, _I, _VP, _I, ctypes.POINTER(rmdf_params), _VP,
                         ctypes.POINTER(_VP)]),
    "rmdf_push_frame": (_I, [_VP, _VP]),
    "rmdf_push_frames": (_I, [_VP, _I, _VP, _VP]),
    "rmdf_velocity": (_I, [_VP, _VP, _VP]),
    "rmdf_output": (_I, [_VP, _VP]),
    "rmdf_frames_pushed": (_I, [_VP, ctypes.POINTER(_LL)]),
    "rmdf_nonfinite_count": (_I, [_VP, ctypes.POINTER(_LL)]),
    "rmdf_spectrum": (_I, [_VP, _I, _VP, _VP, _VP]),
    "rmdf_spectrum_noalloc": (_I, [_VP, _I, _VP, _VP, _VP]),
    "rmdf_smoothed_r": (_I, [_VP, _VP]),
    "rmdf_set_timing": (_I, [_VP, _I]),
    "rmdf_kernel_time": (_I, [_VP, _I, ctypes.POINTER(_D), ctypes.POINTER(_LL)]),
    "rmdf_device_bytes": (_I, [_VP, ctypes.POINTER(_SZ)]),
    "rmdf_state_bytes": (_I, [_VP, ctypes.POINTER(_SZ)]),
    "rmdf_save_state": (_I, [_VP, _VP, _SZ]),
    "rmdf_load_state": (_I, [_VP, _VP, _SZ]),
    "rmdf_kernel_variant": (_I, [_VP, ctypes.POINTER(_I)]),
    "rmdf_coeff_lattice": (_I, [_VP, ctypes.POINTER(_I)]),
    "rmdf_tile_rows": (_I, [_VP, ctypes.POINTER(_I)]),
    "rmdf_cfar": (_I, [_VP, _I, _I, _I, _I, ctypes.c_float, _VP, _VP, _VP]),
    "rmdf_hbm_probe": (_I, [_I, _VP, _VP, _SZ, _I, _I, _VP]),
    "rmdf_destroy": (_I, [_VP]),
    "rmdf_last_error": (ctypes.c_char_p, [_VP]),
    "rmdf_mlp_set_weights": (_I, [_VP, _VP, _SZ]),
    "rmdf_features": (_I, [_VP, _VP]),
    "rmdf_learned_output": (_I, [_VP, _VP]),
    "rmdf_learned_network": (_I, [_VP, _VP, _I, _VP]),
    "rmdf_mlp_gemm_nt": (_I, [_VP, _I, _VP, _I, _I, _I, _I, _VP, _I, _VP, _I, _VP, _VP, _I, _VP]),
    "rmdf_mlp_transpose": (_I, [_VP, _VP, _I, _I, _VP, _VP]),
    "rmdf_mlp_head": (_I, [_VP, _VP, _VP, _VP, _I, ctypes.c_float, ctypes.c_float, _VP, _VP, _VP, _VP, _VP]),
    "rmdf_mlp_colsum": (_I, [_VP, _I, _I, _VP, _VP]),
    "rmdf_mlp_infer_head": (_I, [_VP, _VP, _VP, _I, _VP, _VP]),
    "rmdf_mlp_adam": (_I, [_VP, _VP, _VP, _VP, _VP, _I, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                           ctypes.c_float, _I, _VP]),
    "rmdf_mlp_to_bf16": (_I, [_VP, _VP, ctypes.c_longlong, _VP]),
    "rmdf_batch_create": (_I, [_I, _VP, ctypes.POINTER(rmdf_params), _VP, ctypes.POINTER(_VP)]),
    "rmdf_batch_input": (_I, [_VP, _I, ctypes.POINTER(_VP)]),
    "rmdf_batch_launch": (_I, [_VP]),
    "rmdf_batch_push": (_I, [_VP, _VP]),
    "rmdf_batch_output": (_I, [_VP, _I, _VP, _VP, _VP]),
    "rmdf_batch_stream_ctx": (_I, [_VP, _I, ctypes.POINTER(_VP)]),
    "rmdf_batch_set_tiles": (_I, [_VP, _I, _I]),
    "rmdf_batch_set_schedule": (_I, [_VP, _I]),
    "rmdf_batch_autotune": (_I, [_VP, _I, ctypes.c_char_p, _SZ]),
    "rmdf_batch_set_timing": (_I, [_VP, _I]),
    "rmdf_batch_latency": (_I, [_VP, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float),
                                ctypes.POINTER(ctypes.c_float), ctypes.POINTER(_LL)]),
    "rmdf_batch_destroy": (_I, [_VP]),
    "rmdf_batch_last_error": (ctypes.c_char_p, [_VP]),
}


class rmdf_stream_desc(ctypes.Structure):
    _fields_ = [("H", ctypes.c_int), ("W", ctypes.c_int), ("Kx", ctypes.c_int), ("Ky", ctypes.c_int),
                ("Kt", ctypes.c_int), ("vgrid_x", ctypes.c_void_p), ("vgrid_y", ctypes.c_void_p),
                ("nvx", ctypes.c_int), ("nvy", ctypes.c_int)]


def lib():
    """Load librmdf.so (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(SO_PATH):
            raise RuntimeError("librmdf.so is not built (run __graft_entry__.build() or "
                               "python paper_1408_3526_amd/build.py); there is no fallback")
        L = ctypes.CDLL(SO_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _LIB = L
    return _LIB


def exported_names():
    return list(_SIGS)


def _check(status: int, ctx=None):
    if status != RMDF_OK:
        msg = lib().rmdf_last_error(ctx)
        raise RmdfError(status, msg.decode() if msg else "")


def _bcheck(status: int, b=None):
    if status != RMDF_OK:
        msg = lib().rmdf_batch_last_error(b)
        raise RmdfError(status, msg.decode() if msg else "")


def _dev_ptr(t, dtype=None, numel=None, name="tensor"):
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a HIP device tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if dtype is not None and t.dtype != dtype:
        raise TypeError("%s must have dtype %s" % (name, dtype))
    if numel is not None and t.numel() != numel:
        raise ValueError("%s must have %d elements, has %d" % (name, numel, t.numel()))
    return t.data_ptr()


def _buf_ptr(buf, writable):
    """Address and size in bytes of a contiguous byte buffer: a CUDA tensor or
    a numpy array in host memory."""
    import torch
    if isinstance(buf, torch.Tensor):
        if not buf.is_cuda:
            raise TypeError("state buffer tensors must be on the HIP device (use a numpy array for host memory)")
        if not buf.is_contiguous():
            raise ValueError("state buffer must be contiguous")
        return buf.data_ptr(), buf.numel() * buf.element_size()
    if isinstance(buf, np.ndarray):
        if not buf.flags["C_CONTIGUOUS"] or (writable and not buf.flags["WRITEABLE"]):
            raise ValueError("state buffer must be a contiguous%s numpy array" % (" writable" if writable else ""))
        return buf.ctypes.data, buf.nbytes
    raise TypeError("state buffer must be a CUDA tensor or a numpy array")


# ---- C-named functions -------------------------------------------------------

def rmdf_params_default() -> rmdf_params:
    p = rmdf_params()
    lib().rmdf_params_default(ctypes.byref(p))
    return p


def rmdf_create(H, W, Kx, Ky, Kt, vgrid_x, vgrid_y, params: rmdf_params | None = None, stream=None):
    gx = np.ascontiguousarray(vgrid_x, np.float32)
    gy = np.ascontiguousarray(vgrid_y, np.float32)
    ctx = _VP()
    s = None if stream is None else ctypes.c_void_p(int(stream))
    st = lib().rmdf_create(int(H), int(W), int(Kx), int(Ky), int(Kt), gx.ctypes.data, len(gx),
                           gy.ctypes.data, len(gy), None if params is None else ctypes.byref(params), s,
                           ctypes.byref(ctx))
    _check(st, None)
    return ctx


def rmdf_push_frame(ctx, frame_ptr: int):
    _check(lib().rmdf_push_frame(ctx, frame_ptr), ctx)


def rmdf_velocity(ctx, vxy_ptr, idx_ptr):
    _check(lib().rmdf_velocity(ctx, vxy_ptr, idx_ptr), ctx)


def rmdf_output(ctx, out_ptr):
    _check(lib().rmdf_output(ctx, out_ptr), ctx)


def rmdf_destroy(ctx):
    lib().rmdf_destroy(ctx)


# ---- convenience wrapper -----------------------------------------------------

class Filter:
    """One filter context.  Every call is enqueued on the torch stream that was
    current when the Filter was created (or on ``stream``, a raw hipStream_t
    handle); tensors passed in and returned belong to that stream."""

    def __init__(self, H, W, Kx, Ky, Kt, vgrid_x, vgrid_y, *, Bx=-1, By=-1, delay=(-1, -1, -1),
                 alpha=-1.0, velocity_mode=VEL_SEARCH, fixed_v=(0.0, 0.0), conf_threshold=0.9,
                 tile_rows=0, kernel_variant=0, write_features=False, temporal=TEMPORAL_OBSERVER, stream=None,
                 use_torch_stream=True):
        import torch
        p = rmdf_params_default()
        p.Bx, p.By = int(Bx), int(By)
        p.delay_x, p.delay_y, p.delay_t = (int(v) for v in delay)
        p.alpha = float(alpha)
        p.velocity_mode = int(velocity_mode)
        p.fixed_vx, p.fixed_vy = (float(v) for v in fixed_v)
        p.conf_threshold = float(conf_threshold)
        p.tile_rows = int(tile_rows)
        p.kernel_variant = int(kernel_variant)
        p.write_features = int(bool(write_features))
        p.temporal = int(temporal)
        if stream is None and use_torch_stream:
            stream = torch.cuda.current_stream().cuda_stream
        self.H, self.W, self.M = int(H), int(W), (int(Kx), int(Ky), int(Kt))
        self.nvx, self.nvy = len(vgrid_x), len(vgrid_y)
        self.nv = self.nvx * self.nvy
        self.gx = np.asarray(vgrid_x, np.float32)
        self.gy = np.asarray(vgrid_y, np.float32)
        self.ctx = rmdf_create(H, W, Kx, Ky, Kt, vgrid_x, vgrid_y, p, stream)

    def push_frame(self, frame):
        import torch
        rmdf_push_frame(self.ctx, _dev_ptr(frame, torch.float32, self.H * self.W, "frame"))

    def push_frames(self, frames, outs=None):
        """rmdf_push_frames: push frames in order (a list of [H, W] float32
        CUDA tensors); pairs go through one pass of the per-pixel kernel where
        the context allows it.  outs: None, or a list of the same length whose
        entries are None or [H, W] float32 CUDA tensors that receive each
        frame's output."""
        import torch
        n = len(frames)
        fp = (ctypes.c_void_p * n)(*[_dev_ptr(f, torch.float32, self.H * self.W, "frame") for f in frames])
        op = None
        if outs is not None:
            if len(outs) != n:
                raise ValueError("outs must have one entry per frame")
            op = (ctypes.c_void_p * n)(*[None if o is None else _dev_ptr(o, torch.float32, self.H * self.W, "out")
                                         for o in outs])
        _check(lib().rmdf_push_frames(self.ctx, n, fp, op), self.ctx)

    def output(self, out=None):
        import torch
        if out is None:
            out = torch.empty((self.H, self.W), dtype=torch.float32, device="cuda")
        rmdf_output(self.ctx, _dev_ptr(out, torch.float32, self.H * self.W, "out"))
        return out

    def velocity(self, vxy=None, idx=None):
        import torch
        if vxy is None:
            vxy = torch.empty((self.H, self.W, 2), dtype=torch.float32, device="cuda")
        if idx is None:
            idx = torch.empty((self.H, self.W), dtype=torch.int32, device="cuda")
        rmdf_velocity(self.ctx, _dev_ptr(vxy, torch.float32, 2 * self.H * self.W, "vxy"),
                      _dev_ptr(idx, torch.int32, self.H * self.W, "idx"))
        return vxy, idx

    def spectrum(self, xs, ys):
        import torch
        xs = np.ascontiguousarray(xs, np.int32)
        ys = np.ascontiguousarray(ys, np.int32)
        n = len(xs)
        Mx, My, Mz = self.M
        out = torch.empty((n, Mx, My, Mz, 2), dtype=torch.float32, device="cuda")
        _check(lib().rmdf_spectrum(self.ctx, n, xs.ctypes.data, ys.ctypes.data, out.data_ptr()), self.ctx)
        return torch.view_as_complex(out)

    def spectrum_noalloc(self, xs, ys, out=None):
        """rmdf_spectrum_noalloc: the same result without any device allocation
        inside the library (out: a caller buffer [n, Mx, My, Mz, 2] FP32)."""
        import torch
        xs = np.ascontiguousarray(xs, np.int32)
        ys = np.ascontiguousarray(ys, np.int32)
        n = len(xs)
        Mx, My, Mz = self.M
        if out is None:
            out = torch.empty((n, Mx, My, Mz, 2), dtype=torch.float32, device="cuda")
        ptr = _dev_ptr(out, torch.float32, n * Mx * My * Mz * 2, "out")
        _check(lib().rmdf_spectrum_noalloc(self.ctx, n, xs.ctypes.data, ys.ctypes.data, ptr), self.ctx)
        return torch.view_as_complex(out)

    def smoothed_r(self):
        import torch
        out = torch.empty((self.H, self.W, self.nv), dtype=torch.float32, device="cuda")
        _check(lib().rmdf_smoothed_r(self.ctx, out.data_ptr()), self.ctx)
        return out

    def set_timing(self, on: bool = True, kernels=None):
        """Per-kernel HIP-event timing: all kernels (on), none, or only those
        listed in kernels (0 pixel, 1 row, 2 ingest, 3 network, 4 finish)."""
        mask = (-1 if on else 0) if kernels is None else sum(1 << int(k) for k in kernels)
        _check(lib().rmdf_set_timing(self.ctx, int(mask)), self.ctx)

    def kernel_time(self, which: int):
        ms, n = ctypes.c_double(), ctypes.c_longlong()
        _check(lib().rmdf_kernel_time(self.ctx, int(which), ctypes.byref(ms), ctypes.byref(n)), self.ctx)
        return ms.value, n.value

    def set_weights(self, blob):
        """Learned-mode weights: FP32 array W1 (128x1152), b1, W2 (64x128), b2,
        W3 (3x64), b3 (see rmdf_mlp_set_weights)."""
        w = np.ascontiguousarray(blob, np.float32)
        _check(lib().rmdf_mlp_set_weights(self.ctx, w.ctypes.data, w.nbytes), self.ctx)

    def features(self):
        """Learned-model input features of the latest frame, [H, W, 1152] BF16
        (returned as a torch.bfloat16 tensor)."""
        import torch
        out = torch.empty((self.H, self.W, 1152), dtype=torch.bfloat16, device="cuda")
        _check(lib().rmdf_features(self.ctx, out.data_ptr()), self.ctx)
        return out

    def learned_output(self):
        import torch
        out = torch.empty((self.H, self.W, 3), dtype=torch.float32, device="cuda")
        _check(lib().rmdf_learned_output(self.ctx, out.data_ptr()), self.ctx)
        return out

    def learned_network(self, feat):
        """rmdf_learned_network: the context's network on caller features
        (torch BF16 [n, 1152] on the GPU); returns [n, 3] (vx, vy, confidence)."""
        import torch
        n = feat.shape[0]
        ptr = _dev_ptr(feat, torch.bfloat16, n * 1152, "feat")
        out = torch.empty((n, 3), dtype=torch.float32, device="cuda")
        _check(lib().rmdf_learned_network(self.ctx, ptr, n, out.data_ptr()), self.ctx)
        return out

    def kernel_name(self) -> str:
        """Name of the per-pixel kernel this context launches."""
        v = ctypes.c_int()
        _check(lib().rmdf_kernel_variant(self.ctx, ctypes.byref(v)), self.ctx)
        Mx, My, Mz = self.M
        return "k_pixel16" if v.value == 2 else "k_pixel<%d,%d,%d>" % (Mx, My, Mz)

    def tile_rows(self) -> int:
        """Rows per work tile of the pixel kernel (after the automatic choice)."""
        v = ctypes.c_int()
        _check(lib().rmdf_tile_rows(self.ctx, ctypes.byref(v)), self.ctx)
        return v.value

    def coeff_lattice(self) -> int:
        """16 s when the background coefficients use the lattice table (grid
        step 1/s px/frame), else 0."""
        q = ctypes.c_int()
        _check(lib().rmdf_coeff_lattice(self.ctx, ctypes.byref(q)), self.ctx)
        return q.value

    def frames_pushed(self) -> int:
        n = ctypes.c_longlong()
        _check(lib().rmdf_frames_pushed(self.ctx, ctypes.byref(n)), self.ctx)
        return n.value

    def nonfinite_count(self) -> int:
        n = ctypes.c_longlong()
        _check(lib().rmdf_nonfinite_count(self.ctx, ctypes.byref(n)), self.ctx)
        return n.value

    def device_bytes(self) -> int:
        n = ctypes.c_size_t()
        _check(lib().rmdf_device_bytes(self.ctx, ctypes.byref(n)), self.ctx)
        return n.value

    def state_bytes(self) -> int:
        n = ctypes.c_size_t()
        _check(lib().rmdf_state_bytes(self.ctx, ctypes.byref(n)), self.ctx)
        return n.value

    def save_state(self, buf=None):
        """rmdf_save_state into buf (a uint8 CUDA tensor or a writable uint8
        numpy array of at least state_bytes() bytes; None: a new CUDA tensor),
        which is returned."""
        import torch
        n = self.state_bytes()
        if buf is None:
            buf = torch.empty(n, dtype=torch.uint8, device="cuda")
        ptr, size = _buf_ptr(buf, writable=True)
        _check(lib().rmdf_save_state(self.ctx, ptr, size), self.ctx)
        return buf

    def load_state(self, buf):
        """rmdf_load_state from a buffer written by save_state (CUDA tensor or
        numpy array)."""
        ptr, size = _buf_ptr(buf, writable=False)
        _check(lib().rmdf_load_state(self.ctx, ptr, size), self.ctx)

    def close(self):
        if getattr(self, "ctx", None):
            rmdf_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Batch:
    """Many independent streams advanced together (one hipGraph launch per
    step).  ``streams`` is a list of dicts with H, W, M=(Kx, Ky, Kt), gx, gy."""

    def __init__(self, streams, *, tile_rows=0, kernel_variant=0, velocity_mode=VEL_SEARCH, fixed_v=(0.0, 0.0), temporal=TEMPORAL_OBSERVER,
                 stream=None):
        import torch
        self.specs = []
        descs = (rmdf_stream_desc * len(streams))()
        self._keep = []
        for i, sp in enumerate(streams):
            gx = np.ascontiguousarray(sp["gx"], np.float32)
            gy = np.ascontiguousarray(sp["gy"], np.float32)
            self._keep += [gx, gy]
            Mx, My, Mz = sp["M"]
            descs[i] = rmdf_stream_desc(int(sp["H"]), int(sp["W"]), Mx, My, Mz, gx.ctypes.data, gy.ctypes.data,
                                        len(gx), len(gy))
            self.specs.append(dict(sp, nv=len(gx) * len(gy)))
        p = rmdf_params_default()
        p.tile_rows = int(tile_rows)
        p.kernel_variant = int(kernel_variant)
        p.velocity_mode = int(velocity_mode)
        p.fixed_vx, p.fixed_vy = (float(v) for v in fixed_v)
        p.temporal = int(temporal)
        if stream is None:
            self.torch_stream = torch.cuda.Stream()
            stream = self.torch_stream.cuda_stream
        else:
            self.torch_stream = torch.cuda.ExternalStream(int(stream))
        self.stream_handle = int(stream)
        self.b = _VP()
        _bcheck(lib().rmdf_batch_create(len(streams), descs, ctypes.byref(p), ctypes.c_void_p(self.stream_handle),
                                        ctypes.byref(self.b)), None)
        self.n = len(streams)

    def input(self, s: int):
        """Device address of stream s's next input frame (H*W FP32)."""
        ptr = _VP()
        _bcheck(lib().rmdf_batch_input(self.b, int(s), ctypes.byref(ptr)), self.b)
        return ptr.value

    # The batch runs on its own stream: work the caller queued on torch's
    # current stream (frames written, output buffers freed) is ordered before
    # each call, and outputs are ordered back onto the current stream.
    def launch(self):
        import torch
        self.torch_stream.wait_stream(torch.cuda.current_stream())
        _bcheck(lib().rmdf_batch_launch(self.b), self.b)

    def push(self, frames):
        import torch
        ptrs = (ctypes.c_void_p * self.n)()
        for i, fr in enumerate(frames):
            sp = self.specs[i]
            ptrs[i] = _dev_ptr(fr, torch.float32, sp["H"] * sp["W"], "frame %d" % i)
        self.torch_stream.wait_stream(torch.cuda.current_stream())
        _bcheck(lib().rmdf_batch_push(self.b, ptrs), self.b)
        for fr in frames:
            fr.record_stream(self.torch_stream)

    def output(self, s: int):
        import torch
        sp = self.specs[s]
        out = torch.empty((sp["H"], sp["W"]), dtype=torch.float32, device="cuda")
        vxy = torch.empty((sp["H"], sp["W"], 2), dtype=torch.float32, device="cuda")
        idx = torch.empty((sp["H"], sp["W"]), dtype=torch.int32, device="cuda")
        cur = torch.cuda.current_stream()
        self.torch_stream.wait_stream(cur)
        _bcheck(lib().rmdf_batch_output(self.b, int(s), out.data_ptr(), vxy.data_ptr(), idx.data_ptr()), self.b)
        cur.wait_stream(self.torch_stream)
        for x in (out, vxy, idx):
            x.record_stream(self.torch_stream)
        return out, vxy, idx

    def set_tiles(self, s: int, tile_rows: int):
        _bcheck(lib().rmdf_batch_set_tiles(self.b, int(s), int(tile_rows)), self.b)

    def set_schedule(self, schedule: int):
        """0 one kernel per tile family, 1 one mixed kernel, 2 small families
        on a parallel graph branch, 3 as 2 with the small families launched
        first (rmdf_batch_set_schedule)."""
        _bcheck(lib().rmdf_batch_set_schedule(self.b, int(schedule)), self.b)

    def autotune(self, iters: int = 5) -> str:
        buf = ctypes.create_string_buffer(4096)
        _bcheck(lib().rmdf_batch_autotune(self.b, int(iters), buf, 4096), self.b)
        return buf.value.decode()

    def set_timing(self, on: bool):
        _bcheck(lib().rmdf_batch_set_timing(self.b, int(bool(on))), self.b)

    def latency(self):
        p50, p99, mean, n = ctypes.c_float(), ctypes.c_float(), ctypes.c_float(), ctypes.c_longlong()
        _bcheck(lib().rmdf_batch_latency(self.b, ctypes.byref(p50), ctypes.byref(p99), ctypes.byref(mean),
                                         ctypes.byref(n)), self.b)
        return {"p50_ms": p50.value, "p99_ms": p99.value, "mean_ms": mean.value, "steps": n.value}

    def synchronize(self):
        import torch
        torch.cuda.synchronize()

    def close(self):
        if getattr(self, "b", None):
            lib().rmdf_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- learned-model kernels on torch tensors (argument marshalling only) ----

def _stream_handle():
    import torch
    return torch.cuda.current_stream().cuda_stream


def _p(t):
    return None if t is None else t.data_ptr()


def mlp_gemm_nt(A, B, bias=None, epi=0, aux=None, out_f32=None, out_bf16=None):
    """C = epi(A @ B.T + bias); A [M, K], B [N, K] torch.bfloat16 contiguous."""
    M, K = A.shape
    N = B.shape[0]
    ldc = (out_f32 if out_f32 is not None else out_bf16).shape[1]
    _check(lib().rmdf_mlp_gemm_nt(A.data_ptr(), A.shape[1], B.data_ptr(), B.shape[1], M, N, K, _p(bias), int(epi),
                                  _p(aux), 0 if aux is None else aux.shape[1], _p(out_f32), _p(out_bf16), ldc,
                                  ctypes.c_void_p(_stream_handle())))


def mlp_transpose(inp, out):
    import torch
    R, C = inp.shape
    if inp.dtype == torch.bfloat16:
        _check(lib().rmdf_mlp_transpose(inp.data_ptr(), None, R, C, out.data_ptr(), ctypes.c_void_p(_stream_handle())))
    else:
        _check(lib().rmdf_mlp_transpose(None, inp.data_ptr(), R, C, out.data_ptr(), ctypes.c_void_p(_stream_handle())))


def mlp_head(h2, W3, b3, labels, wv, half_step, dh2, dW3, db3, loss):
    _check(lib().rmdf_mlp_head(h2.data_ptr(), W3.data_ptr(), b3.data_ptr(), labels.data_ptr(), h2.shape[0],
                               float(wv), float(half_step), dh2.data_ptr(), dW3.data_ptr(), db3.data_ptr(),
                               loss.data_ptr(), ctypes.c_void_p(_stream_handle())))


def mlp_colsum(inp, out):
    R, C = inp.shape
    _check(lib().rmdf_mlp_colsum(inp.data_ptr(), R, C, out.data_ptr(), ctypes.c_void_p(_stream_handle())))


def mlp_infer_head(h2, W3, b3, out):
    _check(lib().rmdf_mlp_infer_head(h2.data_ptr(), W3.data_ptr(), b3.data_ptr(), h2.shape[0], out.data_ptr(),
                                     ctypes.c_void_p(_stream_handle())))


def mlp_adam(p, g, m, v, p_bf16, lr, step, b1=0.9, b2=0.999, eps=1e-8):
    _check(lib().rmdf_mlp_adam(p.data_ptr(), g.data_ptr(), m.data_ptr(), v.data_ptr(), _p(p_bf16), p.numel(),
                               float(lr), float(b1), float(b2), float(eps), int(step),
                               ctypes.c_void_p(_stream_handle())))


def mlp_to_bf16(inp, out):
    _check(lib().rmdf_mlp_to_bf16(inp.data_ptr(), out.data_ptr(), inp.numel(), ctypes.c_void_p(_stream_handle())))


def cfar(x, guard: int, train: int, k: float, want_level: bool = False):
    """Two-sided cell-averaging CFAR (rmdf_cfar) on a [H, W] float32 CUDA
    tensor, on torch's current stream.  Returns the detections (uint8, 0/1)
    and, if asked, the per-pixel sigma estimate."""
    import torch
    H, W = x.shape
    xp = _dev_ptr(x, torch.float32, H * W, "image")
    det = torch.empty((H, W), dtype=torch.uint8, device=x.device)
    lev = torch.empty((H, W), dtype=torch.float32, device=x.device) if want_level else None
    _check(lib().rmdf_cfar(xp, int(H), int(W), int(guard), int(train), float(k), det.data_ptr(), _p(lev),
                           ctypes.c_void_p(_stream_handle())))
    return (det, lev) if want_level else det


def hbm_probe(kind: int, src, dst, nbytes: int, n_blocks: int, nt: bool = False):
    """One pass of the HBM streaming probe (rmdf_hbm_probe) on torch's current
    stream: kind 0 read src (dst: n_blocks FP32 partial sums), 1 write dst,
    2 copy src to dst."""
    _check(lib().rmdf_hbm_probe(int(kind), None if src is None else src.data_ptr(), dst.data_ptr(), int(nbytes),
                                int(n_blocks), int(bool(nt)), _stream_handle()))
