"""Python binding of libgls (ctypes).  Argument marshalling only: every step
of the solve runs in the HIP library.  PyTorch provides device memory,
pinned host memory and streams.

Layouts (torch row-major views of the library's column-major matrices):
  Phi  (n, n)       symmetric
  XL   (n, p-1)     passed to the library as (p-1, n) contiguous
  y    (n,)
  XR   (mb, n)      one SNP per row  == column-major n x mb
  b    (mb, p)      one SNP per row  == column-major p x mb
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgls.so")

GLS_FP64, GLS_FP32_IR, GLS_FP16_IR, GLS_BF16_IR, GLS_INT8_EMU = 0, 1, 2, 3, 4
PRECISIONS = {"fp64": GLS_FP64, "fp32_ir": GLS_FP32_IR, "fp16_ir": GLS_FP16_IR, "bf16_ir": GLS_BF16_IR,
              "int8_emu": GLS_INT8_EMU}
GLS_KEEP_FOR_GRAD = 1
GLS_STREAM_SERIAL = 2

STATUS = {0: "GLS_OK", -1: "GLS_ERR_ARG", -2: "GLS_ERR_NOT_SPD", -3: "GLS_ERR_HIP",
          -4: "GLS_ERR_WORKSPACE", -5: "GLS_ERR_STATE", -6: "GLS_ERR_RANK"}


class GlsOpts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("refine_sweeps", ctypes.c_int32),
                ("block_cols", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class GlsStreamStats(ctypes.Structure):
    _fields_ = [("blocks", ctypes.c_int64), ("h2d_bytes", ctypes.c_int64), ("d2h_bytes", ctypes.c_int64),
                ("wall_ms", ctypes.c_double), ("compute_ms", ctypes.c_double), ("file_bytes", ctypes.c_int64),
                ("read_ms", ctypes.c_double)]


class GlsPhaseStats(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64 * 4), ("ms", ctypes.c_double * 4)]


PHASES = ("whiten", "residual", "snp", "backward")


class GLSError(RuntimeError):
    def __init__(self, status: int, msg: str, info: int = 0):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status
        self.info = info


_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32
_D = ctypes.c_double

# name -> (restype, argtypes); every symbol include/gls.h declares
SIGNATURES = {
    "gls_workspace_bytes": (ctypes.c_size_t, [_I64, _I32, ctypes.POINTER(GlsOpts)]),
    "gls_setup": (ctypes.c_int, [ctypes.POINTER(_P), _I64, _I32, _P, _I64, _D, _P, _I64, _P, _P,
                                 ctypes.c_size_t, ctypes.POINTER(GlsOpts), _P, ctypes.POINTER(_I64)]),
    "gls_block": (ctypes.c_int, [_P, _I32, _P, _I64, _P, _I64, _P, _P, _P, _P]),
    "gls_stream": (ctypes.c_int, [_P, _I64, _I64, _P, _I64, _P, _P, _P, _P, _P, _P,
                                  ctypes.POINTER(GlsStreamStats)]),
    "gls_block_u8": (ctypes.c_int, [_P, _I32, _P, _I64, _P, _I64, _P, _P, _P, _P]),
    "gls_stream_u8": (ctypes.c_int, [_P, _I64, _I64, _P, _I64, _P, _P, _P, _P, _P, _P,
                                     ctypes.POINTER(GlsStreamStats)]),
    "gls_block_u2": (ctypes.c_int, [_P, _I32, _P, _I64, _P, _I64, _P, _P, _P, _P]),
    "gls_stream_u2": (ctypes.c_int, [_P, _I64, _I64, _P, _I64, _P, _P, _P, _P, _P, _P,
                                     ctypes.POINTER(GlsStreamStats)]),
    "gls_stream_file_host_bytes": (ctypes.c_size_t, [_P, _I32]),
    "gls_stream_file": (ctypes.c_int, [_P, ctypes.c_char_p, _I64, _I32, _I64, _I64, _P, ctypes.c_size_t,
                                       _P, _P, _P, _P, _P, _P, ctypes.POINTER(GlsStreamStats)]),
    "gls_backward_block": (ctypes.c_int, [_P, _I32, _P, _I64, _P, _P, _P, _P, _P]),
    "gls_backward_finish": (ctypes.c_int, [_P, _P, _P, _P]),
    "gls_stream_backward": (ctypes.c_int, [_P, _I64, _I64, _P, _I64, _P, _P, _P, _P, _P, _P,
                                           ctypes.POINTER(GlsStreamStats)]),
    "gls_stream_backward_file": (ctypes.c_int, [_P, ctypes.c_char_p, _I64, _I32, _I64, _I64, _P, ctypes.c_size_t,
                                                _P, _P, _P, _P, _P, _P, ctypes.POINTER(GlsStreamStats)]),
    "gls_profile_enable": (ctypes.c_int, [_P, _I32]),
    "gls_profile_read": (ctypes.c_int, [_P, ctypes.POINTER(GlsPhaseStats), _I32]),
    "gls_destroy": (None, [_P]),
    "gls_solve_noalloc": (ctypes.c_int, [_I64, _I32, _P, _I64, _D, _P, _I64, _P, _I64, _P, _I64, _P, _I64, _P, _P,
                                         _P, ctypes.POINTER(GlsOpts), _P, ctypes.POINTER(_I64)]),
    "gls_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "gls_last_error": (ctypes.c_char_p, []),
}

_lib = None

# gls_stream_file's elem_bits for each file format
_FILE_BITS = {torch.float64: 64, "f64": 64, torch.uint8: 8, "u8": 8, "u2": 2}


def lib() -> ctypes.CDLL:
    """The loaded HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1302_4332_amd.build_lib`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(status: int, info: int = 0):
    if status != 0:
        raise GLSError(status, lib().gls_last_error().decode(), info)


def _ptr(t: torch.Tensor | None):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(s=None):
    s = torch.cuda.current_stream() if s is None else s
    return ctypes.c_void_p(s.cuda_stream)


def _need(t: torch.Tensor, name: str, dtype=torch.float64, cuda=True):
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if cuda and not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def make_opts(block_cols: int, precision="fp64", refine_sweeps: int = 0, keep_for_grad: bool = False,
              serial_stream: bool = False) -> GlsOpts:
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    flags = (GLS_KEEP_FOR_GRAD if keep_for_grad else 0) | (GLS_STREAM_SERIAL if serial_stream else 0)
    return GlsOpts(prec, int(refine_sweeps), int(block_cols), flags)


def workspace_bytes(n: int, p: int, opts: GlsOpts) -> int:
    return int(lib().gls_workspace_bytes(n, p, ctypes.byref(opts)))


# size of the library's static device scratch behind gls_solve_noalloc
NOALLOC_SCRATCH_BYTES = 64 << 20


def solve_noalloc(Phi, h2, XL, y, XR, b, sigma2, v, status, *, block_cols: int, precision="fp64",
                  refine_sweeps: int = 0, stream=None):
    """gls_solve_noalloc: setup and every SNP of XR (m, n) into caller-provided
    outputs b (m, p), sigma2, v (m,) float64 and status (m,) int32, with the
    library's static scratch as workspace (nothing is allocated).  Synchronous."""
    for t, name in ((Phi, "Phi"), (y, "y"), (XR, "XR"), (b, "b"), (sigma2, "sigma2"), (v, "v")):
        _need(t, name)
    _need(status, "status", torch.int32)
    n = Phi.shape[0]
    if XL is None:
        XL = torch.empty((n, 0), dtype=torch.float64, device=Phi.device)
    p = XL.shape[1] + 1
    m = XR.shape[0]
    if tuple(Phi.shape) != (n, n) or tuple(y.shape) != (n,) or XL.shape[0] != n:
        raise ValueError("Phi must be (n, n), y (n,), XL (n, p - 1)")
    if XR.dim() != 2 or XR.shape[1] != n or tuple(b.shape) != (m, p) or sigma2.shape[0] != m \
            or v.shape[0] != m or status.shape[0] != m:
        raise ValueError(f"XR must be (m, {n}), b (m, {p}), sigma2, v and status (m,)")
    XLc = XL.t().contiguous() if p > 1 else None
    opts = make_opts(block_cols, precision, refine_sweeps)
    info = ctypes.c_int64(0)
    st = lib().gls_solve_noalloc(n, p, _ptr(Phi), n, float(h2), _ptr(XLc), n, _ptr(y), m, _ptr(XR), n, _ptr(b), p,
                                 _ptr(sigma2), _ptr(v), _ptr(status), ctypes.byref(opts), _stream(stream),
                                 ctypes.byref(info))
    _check(st, info.value)


class GLSContext:
    """One study: setup on construction, then SNP blocks.

    Phi (n, n), XL (n, p-1), y (n,) are float64 CUDA tensors.
    """

    def __init__(self, Phi, h2, XL, y, *, block_cols: int, precision="fp64", refine_sweeps: int = 0,
                 keep_for_grad: bool = False, serial_stream: bool = False, stream=None):
        _need(Phi, "Phi")
        _need(y, "y")
        n = Phi.shape[0]
        if Phi.dim() != 2 or Phi.shape[1] != n:
            raise ValueError(f"Phi must be square, got {tuple(Phi.shape)}")
        if tuple(y.shape) != (n,):
            raise ValueError(f"y must have shape ({n},), got {tuple(y.shape)}")
        if XL is None:
            XL = torch.empty((n, 0), dtype=torch.float64, device=Phi.device)
        _need(XL.contiguous(), "XL")
        if XL.dim() != 2 or XL.shape[0] != n:
            raise ValueError(f"XL must have shape ({n}, p - 1), got {tuple(XL.shape)}")
        if XL.device != Phi.device or y.device != Phi.device:
            raise ValueError("Phi, XL and y must be on the same device")
        p = XL.shape[1] + 1
        XLc = XL.t().contiguous() if XL.shape[1] else None
        self.n, self.p = n, p
        self.opts = make_opts(block_cols, precision, refine_sweeps, keep_for_grad, serial_stream)
        nbytes = workspace_bytes(n, p, self.opts)
        if nbytes == 0:
            raise GLSError(-1, f"invalid sizes or options (n={n}, p={p}, block_cols={block_cols})")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=Phi.device)
        h = ctypes.c_void_p()
        info = ctypes.c_int64(0)
        st = lib().gls_setup(ctypes.byref(h), n, p, _ptr(Phi), n, float(h2), _ptr(XLc), n, _ptr(y),
                             _ptr(self.workspace), nbytes, ctypes.byref(self.opts), _stream(stream),
                             ctypes.byref(info))
        _check(st, info.value)
        self.handle = h
        self.block_cols = block_cols
        self._streams = set()

    def _use(self, stream):
        """The stream the library will enqueue on; a stream other than the one the
        workspace was allocated on is recorded with the caching allocator, so the
        workspace is not handed out again while work queued there may still run."""
        s = torch.cuda.current_stream() if stream is None else stream
        key = s.cuda_stream
        if key not in self._streams:
            self._streams.add(key)
            self.workspace.record_stream(s)
        return ctypes.c_void_p(key)

    def close(self):
        if getattr(self, "handle", None):
            lib().gls_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def profile(self, on: bool = True):
        _check(lib().gls_profile_enable(self.handle, 1 if on else 0))

    def profile_read(self, reset: bool = True) -> dict:
        """{phase: (timed launches, summed device ms)} from the library's HIP events."""
        ps = GlsPhaseStats()
        _check(lib().gls_profile_read(self.handle, ctypes.byref(ps), 1 if reset else 0))
        return {name: (int(ps.launches[i]), float(ps.ms[i])) for i, name in enumerate(PHASES)}

    def block_into(self, XR, b, sigma2, v, status, stream=None):
        """Solve one block into caller-provided outputs (no allocation)."""
        _need(XR, "XR")
        mb = XR.shape[0]
        if XR.dim() != 2 or XR.shape[1] != self.n:
            raise ValueError(f"XR must have shape (mb, {self.n})")
        for t, name, dt in ((b, "b", torch.float64), (sigma2, "sigma2", torch.float64),
                            (v, "v", torch.float64), (status, "status", torch.int32)):
            _need(t, name, dt)
            if t.shape[0] != mb or (name == "b" and tuple(t.shape) != (mb, self.p)):
                raise ValueError(f"{name} has the wrong shape {tuple(t.shape)}")
        st = lib().gls_block(self.handle, mb, _ptr(XR), self.n,
                             _ptr(b), self.p, _ptr(sigma2), _ptr(v), _ptr(status), self._use(stream))
        _check(st)

    def _dosage_block_into(self, entry, rowbytes, G, b, sigma2, v, status, stream):
        _need(G, "G", torch.uint8)
        mb = G.shape[0]
        if G.dim() != 2 or G.shape[1] != rowbytes:
            raise ValueError(f"G must have shape (mb, {rowbytes})")
        for t, name, dt in ((b, "b", torch.float64), (sigma2, "sigma2", torch.float64),
                            (v, "v", torch.float64), (status, "status", torch.int32)):
            _need(t, name, dt)
            if t.shape[0] != mb or (name == "b" and tuple(t.shape) != (mb, self.p)):
                raise ValueError(f"{name} has the wrong shape {tuple(t.shape)}")
        _check(entry(self.handle, mb, _ptr(G), rowbytes, _ptr(b), self.p, _ptr(sigma2), _ptr(v),
                     _ptr(status), self._use(stream)))

    def _outputs(self, mb, dev):
        return (torch.empty((mb, self.p), dtype=torch.float64, device=dev),
                torch.empty(mb, dtype=torch.float64, device=dev),
                torch.empty(mb, dtype=torch.float64, device=dev),
                torch.empty(mb, dtype=torch.int32, device=dev))

    def block_u8_into(self, G, b, sigma2, v, status, stream=None):
        """One block of genotype bytes (mb, n) uint8 CUDA into caller-provided outputs."""
        self._dosage_block_into(lib().gls_block_u8, self.n, G, b, sigma2, v, status, stream)

    def block_u8(self, G, stream=None):
        out = self._outputs(G.shape[0], G.device)
        self.block_u8_into(G, *out, stream)
        return out

    def block_u2_into(self, G2, b, sigma2, v, status, stream=None):
        """One block of packed 2-bit dosages (mb, ceil(n / 4)) uint8 CUDA (the layout
        of ``synth.pack_dosages_2bit``) into caller-provided outputs."""
        self._dosage_block_into(lib().gls_block_u2, (self.n + 3) // 4, G2, b, sigma2, v, status, stream)

    def block_u2(self, G2, stream=None):
        out = self._outputs(G2.shape[0], G2.device)
        self.block_u2_into(G2, *out, stream)
        return out

    def block(self, XR, stream=None):
        """XR: (mb, n) float64 CUDA.  Returns b (mb, p), sigma2, v, status."""
        mb = XR.shape[0]
        dev = XR.device
        b = torch.empty((mb, self.p), dtype=torch.float64, device=dev)
        s2 = torch.empty(mb, dtype=torch.float64, device=dev)
        v = torch.empty(mb, dtype=torch.float64, device=dev)
        status = torch.empty(mb, dtype=torch.int32, device=dev)
        self.block_into(XR, b, s2, v, status, stream)
        return b, s2, v, status

    def stream_file(self, path: str, m: int, fmt=torch.float64, offset: int = 0, col0: int = 0, out=None,
                    host_ws=None, compute_stream=None, copy_stream=None):
        """Stream SNPs [col0, m) from a SNP-major file; fmt is torch.float64,
        torch.uint8 (genotype bytes) or "u2" (packed 2-bit dosages)."""
        elem = _FILE_BITS[fmt]
        need = int(lib().gls_stream_file_host_bytes(self.handle, elem))
        if host_ws is None or host_ws.numel() < need:
            host_ws = torch.empty(need, dtype=torch.uint8).pin_memory()
        if out is None:
            out = (torch.full((m, self.p), float("nan"), dtype=torch.float64).pin_memory(),
                   torch.full((m,), float("nan"), dtype=torch.float64).pin_memory(),
                   torch.full((m,), float("nan"), dtype=torch.float64).pin_memory(),
                   torch.full((m,), -1, dtype=torch.int32).pin_memory())
        b, s2, v, status = out
        stats = GlsStreamStats()
        cs = compute_stream or torch.cuda.current_stream()
        xs = self._use(copy_stream) if copy_stream is not None else ctypes.c_void_p(None)
        st = lib().gls_stream_file(self.handle, path.encode(), offset, elem, m, col0, _ptr(host_ws), host_ws.numel(),
                                   _ptr(b), _ptr(s2), _ptr(v), _ptr(status), self._use(cs), xs,
                                   ctypes.byref(stats))
        _check(st)
        return (b, s2, v, status), stats

    def stream(self, XR_host, col0: int = 0, out=None, compute_stream=None, copy_stream=None, packed=False):
        """Stream SNPs [col0, m) of a pinned host tensor XR_host: (m, n) float64
        or uint8 genotype bytes, or with packed=True (m, ceil(n / 4)) uint8
        packed 2-bit dosages.

        The study runs after the work queued on compute_stream (default: the
        current stream).  With copy_stream None it runs on the handle's own
        compute and copy streams, which setup checked do not share a hardware
        queue; a caller-given copy stream gets no such check.  Returns
        (b, sigma2, v, status) host tensors and the stats struct.
        """
        _need(XR_host, "XR_host", XR_host.dtype if XR_host.dtype in (torch.uint8, torch.float64) else torch.float64,
              cuda=False)
        if XR_host.is_cuda:
            raise TypeError("XR_host must be a host tensor (page-locked: .pin_memory())")
        if packed:
            _need(XR_host, "XR_host", torch.uint8, cuda=False)
            entry, rowlen = lib().gls_stream_u2, (self.n + 3) // 4
        else:
            entry, rowlen = (lib().gls_stream_u8 if XR_host.dtype == torch.uint8 else lib().gls_stream), self.n
        if XR_host.dim() != 2 or XR_host.shape[1] != rowlen:
            raise ValueError(f"XR_host must have shape (m, {rowlen})")
        m = XR_host.shape[0]
        if out is None:
            out = (torch.full((m, self.p), float("nan"), dtype=torch.float64).pin_memory(),
                   torch.full((m,), float("nan"), dtype=torch.float64).pin_memory(),
                   torch.full((m,), float("nan"), dtype=torch.float64).pin_memory(),
                   torch.full((m,), -1, dtype=torch.int32).pin_memory())
        b, s2, v, status = out
        for t, name, dt, shape in ((b, "b", torch.float64, (m, self.p)), (s2, "sigma2", torch.float64, (m,)),
                                   (v, "v", torch.float64, (m,)), (status, "status", torch.int32, (m,))):
            _need(t, name, dt, cuda=False)
            if tuple(t.shape) != shape:
                raise ValueError(f"{name} must have shape {shape}, got {tuple(t.shape)}")
        stats = GlsStreamStats()
        cs = compute_stream or torch.cuda.current_stream()
        xs = self._use(copy_stream) if copy_stream is not None else ctypes.c_void_p(None)
        st = entry(self.handle, m, col0, _ptr(XR_host), rowlen, _ptr(b), _ptr(s2), _ptr(v),
                   _ptr(status), self._use(cs), xs, ctypes.byref(stats))
        _check(st)
        return (b, s2, v, status), stats


    def stream_backward(self, XR_host, b_bar, sigma2_bar, v_bar, col0: int = 0, XR_grad=None, compute_stream=None,
                        copy_stream=None):
        """Adjoint of a streamed study (the handle needs keep_for_grad=True):
        SNPs [col0, m) of the pinned host tensor XR_host (m, n) float64 with the
        cotangents b_bar (m, p), sigma2_bar (m,), v_bar (m,) of its outputs
        (float64 host tensors, page-locked for overlapped copies).  XR_grad,
        if given, is a host tensor (m, n) that receives d loss / d X_R.  The
        adjoint sums add up in the handle until backward_finish().  Streams as
        for stream().  Returns the stats struct."""
        _need(XR_host, "XR_host", cuda=False)
        if XR_host.is_cuda:
            raise TypeError("XR_host must be a host tensor (page-locked: .pin_memory())")
        if XR_host.dim() != 2 or XR_host.shape[1] != self.n:
            raise ValueError(f"XR_host must have shape (m, {self.n})")
        m = XR_host.shape[0]
        for t, name, shape in ((b_bar, "b_bar", (m, self.p)), (sigma2_bar, "sigma2_bar", (m,)),
                               (v_bar, "v_bar", (m,))) + (((XR_grad, "XR_grad", (m, self.n)),) if XR_grad is not None
                                                           else ()):
            _need(t, name, cuda=False)
            if t.is_cuda or tuple(t.shape) != shape:
                raise ValueError(f"{name} must be a host tensor of shape {shape}")
        stats = GlsStreamStats()
        cs = compute_stream or torch.cuda.current_stream()
        xs = self._use(copy_stream) if copy_stream is not None else ctypes.c_void_p(None)
        st = lib().gls_stream_backward(self.handle, m, col0, _ptr(XR_host), self.n, _ptr(b_bar), _ptr(sigma2_bar),
                                       _ptr(v_bar), _ptr(XR_grad), self._use(cs), xs, ctypes.byref(stats))
        _check(st)
        return stats

    def stream_backward_file(self, path: str, m: int, b_bar, sigma2_bar, v_bar, fmt=torch.float64, offset: int = 0,
                             col0: int = 0, XR_grad=None, host_ws=None, compute_stream=None, copy_stream=None):
        """stream_backward for SNPs [col0, m) read from a SNP-major file, in the
        formats of stream_file (torch.float64, torch.uint8 or "u2"); XR_grad, if
        given, is a host tensor (m, n) float64.  Returns the stats struct."""
        elem = _FILE_BITS[fmt]
        for t, name, shape in ((b_bar, "b_bar", (m, self.p)), (sigma2_bar, "sigma2_bar", (m,)), (v_bar, "v_bar", (m,))) + (
                ((XR_grad, "XR_grad", (m, self.n)),) if XR_grad is not None else ()):
            _need(t, name, cuda=False)
            if t.is_cuda or tuple(t.shape) != shape:
                raise ValueError(f"{name} must be a host tensor of shape {shape}")
        need = int(lib().gls_stream_file_host_bytes(self.handle, elem))
        if host_ws is None or host_ws.numel() < need:
            host_ws = torch.empty(need, dtype=torch.uint8).pin_memory()
        stats = GlsStreamStats()
        cs = compute_stream or torch.cuda.current_stream()
        xs = self._use(copy_stream) if copy_stream is not None else ctypes.c_void_p(None)
        st = lib().gls_stream_backward_file(self.handle, path.encode(), offset, elem, m, col0, _ptr(host_ws),
                                            host_ws.numel(), _ptr(b_bar), _ptr(sigma2_bar), _ptr(v_bar),
                                            _ptr(XR_grad), self._use(cs), xs, ctypes.byref(stats))
        _check(st)
        return stats

    def backward_finish(self, stream=None):
        """(y_grad (n,), h2_grad (1,)) device tensors from the adjoint sums of the
        blocks passed since setup or the last finish; resets the sums."""
        dev = self.workspace.device
        y_grad = torch.empty(self.n, dtype=torch.float64, device=dev)
        h2_grad = torch.empty(1, dtype=torch.float64, device=dev)
        _check(lib().gls_backward_finish(self.handle, _ptr(y_grad), _ptr(h2_grad), self._use(stream)))
        return y_grad, h2_grad


def stream_grad(Phi, h2, XL, y, XR_host, loss, *, block_cols: int, precision="fp64", refine_sweeps: int = 0,
                XR_grad=None):
    """d loss / d (y, h2) (and d loss / d X_R into the host tensor XR_grad, if
    given) for a study whose SNPs (XR_host: pinned (m, n) float64) stay in host
    memory: the study is streamed forward (gls_stream), loss(b, sigma2, v) is
    differentiated by torch on the device outputs, and the study is streamed
    again through the adjoint (gls_stream_backward, then gls_backward_finish).
    Returns (loss value, y_grad, h2_grad, (b, sigma2, v, status) host tensors)."""
    _need(XR_host, "XR_host", cuda=False)   # the adjoint takes FP64 SNP values
    g = GLSContext(Phi, h2, XL, y, block_cols=block_cols, precision=precision, refine_sweeps=refine_sweeps,
                   keep_for_grad=True)
    try:
        outs, _ = g.stream(XR_host)
        dev = Phi.device
        leaves = [t.to(dev).requires_grad_(True) for t in outs[:3]]
        value = loss(*leaves)
        grads = torch.autograd.grad(value, leaves, allow_unused=True)
        cot = [torch.zeros_like(t) if gr is None else gr for t, gr in zip(leaves, grads)]
        cot = [c.detach().cpu().pin_memory() for c in cot]
        g.stream_backward(XR_host, *cot, XR_grad=XR_grad)
        y_grad, h2_grad = g.backward_finish()
        torch.cuda.current_stream().synchronize()
    finally:
        g.close()
    return float(value.detach()), y_grad, h2_grad, outs


def stream_grad_file(Phi, h2, XL, y, path: str, m: int, loss, *, block_cols: int, fmt=torch.float64,
                     offset: int = 0, precision="fp64", refine_sweeps: int = 0, XR_grad=None):
    """stream_grad for a study whose SNPs are read from a SNP-major file (the
    formats of GLSContext.stream_file): the forward stream and the adjoint each
    read the file once (gls_stream_file, gls_stream_backward_file).  Returns
    (loss value, y_grad, h2_grad, (b, sigma2, v, status) host tensors)."""
    g = GLSContext(Phi, h2, XL, y, block_cols=block_cols, precision=precision, refine_sweeps=refine_sweeps,
                   keep_for_grad=True)
    try:
        need = int(lib().gls_stream_file_host_bytes(g.handle, _FILE_BITS[fmt]))
        host_ws = torch.empty(need, dtype=torch.uint8).pin_memory()
        outs, _ = g.stream_file(path, m, fmt, offset=offset, host_ws=host_ws)
        dev = Phi.device
        leaves = [t.to(dev).requires_grad_(True) for t in outs[:3]]
        value = loss(*leaves)
        grads = torch.autograd.grad(value, leaves, allow_unused=True)
        cot = [torch.zeros_like(t) if gr is None else gr for t, gr in zip(leaves, grads)]
        cot = [c.detach().cpu().pin_memory() for c in cot]
        g.stream_backward_file(path, m, *cot, fmt=fmt, offset=offset, XR_grad=XR_grad, host_ws=host_ws)
        y_grad, h2_grad = g.backward_finish()
        torch.cuda.current_stream().synchronize()
    finally:
        g.close()
    return float(value.detach()), y_grad, h2_grad, outs


class GLSFunction(torch.autograd.Function):
    """(b, sigma2, v) of every SNP as a differentiable function of y, X_R and h2.

    Forward runs the library's setup and block path; backward is the
    library's hand-written adjoint (gls_backward_block per block, then
    gls_backward_finish), which recomputes each block's whitened SNPs instead
    of storing them.  Phi and X_L are constants.

        b, sigma2, v = GLSFunction.apply(y, XR, h2, Phi, XL, block_cols, precision, sweeps)

    y (n,), XR (m, n), Phi (n, n), XL (n, p-1): float64 CUDA tensors; h2 a
    float64 scalar tensor.
    """

    @staticmethod
    def forward(ctx, y, XR, h2, Phi, XL, block_cols, precision="fp64", sweeps=0):
        g = GLSContext(Phi, float(h2), XL, y.detach().contiguous(), block_cols=block_cols, precision=precision,
                       refine_sweeps=sweeps, keep_for_grad=True)
        XRd = XR.detach().contiguous()
        m = XRd.shape[0]
        dev = XRd.device
        b = torch.empty((m, g.p), dtype=torch.float64, device=dev)
        s2 = torch.empty(m, dtype=torch.float64, device=dev)
        v = torch.empty(m, dtype=torch.float64, device=dev)
        st = torch.empty(m, dtype=torch.int32, device=dev)
        for j0 in range(0, m, block_cols):
            j1 = min(m, j0 + block_cols)
            g.block_into(XRd[j0:j1], b[j0:j1], s2[j0:j1], v[j0:j1], st[j0:j1])
        ctx.g = g
        ctx.block_cols = block_cols
        ctx.h2_shape = h2.shape if isinstance(h2, torch.Tensor) else ()
        ctx.save_for_backward(XRd)
        return b, s2, v

    @staticmethod
    def backward(ctx, bbar, s2bar, vbar):
        g = ctx.g
        (XR,) = ctx.saved_tensors
        m, n = XR.shape
        dev = XR.device
        z = lambda shape: torch.zeros(shape, dtype=torch.float64, device=dev)
        bbar = z((m, g.p)) if bbar is None else bbar.contiguous()
        s2bar = z(m) if s2bar is None else s2bar.contiguous()
        vbar = z(m) if vbar is None else vbar.contiguous()
        want_xr = ctx.needs_input_grad[1]
        XR_grad = torch.empty_like(XR) if want_xr else None
        stream = _stream()
        for j0 in range(0, m, ctx.block_cols):
            j1 = min(m, j0 + ctx.block_cols)
            st = lib().gls_backward_block(g.handle, j1 - j0, _ptr(XR[j0:j1]), n, _ptr(bbar[j0:j1]),
                                          _ptr(s2bar[j0:j1]), _ptr(vbar[j0:j1]),
                                          _ptr(XR_grad[j0:j1]) if want_xr else None, stream)
            _check(st)
        y_grad = torch.empty(n, dtype=torch.float64, device=dev)
        h2_grad = torch.empty(1, dtype=torch.float64, device=dev)
        _check(lib().gls_backward_finish(g.handle, _ptr(y_grad), _ptr(h2_grad), stream))
        torch.cuda.current_stream().synchronize()
        g.close()
        ctx.g = None
        return y_grad, XR_grad, h2_grad.reshape(ctx.h2_shape), None, None, None, None, None


def t2_loss(b, sigma2, v):
    """Sum over SNPs of squared t-statistics of the SNP coefficient."""
    return (b[:, -1] ** 2 / (sigma2 * v)).sum()
