"""ctypes binding of the C ABI in include/corr2d.h (libcorr2d.so).

The functions keep the C names and only marshal arguments: every step of the
correlation runs in the library's HIP kernels.  Device buffers are passed as
torch tensors (their data pointers) or raw integer addresses; streams as a
``torch.cuda.Stream`` or a raw ``hipStream_t`` integer.  There is no CPU
fallback: if the library is missing, loading it raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcorr2d.so")

# enums of corr2d.h
OK, EINVAL, EWORKSPACE, EUNSUPPORTED, EDEVICE, ENOMEM = range(6)
PREC = {"f64": 0, "f32": 1, "split_bf16": 2, "bf16": 3, "f16": 4, "fp8_e4m3": 5, "split_f16": 6}
BASIS = {"fourier": 0, "time": 1, "auto": 2}
HILBERT = {"noda": 0, "circular": 1, "r_compat": 2}
INTERP = {"none": 0, "linear": 1, "spline": 2}
NORM = {"noda": 0, "paper": 1, "custom": 2}
LAYOUT = {"full": 0, "upper_packed": 1, "upper_aligned": 2}
LAYOUT_NAMES = {v: k for k, v in LAYOUT.items()}
DTYPE = {"f64": 0, "f32": 1}
FLAG_PER_BAND_SCALE = 0x1
FLAG_NO_PER_BAND_SCALE = 0x2
FLAG_SEQUENTIAL = 0x4
FLAG_NO_GRAPH = 0x8
FLAG_TRANSFORM_MATMUL = 0x10
FLAG_SPLIT_ROWS = 0x20

EXPORTED = [
    "corr2d_desc_init", "corr2d_plan", "corr2d_batched_plan", "corr2d_plan_destroy",
    "corr2d_workspace_bytes", "corr2d_plan_get_info", "corr2d_homo", "corr2d_hetero",
    "corr2d_batched", "corr2d_status_str", "corr2d_last_error", "corr2d_version",
    "corr2d_set_timing_events", "corr2d_homo_noalloc",
]
NOALLOC_SCRATCH_BYTES = 64 << 20   # CORR2D_NOALLOC_SCRATCH_BYTES


class corr2d_desc(ctypes.Structure):
    _fields_ = [
        ("m", ctypes.c_int64), ("n1", ctypes.c_int64), ("n2", ctypes.c_int64),
        ("ld_in1", ctypes.c_int64), ("ld_in2", ctypes.c_int64), ("ld_out", ctypes.c_int64),
        ("in_dtype", ctypes.c_int32), ("out_dtype", ctypes.c_int32), ("prec", ctypes.c_int32),
        ("basis", ctypes.c_int32), ("hilbert", ctypes.c_int32), ("norm_mode", ctypes.c_int32),
        ("norm_value", ctypes.c_double), ("out_layout", ctypes.c_int32),
        ("flags", ctypes.c_uint32), ("tile", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("scale_alpha", ctypes.c_double),
        ("t_in", ctypes.POINTER(ctypes.c_double)), ("m_in", ctypes.c_int64),
        ("interp", ctypes.c_int32), ("reserved2", ctypes.c_int32),
        ("split_tol", ctypes.c_double),
    ]


class corr2d_item(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64), ("in_offset", ctypes.c_int64),
                ("ld_in", ctypes.c_int64), ("out_offset", ctypes.c_int64)]


class corr2d_plan_info(ctypes.Structure):
    _fields_ = [
        ("k_pad", ctypes.c_int64), ("n_pad", ctypes.c_int64), ("tiles", ctypes.c_int64),
        ("tile", ctypes.c_int32), ("tile_m", ctypes.c_int32), ("tile_n", ctypes.c_int32),
        ("per_band_scale", ctypes.c_int32), ("c", ctypes.c_double),
        ("workspace_bytes", ctypes.c_size_t), ("items", ctypes.c_int64),
        ("out_elements", ctypes.c_int64), ("transform", ctypes.c_int32), ("basis", ctypes.c_int32),
        ("ref1_offset", ctypes.c_size_t), ("ref2_offset", ctypes.c_size_t),
        ("sel_offset", ctypes.c_size_t),
    ]


_lib = None


def lib():
    """Load libcorr2d.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1808_00685_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, sz, st = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int
        plan_p = ctypes.POINTER(ctypes.c_void_p)
        L.corr2d_desc_init.argtypes = [ctypes.POINTER(corr2d_desc)]
        L.corr2d_desc_init.restype = None
        L.corr2d_plan.argtypes = [plan_p, ctypes.POINTER(corr2d_desc)]
        L.corr2d_plan.restype = st
        L.corr2d_batched_plan.argtypes = [plan_p, ctypes.POINTER(corr2d_desc),
                                          ctypes.POINTER(corr2d_item), ctypes.c_int64]
        L.corr2d_batched_plan.restype = st
        L.corr2d_plan_destroy.argtypes = [vp]
        L.corr2d_plan_destroy.restype = st
        L.corr2d_workspace_bytes.argtypes = [vp, ctypes.POINTER(sz)]
        L.corr2d_workspace_bytes.restype = st
        L.corr2d_plan_get_info.argtypes = [vp, ctypes.POINTER(corr2d_plan_info)]
        L.corr2d_plan_get_info.restype = st
        L.corr2d_homo.argtypes = [vp, vp, vp, vp, vp, vp, sz, vp]
        L.corr2d_homo.restype = st
        L.corr2d_homo_noalloc.argtypes = [vp, vp, vp, vp, vp, vp]
        L.corr2d_homo_noalloc.restype = st
        L.corr2d_hetero.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
        L.corr2d_hetero.restype = st
        L.corr2d_batched.argtypes = [vp, vp, vp, vp, vp, sz, vp]
        L.corr2d_batched.restype = st
        L.corr2d_status_str.argtypes = [st]
        L.corr2d_status_str.restype = ctypes.c_char_p
        L.corr2d_last_error.argtypes = []
        L.corr2d_last_error.restype = ctypes.c_char_p
        L.corr2d_set_timing_events.argtypes = [vp, vp]
        L.corr2d_set_timing_events.restype = st
        L.corr2d_version.argtypes = []
        L.corr2d_version.restype = ctypes.c_char_p
        _lib = L
    return _lib


class Corr2dError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{corr2d_status_str(status)}: {msg}")
        self.status = status


def _check(status):
    if status != OK:
        raise Corr2dError(status, corr2d_last_error())
    return status


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(s):
    if s is None:
        try:
            import torch
            if torch.cuda.is_available():
                return torch.cuda.current_stream().cuda_stream
        except Exception:
            pass
        return None
    if isinstance(s, int):
        return s
    return s.cuda_stream


# --------------------------------------------------------------------------
# The C functions, same names
# --------------------------------------------------------------------------
def corr2d_status_str(status) -> str:
    return lib().corr2d_status_str(int(status)).decode()


def corr2d_last_error() -> str:
    return lib().corr2d_last_error().decode()


def corr2d_version() -> str:
    return lib().corr2d_version().decode()


def corr2d_desc_init(**fields) -> corr2d_desc:
    """Defaults of the library, then the given fields (enum names accepted)."""
    d = corr2d_desc()
    lib().corr2d_desc_init(ctypes.byref(d))
    maps = {"prec": PREC, "basis": BASIS, "hilbert": HILBERT, "norm_mode": NORM,
            "out_layout": LAYOUT, "in_dtype": DTYPE, "out_dtype": DTYPE, "interp": INTERP}
    for k, v in fields.items():
        if k == "t_in":
            # perturbation values of the input rows (read when the plan is
            # made); the array stays referenced by the descriptor
            if v is None:
                continue
            import numpy as np
            arr = np.ascontiguousarray(v, dtype=np.float64)
            d._t_in_ref = arr
            d.t_in = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            if "m_in" not in fields:
                d.m_in = len(arr)
            continue
        if k in maps and isinstance(v, str):
            v = maps[k][v]
        setattr(d, k, v)
    return d


def corr2d_plan(desc: corr2d_desc, check=True):
    """Returns (status, plan handle)."""
    h = ctypes.c_void_p()
    s = lib().corr2d_plan(ctypes.byref(h), ctypes.byref(desc))
    if check:
        _check(s)
    return s, h.value


def corr2d_batched_plan(common: corr2d_desc, items, check=True):
    arr = (corr2d_item * len(items))()
    for i, it in enumerate(items):
        arr[i] = it if isinstance(it, corr2d_item) else corr2d_item(*it)
    h = ctypes.c_void_p()
    s = lib().corr2d_batched_plan(ctypes.byref(h), ctypes.byref(common), arr, len(items))
    if check:
        _check(s)
    return s, h.value


def corr2d_plan_destroy(plan):
    return _check(lib().corr2d_plan_destroy(plan))


def corr2d_workspace_bytes(plan) -> int:
    b = ctypes.c_size_t()
    _check(lib().corr2d_workspace_bytes(plan, ctypes.byref(b)))
    return b.value


def corr2d_plan_get_info(plan) -> corr2d_plan_info:
    info = corr2d_plan_info()
    _check(lib().corr2d_plan_get_info(plan, ctypes.byref(info)))
    return info


def corr2d_set_timing_events(before, after):
    return _check(lib().corr2d_set_timing_events(before, after))


def corr2d_homo(plan, y, ref, phi, psi, ws, ws_bytes=None, stream=None, check=True):
    if ws_bytes is None:
        ws_bytes = ws.numel() * ws.element_size()
    s = lib().corr2d_homo(plan, _ptr(y), _ptr(ref), _ptr(phi), _ptr(psi), _ptr(ws), ws_bytes,
                          _stream(stream))
    return _check(s) if check else s


def corr2d_homo_noalloc(plan, y, ref, phi, psi, stream=None, check=True):
    s = lib().corr2d_homo_noalloc(plan, _ptr(y), _ptr(ref), _ptr(phi), _ptr(psi), _stream(stream))
    return _check(s) if check else s


def corr2d_hetero(plan, y1, ref1, y2, ref2, phi, psi, ws, ws_bytes=None, stream=None, check=True):
    if ws_bytes is None:
        ws_bytes = ws.numel() * ws.element_size()
    s = lib().corr2d_hetero(plan, _ptr(y1), _ptr(ref1), _ptr(y2), _ptr(ref2), _ptr(phi),
                            _ptr(psi), _ptr(ws), ws_bytes, _stream(stream))
    return _check(s) if check else s


def corr2d_batched(plan, y_base, phi_base, psi_base, ws, ws_bytes=None, stream=None, check=True):
    if ws_bytes is None:
        ws_bytes = ws.numel() * ws.element_size()
    s = lib().corr2d_batched(plan, _ptr(y_base), _ptr(phi_base), _ptr(psi_base), _ptr(ws),
                             ws_bytes, _stream(stream))
    return _check(s) if check else s


# --------------------------------------------------------------------------
# Small conveniences over torch memory (allocation only)
# --------------------------------------------------------------------------
class Plan:
    """Owns a plan handle; destroys it when garbage collected."""

    def __init__(self, desc=None, items=None, **fields):
        if desc is None:
            desc = corr2d_desc_init(**fields)
        self.desc = desc
        if items is None:
            _, self.handle = corr2d_plan(desc)
        else:
            _, self.handle = corr2d_batched_plan(desc, items)
        self.info = corr2d_plan_get_info(self.handle)
        self.ws_bytes = corr2d_workspace_bytes(self.handle)

    def workspace(self, device="cuda"):
        import torch
        return torch.empty(max(self.ws_bytes, 256), dtype=torch.uint8, device=device)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None:
            _lib.corr2d_plan_destroy(h)
            self.handle = None


def upper_aligned_index(i, j, n):
    """Offset of element (i, j), i <= j < n, in the UPPER_ALIGNED layout
    (corr2d_upper_aligned_index of the C header); works on numpy arrays."""
    import numpy as np
    i = np.asarray(i, dtype=np.int64)
    j = np.asarray(j, dtype=np.int64)
    n32 = (int(n) + 31) // 32 * 32
    q, r = i // 32, i % 32
    return i * n32 - 32 * (16 * q * (q - 1) + r * q) + (j - 32 * q)


def upper_aligned_elements(n):
    """Elements of one UPPER_ALIGNED output plane (corr2d_upper_aligned_elements)."""
    return int(upper_aligned_index(n, 32 * (n // 32), n))


def out_elements(layout, n1, n2=0):
    """Elements of one output plane of an n1 x n1 (or n1 x n2) correlation."""
    if layout == "upper_packed":
        return n1 * (n1 + 1) // 2
    if layout == "upper_aligned":
        return upper_aligned_elements(n1)
    return n1 * (n2 or n1)


def homo(y, ref=None, prec="split_bf16", out_dtype=None, layout="full", basis="auto",
         hilbert="noda", norm="noda", norm_value=0.0, flags=0, tile=0, alpha=0.0,
         t_in=None, interp="none", m_out=None, stream=None, split_tol=0.0):
    """Homocorrelation of y (torch, m x n, float64/float32, on the GPU).  With
    interp "linear" or "spline", y's rows were taken at perturbation values
    t_in and are resampled on m_out (default: as many) equidistant values."""
    import torch
    m, n = y.shape
    if interp != "none":
        m = m_out or m
    if out_dtype is None:
        out_dtype = "f64" if prec == "f64" else "f32"
    plan = Plan(m=m, n1=n, n2=0, ld_in1=y.stride(0),
                in_dtype="f64" if y.dtype == torch.float64 else "f32",
                out_dtype=out_dtype, prec=prec, basis=basis, hilbert=hilbert, norm_mode=norm,
                norm_value=norm_value, out_layout=layout, flags=flags, tile=tile,
                scale_alpha=alpha, t_in=t_in, interp=interp, split_tol=split_tol)
    tdt = torch.float64 if out_dtype == "f64" else torch.float32
    numel = out_elements(layout, n)
    phi = torch.empty(numel, dtype=tdt, device=y.device)
    psi = torch.empty(numel, dtype=tdt, device=y.device)
    ws = plan.workspace(y.device)
    corr2d_homo(plan.handle, y, ref, phi, psi, ws, stream=stream)
    if layout == "full":
        phi, psi = phi.view(n, n), psi.view(n, n)
    return phi, psi, plan, ws


def hetero(y1, y2, ref1=None, ref2=None, prec="split_bf16", out_dtype=None, basis="auto",
           hilbert="noda", norm="noda", norm_value=0.0, flags=0, tile=0, alpha=0.0,
           t_in=None, interp="none", m_out=None, stream=None, split_tol=0.0):
    """Heterocorrelation of y1 (m x n1) with y2 (m x n2), both on the GPU;
    interp, t_in, m_out as for homo()."""
    import torch
    m, n1 = y1.shape
    m2, n2 = y2.shape
    if m != m2:
        raise ValueError(f"y1 has {m} perturbation steps and y2 {m2}: both sets need the same")
    if interp != "none":
        m = m_out or m
    if out_dtype is None:
        out_dtype = "f64" if prec == "f64" else "f32"
    plan = Plan(m=m, n1=n1, n2=n2, ld_in1=y1.stride(0), ld_in2=y2.stride(0),
                in_dtype="f64" if y1.dtype == torch.float64 else "f32",
                out_dtype=out_dtype, prec=prec, basis=basis, hilbert=hilbert, norm_mode=norm,
                norm_value=norm_value, out_layout="full", flags=flags, tile=tile,
                scale_alpha=alpha, t_in=t_in, interp=interp, split_tol=split_tol)
    tdt = torch.float64 if out_dtype == "f64" else torch.float32
    phi = torch.empty(n1, n2, dtype=tdt, device=y1.device)
    psi = torch.empty(n1, n2, dtype=tdt, device=y1.device)
    ws = plan.workspace(y1.device)
    corr2d_hetero(plan.handle, y1, ref1, y2, ref2, phi, psi, ws, stream=stream)
    return phi, psi, plan, ws


def selection(ws, plan):
    """The row selection a completed row-selective call left in its
    workspace: (K blocks that carried the low plane, the K-block order), read
    back to the host (int32 record at plan info sel_offset)."""
    info = plan.info if hasattr(plan, "info") else corr2d_plan_get_info(plan)
    if not info.sel_offset:
        return None
    import torch
    nkb = info.k_pad // 16
    rec = ws[info.sel_offset:info.sel_offset + 4 * (1 + nkb)].view(torch.int32).cpu().tolist()
    return rec[0], rec[1:]


def workspace_vector(ws, offset, n):
    """The n doubles at byte offset `offset` of the workspace tensor ws, as a
    float64 view (no copy, no device work)."""
    import torch
    return ws[offset:offset + 8 * n].view(torch.float64)


class Corr2D:
    """What the paper's corr2d() returns (Sec. 3), over device tensors:

    phi, psi    synchronous and asynchronous spectra, in the plan's layout
                (n1 x n2 for the full layout, else one packed triangle)
    ft          phi + i psi as one complex tensor (built on first access)
    ref1, ref2  the reference spectra the call subtracted: the perturbation
                means computed by the centring kernels in FP64, or the
                caller's references (float64 views of the workspace)
    wave1, wave2  the spectral axes given by the caller, else 0 .. n - 1
    plan, ws    the plan and the workspace the views above live in
    """

    def __init__(self, phi, psi, ref1, ref2, wave1, wave2, plan, ws):
        self.phi, self.psi = phi, psi
        self.ref1, self.ref2 = ref1, ref2
        self.wave1, self.wave2 = wave1, wave2
        self.plan, self.ws = plan, ws
        self._ft = None

    @property
    def ft(self):
        if self._ft is None:
            import torch
            self._ft = torch.complex(self.phi, self.psi)
        return self._ft


def corr2d(y1, y2=None, ref1=None, ref2=None, wave1=None, wave2=None, layout="full", **kw):
    """The paper's corr2d() (Sec. 3): the homocorrelation of y1 (m x n1, on
    the GPU), or with y2 (m x n2) the heterocorrelation; ref1 / ref2 replace
    the perturbation means (Eq. (dynspec)).  The other keywords are those of
    homo() and hetero() (prec, basis, hilbert, norm, alpha, interp, ...).
    Asynchronous on the stream like them; returns a Corr2D."""
    import torch
    n1 = y1.shape[1]
    if y2 is None:
        if ref2 is not None or wave2 is not None:
            raise ValueError("ref2 and wave2 belong to a heterocorrelation (give y2)")
        phi, psi, plan, ws = homo(y1, ref=ref1, layout=layout, **kw)
        n2 = n1
    else:
        if layout != "full":
            raise ValueError("a heterocorrelation has the full layout only")
        phi, psi, plan, ws = hetero(y1, y2, ref1=ref1, ref2=ref2, **kw)
        n2 = y2.shape[1]
    info = plan.info
    r1 = workspace_vector(ws, info.ref1_offset, n1)
    r2 = r1 if y2 is None else workspace_vector(ws, info.ref2_offset, n2)
    w1 = wave1 if wave1 is not None else torch.arange(n1, dtype=torch.float64)
    w2 = wave2 if wave2 is not None else (w1 if y2 is None else torch.arange(n2, dtype=torch.float64))
    return Corr2D(phi, psi, r1, r2, w1, w2, plan, ws)
