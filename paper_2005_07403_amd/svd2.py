"""Python binding of libsvd2 (include/svd2.h): argument marshalling only.

Every step of the batched SVD runs in the HIP kernels of ``libsvd2.so``; this
module builds the pointer structs, passes the current HIP stream and maps
status codes to exceptions.  PyTorch is used for device memory and streams
only.  There is no CPU fallback: if the library is missing, every call raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsvd2.so")

SVD2_OK = 0
STATUS = {0: "SVD2_OK", 1: "SVD2_ERR_NULL", 2: "SVD2_ERR_ALIGN", 3: "SVD2_ERR_ALIAS",
          4: "SVD2_ERR_FLAGS", 5: "SVD2_ERR_HIP", 6: "SVD2_ERR_SIZE", 7: "SVD2_NOT_CONVERGED"}
SVD2_BACKSCALE_NONE = 0
SVD2_BACKSCALE_SAFE = 1
SVD2_BACKSCALE_ALL = 2
SVD2_RESCUE_FP64 = 4
SVD2_RESCUE_QUEUE = 8
SVD2_RESCUE_SIGMA = 16
SVD2_NO_UV = 32
SVD2_SINE_FORM = 64
SVD2_RESCUE_TRI = 128

_P = ctypes.c_void_p
REAL_IN = ["a11", "a21", "a12", "a22"]
REAL_OUT = ["u11", "u21", "u12", "u22", "v11", "v21", "v12", "v22", "smax", "smin", "s"]
CPLX_IN = [f"{e}{p}" for e in REAL_IN for p in ("r", "i")]
CPLX_OUT = [f"{e}{p}" for e in REAL_OUT[:8] for p in ("r", "i")] + ["smax", "smin", "s"]


class dsvd2_args(ctypes.Structure):
    _fields_ = [(k, _P) for k in REAL_IN + REAL_OUT]


class zsvd2_args(ctypes.Structure):
    _fields_ = [(k, _P) for k in CPLX_IN + CPLX_OUT]


class ssvd2_args(ctypes.Structure):
    _fields_ = [(k, _P) for k in REAL_IN + REAL_OUT] + [("nrescued", _P)]


class csvd2_args(ctypes.Structure):
    _fields_ = [(k, _P) for k in CPLX_IN + CPLX_OUT] + [("nrescued", _P)]


REAL_URV = ["r11", "r12", "r22"] + REAL_OUT[:8]
CPLX_URV = ["r11", "r12", "r22"] + CPLX_OUT[:16]


class dsvd2_urv(ctypes.Structure):
    _fields_ = [(k, _P) for k in REAL_URV]


class zsvd2_urv(ctypes.Structure):
    _fields_ = [(k, _P) for k in CPLX_URV]


ssvd2_urv, csvd2_urv = dsvd2_urv, zsvd2_urv


class Svd2Error(RuntimeError):
    def __init__(self, fn: str, status: int, hip: int = 0):
        super().__init__(f"{fn}: {STATUS.get(status, status)}" + (f" (hipError {hip})" if hip else ""))
        self.status = status


_lib = None

EXPORTS = ["dsvd2_batch", "zsvd2_batch", "ssvd2_batch", "csvd2_batch", "svd2_workspace_bytes",
           "dsvd2_batch_urv", "zsvd2_batch_urv", "ssvd2_batch_urv", "csvd2_batch_urv",
           "kog_workspace_bytes", "dkog_step", "zkog_step", "skog_step", "ckog_step", "dkog_sweep",
           "zkog_sweep", "skog_sweep", "ckog_sweep", "dkog_solve", "zkog_solve", "skog_solve",
           "ckog_solve", "dkog_norms", "zkog_norms", "skog_norms", "ckog_norms", "kog_last_hip_error",
           "kog_set_fused_blocks_per_cu", "kog_set_tile_rules", "kog_set_three_step_tiles", "kog_batch_workspace_bytes",
           "kog_batch_solve", "kog_workspace_bytes_flags", "kog_set_two_step_tiles",
           "kog_batch_workspace_bytes_flags", "kog_sigma_workspace_bytes", "dkog_sigma", "zkog_sigma",
           "skog_sigma", "ckog_sigma", "kog_svd_workspace_bytes", "dkog_svd", "zkog_svd", "skog_svd",
           "ckog_svd", "dkog_solve_noalloc", "kog_barrier_probe",
           "svd2_set_launch", "svd2_get_launch", "svd2_set_launch_kind", "svd2_get_launch_kind",
           "svd2_status_string", "svd2_last_hip_error",
           "svd2_probe_f64", "svd2_probe_f32", "svd2_stream_probe"]


def lib() -> ctypes.CDLL:
    """Load libsvd2.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing; build it with "
                               "python paper_2005_07403_amd/build.py (no CPU fallback exists)")
        # torch first: its HIP runtime must be the process's one, which the
        # library then shares (loaded the other way round, the library's calls
        # report hipErrorNoDevice once torch has initialised the GPU)
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        sz, ui, i = ctypes.c_size_t, ctypes.c_uint, ctypes.c_int
        L.dsvd2_batch.argtypes = [sz, ctypes.POINTER(dsvd2_args), ui, _P]
        L.zsvd2_batch.argtypes = [sz, ctypes.POINTER(zsvd2_args), ui, _P]
        L.ssvd2_batch.argtypes = [sz, ctypes.POINTER(ssvd2_args), ui, _P, sz, _P]
        L.csvd2_batch.argtypes = [sz, ctypes.POINTER(csvd2_args), ui, _P, sz, _P]
        L.dsvd2_batch_urv.argtypes = [sz, ctypes.POINTER(dsvd2_args), ctypes.POINTER(dsvd2_urv), ui, _P]
        L.zsvd2_batch_urv.argtypes = [sz, ctypes.POINTER(zsvd2_args), ctypes.POINTER(zsvd2_urv), ui, _P]
        L.ssvd2_batch_urv.argtypes = [sz, ctypes.POINTER(ssvd2_args), ctypes.POINTER(ssvd2_urv), ui, _P, sz,
                                      _P]
        L.csvd2_batch_urv.argtypes = [sz, ctypes.POINTER(csvd2_args), ctypes.POINTER(csvd2_urv), ui, _P, sz,
                                      _P]
        for f in ("dsvd2_batch", "zsvd2_batch", "ssvd2_batch", "csvd2_batch", "dsvd2_batch_urv",
                  "zsvd2_batch_urv", "ssvd2_batch_urv", "csvd2_batch_urv"):
            getattr(L, f).restype = i
        L.svd2_workspace_bytes.argtypes = [sz, ui]
        L.svd2_workspace_bytes.restype = sz
        L.svd2_set_launch.argtypes = [i, i]
        L.svd2_set_launch.restype = i
        L.svd2_get_launch.argtypes = [ctypes.POINTER(i), ctypes.POINTER(i)]
        L.svd2_get_launch.restype = None
        L.svd2_set_launch_kind.argtypes = [i, i, i]
        L.svd2_set_launch_kind.restype = i
        L.svd2_get_launch_kind.argtypes = [i, ctypes.POINTER(i), ctypes.POINTER(i)]
        L.svd2_get_launch_kind.restype = None
        L.svd2_status_string.argtypes = [i]
        L.svd2_status_string.restype = ctypes.c_char_p
        L.svd2_last_hip_error.argtypes = []
        L.svd2_last_hip_error.restype = i
        L.svd2_probe_f64.argtypes = [i, sz, _P, _P, _P, _P, _P]
        L.svd2_probe_f32.argtypes = [i, sz, _P, _P, _P, _P, _P]
        L.svd2_probe_f64.restype = i
        L.svd2_probe_f32.restype = i
        L.svd2_stream_probe.argtypes = [i, sz, _P, _P, _P]
        L.svd2_stream_probe.restype = i
        _lib = L
    return _lib


def _check(fn: str, st: int) -> None:
    if st != SVD2_OK:
        raise Svd2Error(fn, st, lib().svd2_last_hip_error() if st == 5 else 0)


def _nbytes(t) -> int:
    """Size in bytes of a caller's device buffer (any dtype); a host tensor
    is refused, since the kernels would dereference its address."""
    if not t.is_cuda:
        raise ValueError("workspace buffers must be device tensors")
    return t.numel() * t.element_size()


def _stream(stream) -> int:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return int(stream)


def _fill(struct_cls, names, ptrs, extra=None):
    a = struct_cls()
    for k, p in zip(names, ptrs):
        setattr(a, k, p)
    if extra:
        for k, p in extra.items():
            setattr(a, k, p)
    return a


# ---------------------------------------------------------------------------
# raw entry points (pointers as ints), same names as the C ABI
# ---------------------------------------------------------------------------

def dsvd2_batch(n: int, ins, outs, flags: int = 0, stream=None) -> None:
    a = _fill(dsvd2_args, REAL_IN + REAL_OUT, list(ins) + list(outs))
    _check("dsvd2_batch", lib().dsvd2_batch(n, ctypes.byref(a), flags, _stream(stream)))


def zsvd2_batch(n: int, ins, outs, flags: int = 0, stream=None) -> None:
    a = _fill(zsvd2_args, CPLX_IN + CPLX_OUT, list(ins) + list(outs))
    _check("zsvd2_batch", lib().zsvd2_batch(n, ctypes.byref(a), flags, _stream(stream)))


def ssvd2_batch(n: int, ins, outs, flags: int = 0, ws: int = 0, ws_bytes: int = 0,
                nrescued: int = 0, stream=None) -> None:
    a = _fill(ssvd2_args, REAL_IN + REAL_OUT, list(ins) + list(outs), {"nrescued": nrescued})
    _check("ssvd2_batch", lib().ssvd2_batch(n, ctypes.byref(a), flags, ws, ws_bytes,
                                            _stream(stream)))


def csvd2_batch(n: int, ins, outs, flags: int = 0, ws: int = 0, ws_bytes: int = 0,
                nrescued: int = 0, stream=None) -> None:
    a = _fill(csvd2_args, CPLX_IN + CPLX_OUT, list(ins) + list(outs), {"nrescued": nrescued})
    _check("csvd2_batch", lib().csvd2_batch(n, ctypes.byref(a), flags, ws, ws_bytes,
                                            _stream(stream)))


def dsvd2_batch_urv(n: int, ins, outs, f, flags: int = 0, stream=None) -> None:
    a = _fill(dsvd2_args, REAL_IN + REAL_OUT, list(ins) + list(outs))
    u = _fill(dsvd2_urv, REAL_URV, list(f))
    _check("dsvd2_batch_urv", lib().dsvd2_batch_urv(n, ctypes.byref(a), ctypes.byref(u), flags, _stream(stream)))


def zsvd2_batch_urv(n: int, ins, outs, f, flags: int = 0, stream=None) -> None:
    a = _fill(zsvd2_args, CPLX_IN + CPLX_OUT, list(ins) + list(outs))
    u = _fill(zsvd2_urv, CPLX_URV, list(f))
    _check("zsvd2_batch_urv", lib().zsvd2_batch_urv(n, ctypes.byref(a), ctypes.byref(u), flags, _stream(stream)))


def ssvd2_batch_urv(n: int, ins, outs, f, flags: int = 0, ws: int = 0, ws_bytes: int = 0,
                    nrescued: int = 0, stream=None) -> None:
    a = _fill(ssvd2_args, REAL_IN + REAL_OUT, list(ins) + list(outs), {"nrescued": nrescued})
    u = _fill(ssvd2_urv, REAL_URV, list(f))
    _check("ssvd2_batch_urv", lib().ssvd2_batch_urv(n, ctypes.byref(a), ctypes.byref(u), flags, ws, ws_bytes,
                                                    _stream(stream)))


def csvd2_batch_urv(n: int, ins, outs, f, flags: int = 0, ws: int = 0, ws_bytes: int = 0,
                    nrescued: int = 0, stream=None) -> None:
    a = _fill(csvd2_args, CPLX_IN + CPLX_OUT, list(ins) + list(outs), {"nrescued": nrescued})
    u = _fill(csvd2_urv, CPLX_URV, list(f))
    _check("csvd2_batch_urv", lib().csvd2_batch_urv(n, ctypes.byref(a), ctypes.byref(u), flags, ws, ws_bytes,
                                                    _stream(stream)))


def svd2_workspace_bytes(n: int, flags: int) -> int:
    return int(lib().svd2_workspace_bytes(n, flags))


def svd2_set_launch(block: int, per_thread: int) -> None:
    _check("svd2_set_launch", lib().svd2_set_launch(block, per_thread))


def svd2_get_launch() -> tuple:
    b, p = ctypes.c_int(), ctypes.c_int()
    lib().svd2_get_launch(ctypes.byref(b), ctypes.byref(p))
    return b.value, p.value


# element type -> launch-shape kind; the "_nouv" kinds are the SVD2_NO_UV kernels
KIND = {"d": 0, "z": 1, "s": 2, "c": 3, "d_nouv": 4, "z_nouv": 5, "s_nouv": 6, "c_nouv": 7}


def svd2_set_launch_kind(kind: str, block: int, per_thread: int) -> None:
    _check("svd2_set_launch_kind", lib().svd2_set_launch_kind(KIND[kind], block, per_thread))


def svd2_get_launch_kind(kind: str) -> tuple:
    b, p = ctypes.c_int(), ctypes.c_int()
    lib().svd2_get_launch_kind(KIND[kind], ctypes.byref(b), ctypes.byref(p))
    return b.value, p.value


TUNING_PATH = os.path.join(HERE, "tuning.json")


def apply_tuning(path: str = TUNING_PATH) -> dict | None:
    """Load the autotuner's table (if present) into the library: launch shapes
    per element type and Kogbetliantz tile rules.  Returns the table."""
    import json
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        tab = json.load(fh)
    for k, (b, p) in tab.get("svd2_launch", {}).items():
        svd2_set_launch_kind(k, int(b), int(p))
    rules = tab.get("kog_tile_rules")
    if rules:
        kog_set_tile_rules([tuple(int(x) for x in r) for r in rules])
    rules2 = tab.get("kog_two_step_tiles")
    if rules2:
        kog_set_two_step_tiles([tuple(int(x) for x in r) for r in rules2])
    return tab


def svd2_probe(op: int, x, y=None, z=None, out=None, stream=None) -> None:
    """op on device tensors x, y, z -> out (see include/svd2.h)."""
    import torch
    fn = lib().svd2_probe_f64 if x.dtype == torch.float64 else lib().svd2_probe_f32
    ptr = lambda t: 0 if t is None else t.data_ptr()
    _check("svd2_probe", fn(op, x.numel(), ptr(x), ptr(y), ptr(z), ptr(out), _stream(stream)))


def svd2_stream_probe(kind: str, ins, outs, stream=None) -> None:
    """The batched kernel's memory pattern without its arithmetic (diagnostic)."""
    pi = (ctypes.c_void_p * len(ins))(*[t.data_ptr() for t in ins])
    po = (ctypes.c_void_p * len(outs))(*[t.data_ptr() for t in outs])
    _check("svd2_stream_probe", lib().svd2_stream_probe(KIND[kind], ins[0].numel(), pi, po, _stream(stream)))


# ---------------------------------------------------------------------------
# tensor convenience: allocate outputs with torch and call the entry point
# ---------------------------------------------------------------------------

def svd2(trains, flags: int = 0, out=None, ws=None, nrescued=None, stream=None, urv=None):
    """Batched SVD of SoA trains (list of 4 real or 8 re/im device tensors of
    one dtype, element order 11, 21, 12, 22).  Returns the list of output
    trains (11 or 19 tensors: U, V, smax, smin, s) in the order of the C ABI;
    with SVD2_NO_UV only [smax, smin, s] (out, if given, holds those three).
    urv: a list of device trains for the phase outputs of the URV
    factorization (the *_batch_urv entry points): 3 (R only) or 11 / 19
    (R, U_+, V_+); then (out, urv) is returned."""
    import torch
    trains = list(trains)
    cplx = len(trains) == 8
    if len(trains) not in (4, 8):
        raise ValueError("expected 4 (real) or 8 (complex) trains")
    dt = trains[0].dtype
    n = trains[0].numel()
    for t in trains:
        if t.dtype != dt or t.numel() != n or not t.is_cuda or not t.is_contiguous():
            raise ValueError("trains must be contiguous device tensors of one dtype and length")
    nout = 3 if flags & SVD2_NO_UV else (19 if cplx else 11)
    if out is None:
        out = [torch.empty(n, dtype=dt, device=trains[0].device) for _ in range(nout)]
    if len(out) != nout:
        raise ValueError(f"expected {nout} output trains")
    for i, t in enumerate(out):
        _like(t, f"output train {i}", dt, trains[0].device, n)
    if nrescued is not None and (not nrescued.is_cuda or nrescued.element_size() != 4 or nrescued.numel() < 1):
        raise ValueError("nrescued: expected a device tensor of 32-bit integers")
    ins = [t.data_ptr() for t in trains]
    outs = [t.data_ptr() for t in out]
    if nout == 3:
        outs = [0] * (16 if cplx else 8) + outs
    fp = None
    if urv is not None:
        nf = 19 if cplx else 11
        if len(urv) not in (3, nf):
            raise ValueError(f"expected 3 or {nf} phase-output trains")
        for i, t in enumerate(urv):
            _like(t, f"phase-output train {i}", dt, trains[0].device, n)
        fp = [t.data_ptr() for t in urv] + [0] * (nf - len(urv))
    if dt == torch.float64:
        if fp is None:
            (zsvd2_batch if cplx else dsvd2_batch)(n, ins, outs, flags, stream)
        else:
            (zsvd2_batch_urv if cplx else dsvd2_batch_urv)(n, ins, outs, fp, flags, stream)
    elif dt == torch.float32:
        wsb = svd2_workspace_bytes(n, flags)
        if wsb and ws is None:
            ws = torch.empty(wsb, dtype=torch.uint8, device=trains[0].device)
        # the library checks the size the caller's buffer really has
        ws_bytes = 0 if ws is None else _nbytes(ws)
        wsp, nr = 0 if ws is None else ws.data_ptr(), 0 if nrescued is None else nrescued.data_ptr()
        if fp is None:
            (csvd2_batch if cplx else ssvd2_batch)(n, ins, outs, flags, wsp, ws_bytes, nr, stream)
        else:
            (csvd2_batch_urv if cplx else ssvd2_batch_urv)(n, ins, outs, fp, flags, wsp, ws_bytes, nr, stream)
    else:
        raise TypeError(dt)
    return out if urv is None else (out, urv)


# ---------------------------------------------------------------------------
# Kogbetliantz entry points
# ---------------------------------------------------------------------------
SVD2_KOG_UNFUSED = 1
SVD2_KOG_GRAPH = 2
SVD2_KOG_TWO_STEP = 4
SVD2_KOG_THREE_STEP = 8
KOG_DTYPE = {"d": 0, "z": 1, "s": 2, "c": 3}
_kog_ready = False


def _kog():
    global _kog_ready
    L = lib()
    if not _kog_ready:
        i, sz, ui, d = ctypes.c_int, ctypes.c_size_t, ctypes.c_uint, ctypes.c_double
        L.kog_workspace_bytes.argtypes = [i, i]
        L.kog_workspace_bytes.restype = sz
        L.kog_workspace_bytes_flags.argtypes = [i, i, ui]
        L.kog_workspace_bytes_flags.restype = sz
        for x in "dzsc":
            getattr(L, f"{x}kog_step").argtypes = [i, _P, i, i, _P, sz, ui, _P]
            getattr(L, f"{x}kog_sweep").argtypes = [i, _P, i, _P, sz, ui, _P]
            getattr(L, f"{x}kog_solve").argtypes = [i, _P, i, d, i, _P, _P, _P, sz, ui, _P]
            getattr(L, f"{x}kog_norms").argtypes = [i, _P, i, _P, _P, _P, sz, _P]
            getattr(L, f"{x}kog_sigma").argtypes = [i, _P, i, _P, _P, sz, _P]
            getattr(L, f"{x}kog_svd").argtypes = [i, _P, i, _P, i, _P, i, _P, d, i, _P, _P, _P, sz, ui, _P]
            for f in ("step", "sweep", "solve", "norms", "sigma", "svd"):
                getattr(L, f"{x}kog_{f}").restype = i
        L.kog_svd_workspace_bytes.argtypes = [i, i, ui]
        L.kog_svd_workspace_bytes.restype = sz
        L.kog_sigma_workspace_bytes.argtypes = [i, i]
        L.kog_sigma_workspace_bytes.restype = sz
        L.kog_last_hip_error.restype = i
        L.kog_set_fused_blocks_per_cu.argtypes = [i]
        L.kog_set_fused_blocks_per_cu.restype = i
        L.dkog_solve_noalloc.argtypes = [i, _P, i, d, i, _P, _P, ui, _P]
        L.dkog_solve_noalloc.restype = i
        L.kog_barrier_probe.argtypes = [i, i, _P, _P, sz, _P]
        L.kog_barrier_probe.restype = i
        _kog_ready = True
    return L


def _kog_check(fn: str, st: int) -> None:
    if st not in (SVD2_OK, 7):
        raise Svd2Error(fn, st, _kog().kog_last_hip_error() if st == 5 else 0)


def kog_kind(A) -> str:
    """'d', 'z', 's' or 'c' for a square column-major torch tensor."""
    import torch
    return {torch.float64: "d", torch.complex128: "z", torch.float32: "s",
            torch.complex64: "c"}[A.dtype]


def kog_workspace_bytes(N: int, kind: str, flags: int = 0) -> int:
    return int(_kog().kog_workspace_bytes_flags(N, KOG_DTYPE[kind], flags))


def _kog_args(A):
    """A: (N, N) device tensor stored column-major (A.t() contiguous, or a
    Fortran-ordered view).  Returns N, lda, data pointer."""
    if not A.is_cuda:
        raise ValueError("the matrix must be a device tensor")
    N = A.shape[0]
    if A.dim() != 2 or A.shape[1] != N or A.stride(0) != 1:
        raise ValueError("A must be a square column-major device tensor (stride(0) == 1)")
    return N, A.stride(1), A.data_ptr()


def _like(t, name: str, dtype, device, numel: int) -> None:
    """A caller's output tensor must have the element type, device and size
    the library will write (it cannot check them itself)."""
    if t.dtype != dtype or t.device != device or not t.is_contiguous() or t.numel() < numel:
        raise ValueError(f"{name}: expected a contiguous {dtype} tensor of at least {numel} elements on {device}")


def kog_workspace(A, flags: int = 0):
    import torch
    N = A.shape[0]
    return torch.empty(kog_workspace_bytes(N, kog_kind(A), flags), dtype=torch.uint8, device=A.device)


def kog_step(A, t: int, ws=None, flags: int = 0, stream=None) -> None:
    k = kog_kind(A)
    N, lda, ptr = _kog_args(A)
    ws = kog_workspace(A, flags) if ws is None else ws
    _kog_check(f"{k}kog_step", getattr(_kog(), f"{k}kog_step")(N, ptr, lda, t, ws.data_ptr(),
                                                              _nbytes(ws), flags, _stream(stream)))


def kog_sweep(A, ws=None, flags: int = 0, stream=None) -> None:
    k = kog_kind(A)
    N, lda, ptr = _kog_args(A)
    ws = kog_workspace(A, flags) if ws is None else ws
    _kog_check(f"{k}kog_sweep", getattr(_kog(), f"{k}kog_sweep")(N, ptr, lda, ws.data_ptr(),
                                                                _nbytes(ws), flags, _stream(stream)))


def kog_solve(A, tol: float = 1e-14, max_sweeps: int = 40, ws=None, flags: int = 0,
              stream=None) -> dict:
    """Sweeps until off(A) < tol ||A_0||_F.  Returns status, sweeps, off_rel."""
    k = kog_kind(A)
    N, lda, ptr = _kog_args(A)
    ws = kog_workspace(A, flags) if ws is None else ws
    sw, off = ctypes.c_int(), ctypes.c_double()
    st = getattr(_kog(), f"{k}kog_solve")(N, ptr, lda, tol, max_sweeps, ctypes.byref(sw),
                                          ctypes.byref(off), ws.data_ptr(), _nbytes(ws), flags,
                                          _stream(stream))
    _kog_check(f"{k}kog_solve", st)
    return dict(status=st, sweeps=sw.value, off_rel=off.value)


def kog_solve_noalloc(A, tol: float = 1e-14, max_sweeps: int = 40, flags: int = 0,
                      stream=None) -> dict:
    """kog_solve of a real FP64 matrix with the library's own fixed device
    workspace (no allocation by the library or here).  flags: 0 (fused) or
    SVD2_KOG_UNFUSED.  Returns status, sweeps, off_rel."""
    if kog_kind(A) != "d":
        raise ValueError("kog_solve_noalloc takes a real float64 matrix")
    N, lda, ptr = _kog_args(A)
    sw, off = ctypes.c_int(), ctypes.c_double()
    st = _kog().dkog_solve_noalloc(N, ptr, lda, tol, max_sweeps, ctypes.byref(sw), ctypes.byref(off), flags,
                                   _stream(stream))
    _kog_check("dkog_solve_noalloc", st)
    return dict(status=st, sweeps=sw.value, off_rel=off.value)


def kog_barrier_probe(nbar: int, blocks: int, ws, violations=None, stream=None) -> None:
    """Diagnostic: one cooperative launch of `blocks` workgroups passing nbar
    grid barriers (ws: a device uint8 tensor of >= 256 + 4096 * 64 bytes);
    violations (optional device int32 tensor of one element, zeroed by the
    caller) receives the count of epoch-check failures."""
    v = 0 if violations is None else violations.data_ptr()
    if violations is not None:
        _like(violations, "violations", violations.dtype, violations.device, 1)
    _kog_check("kog_barrier_probe", _kog().kog_barrier_probe(nbar, blocks, v, ws.data_ptr(), _nbytes(ws),
                                                             _stream(stream)))


def kog_sigma(A, out=None, ws=None, stream=None):
    """|diag(A)| sorted into descending order, on the device (the singular
    values once A has converged).  Returns a real tensor of length N."""
    import torch
    k = kog_kind(A)
    N, lda, ptr = _kog_args(A)
    real = torch.float64 if k in "dz" else torch.float32
    out = torch.empty(N, dtype=real, device=A.device) if out is None else out
    _like(out, "out", real, A.device, N)
    if ws is None:
        ws = torch.empty(max(int(_kog().kog_sigma_workspace_bytes(N, KOG_DTYPE[k])), 1), dtype=torch.uint8,
                         device=A.device)
    _kog_check(f"{k}kog_sigma", getattr(_kog(), f"{k}kog_sigma")(N, ptr, lda, out.data_ptr(), ws.data_ptr(),
                                                                  _nbytes(ws), _stream(stream)))
    return out


def kog_svd_workspace_bytes(N: int, kind: str, flags: int = 0) -> int:
    return int(_kog().kog_svd_workspace_bytes(N, KOG_DTYPE[kind], flags))


def kog_svd(A, tol: float = 1e-14, max_sweeps: int = 40, U=None, V=None, sigma=None, ws=None,
            flags: int = 0, stream=None) -> dict:
    """SVD A_0 = U diag(sigma) V^* with the transformations accumulated; A is
    replaced by the final iterate.  U, V (column-major, allocated if None)
    and sigma (descending) are returned with status, sweeps, off_rel."""
    import torch
    k = kog_kind(A)
    N, lda, ptr = _kog_args(A)
    if U is None:
        U = torch.empty((N, N), dtype=A.dtype, device=A.device).t()
    if V is None:
        V = torch.empty((N, N), dtype=A.dtype, device=A.device).t()
    for X, name in ((U, "U"), (V, "V")):
        if X.dtype != A.dtype or X.device != A.device or tuple(X.shape) != (N, N):
            raise ValueError(f"{name}: expected an {N}x{N} {A.dtype} tensor on {A.device}")
    _, ldu, uptr = _kog_args(U)
    _, ldv, vptr = _kog_args(V)
    real = torch.float64 if k in "dz" else torch.float32
    sigma = torch.empty(N, dtype=real, device=A.device) if sigma is None else sigma
    _like(sigma, "sigma", real, A.device, N)
    if ws is None:
        ws = torch.empty(kog_svd_workspace_bytes(N, k, flags), dtype=torch.uint8, device=A.device)
    sw, off = ctypes.c_int(), ctypes.c_double()
    st = getattr(_kog(), f"{k}kog_svd")(N, ptr, lda, uptr, ldu, vptr, ldv, sigma.data_ptr(), tol, max_sweeps,
                                        ctypes.byref(sw), ctypes.byref(off), ws.data_ptr(), _nbytes(ws), flags,
                                        _stream(stream))
    _kog_check(f"{k}kog_svd", st)
    return dict(status=st, sweeps=sw.value, off_rel=off.value, U=U, V=V, sigma=sigma)


def kog_norms(A, ws=None, stream=None):
    k = kog_kind(A)
    N, lda, ptr = _kog_args(A)
    ws = kog_workspace(A) if ws is None else ws
    o, t = ctypes.c_double(), ctypes.c_double()
    _kog_check(f"{k}kog_norms", getattr(_kog(), f"{k}kog_norms")(
        N, ptr, lda, ctypes.byref(o), ctypes.byref(t), ws.data_ptr(), _nbytes(ws), _stream(stream)))
    return o.value, t.value


def kog_set_fused_blocks_per_cu(per_cu: int) -> None:
    _kog_check("kog_set_fused_blocks_per_cu", _kog().kog_set_fused_blocks_per_cu(per_cu))


class kog_problem(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int), ("N", ctypes.c_int), ("lda", ctypes.c_int), ("A", _P),
                ("tol", ctypes.c_double), ("max_sweeps", ctypes.c_int), ("status", ctypes.c_int),
                ("sweeps", ctypes.c_int), ("off_rel", ctypes.c_double)]


_batch_ready = False


def _batch():
    global _batch_ready
    L = _kog()
    if not _batch_ready:
        L.kog_batch_workspace_bytes.argtypes = [ctypes.c_int, ctypes.POINTER(kog_problem)]
        L.kog_batch_workspace_bytes.restype = ctypes.c_size_t
        L.kog_batch_workspace_bytes_flags.argtypes = [ctypes.c_int, ctypes.POINTER(kog_problem), ctypes.c_uint]
        L.kog_batch_workspace_bytes_flags.restype = ctypes.c_size_t
        L.kog_batch_solve.argtypes = [ctypes.c_int, ctypes.POINTER(kog_problem), _P, ctypes.c_size_t,
                                      ctypes.c_uint, _P]
        L.kog_batch_solve.restype = ctypes.c_int
        L.kog_set_tile_rules.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                         ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
        L.kog_set_tile_rules.restype = ctypes.c_int
        L.kog_set_two_step_tiles.argtypes = L.kog_set_tile_rules.argtypes
        L.kog_set_two_step_tiles.restype = ctypes.c_int
        L.kog_set_three_step_tiles.argtypes = L.kog_set_tile_rules.argtypes
        L.kog_set_three_step_tiles.restype = ctypes.c_int
        _batch_ready = True
    return L


def kog_set_tile_rules(rules) -> None:
    """rules: list of (max_order, kc, lc) with increasing max_order; [] = default."""
    n = len(rules)
    arr = lambda i: (ctypes.c_int * max(n, 1))(*[r[i] for r in rules])
    _kog_check("kog_set_tile_rules", _batch().kog_set_tile_rules(n, arr(0), arr(1), arr(2)))


def kog_set_two_step_tiles(rules) -> None:
    """rules: list of (max_order, wavefronts per workgroup, lc) with increasing
    max_order, for the two-step kernel; [] = default."""
    n = len(rules)
    arr = lambda i: (ctypes.c_int * max(n, 1))(*[r[i] for r in rules])
    _kog_check("kog_set_two_step_tiles", _batch().kog_set_two_step_tiles(n, arr(0), arr(1), arr(2)))


def kog_set_three_step_tiles(rules) -> None:
    """rules: list of (max_order, wavefronts per workgroup, lc) with increasing
    max_order, for the three-step kernel; [] = default."""
    n = len(rules)
    arr = lambda i: (ctypes.c_int * max(n, 1))(*[r[i] for r in rules])
    _kog_check("kog_set_three_step_tiles", _batch().kog_set_three_step_tiles(n, arr(0), arr(1), arr(2)))


def kog_batch_solve(mats, tols, max_sweeps=40, flags: int = 0, ws=None, stream=None) -> list:
    """Solve many problems at once.  mats: list of square column-major device
    tensors (float64, complex128, float32, complex64); tols: one per problem
    (or a scalar).  Returns a list of dicts (status, sweeps, off_rel)."""
    import torch
    n = len(mats)
    if not hasattr(tols, "__len__"):
        tols = [tols] * n
    if not hasattr(max_sweeps, "__len__"):
        max_sweeps = [max_sweeps] * n
    probs = (kog_problem * max(n, 1))()
    for i, A in enumerate(mats):
        N, lda, ptr = _kog_args(A)
        probs[i].dtype = KOG_DTYPE[kog_kind(A)]
        probs[i].N, probs[i].lda, probs[i].A = N, lda, ptr
        probs[i].tol, probs[i].max_sweeps = float(tols[i]), int(max_sweeps[i])
    L = _batch()
    wsb = int(L.kog_batch_workspace_bytes_flags(n, probs, flags))
    if ws is None:
        ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device=mats[0].device)
    st = L.kog_batch_solve(n, probs, ws.data_ptr(), _nbytes(ws), flags, _stream(stream))
    _kog_check("kog_batch_solve", st)
    return [dict(status=probs[i].status, sweeps=probs[i].sweeps, off_rel=probs[i].off_rel)
            for i in range(n)]
