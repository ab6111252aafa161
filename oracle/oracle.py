"""ctypes binding of the CPU oracle (``liboracle.so``).

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` use it; the product package never imports it.

Matrices are passed as numpy arrays of shape (4, n) in the element order
11, 21, 12, 22 (the record layout of section 8 of arXiv:2005.07403); complex
input is a complex array and is split into the SoA real/imaginary trains of
section 3 before the call.  Results come back in the same shape.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

REF, MIRROR = 0, 1
POLICY = {"ref": REF, "mirror": MIRROR}
BACKSCALE = {"none": 0, "safe": 1, "all": 2}
TRACE_FIELDS = ["s", "c", "r", "r11", "r12", "r22", "mt", "ca", "x", "y", "t2",
                "tphi", "sec2phi", "cphi", "tpsi", "sec2psi", "cpsi", "smax",
                "smin", "n1", "n2", "rescued"]

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise FileNotFoundError(f"{LIB_PATH} missing: run python oracle/build.py")
        _lib = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        for name in ("oracle_dsvd2", "oracle_zsvd2"):
            f = getattr(_lib, name)
            f.argtypes = [ctypes.c_size_t, P, P, ctypes.c_int, ctypes.c_int, ctypes.c_int]
            f.restype = ctypes.c_int
        for name in ("oracle_ssvd2", "oracle_csvd2"):
            f = getattr(_lib, name)
            f.argtypes = [ctypes.c_size_t, P, P, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                          P, ctypes.c_int]
            f.restype = ctypes.c_int
        _lib.oracle_trace_d.argtypes = [P, ctypes.c_int, ctypes.c_int, P]
        _lib.oracle_trace_s.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, P]
        for name in ("oracle_urv_d", "oracle_urv_s"):
            f = getattr(_lib, name)
            f.argtypes = [ctypes.c_size_t, ctypes.c_int, P, P, ctypes.c_int, ctypes.c_int]
            f.restype = ctypes.c_int
        for name in ("oracle_metrics_d", "oracle_metrics_s"):
            f = getattr(_lib, name)
            f.argtypes = [ctypes.c_size_t, ctypes.c_int, P, P, P, P, P, P, ctypes.c_int]
            f.restype = ctypes.c_int
    return _lib


def _ptrs(arrays):
    arr = (ctypes.c_void_p * len(arrays))(*[a.ctypes.data for a in arrays])
    return arr


def split(A: np.ndarray, real_dtype) -> list:
    """(4, n) real or complex -> list of contiguous SoA trains."""
    if np.iscomplexobj(A):
        out = []
        for e in range(4):
            out.append(np.ascontiguousarray(A[e].real, dtype=real_dtype))
            out.append(np.ascontiguousarray(A[e].imag, dtype=real_dtype))
        return out
    return [np.ascontiguousarray(A[e], dtype=real_dtype) for e in range(4)]


def join(trains: list, cplx: bool) -> np.ndarray:
    """SoA trains -> (4, n) array (complex when cplx)."""
    if cplx:
        return np.stack([_cx(trains[2 * e], trains[2 * e + 1]) for e in range(4)])
    return np.stack(trains[:4])


def _cx(re, im):
    out = np.empty(re.shape, dtype=np.complex128 if re.dtype == np.float64 else np.complex64)
    out.real = re
    out.imag = im
    return out


def svd2(A: np.ndarray, dtype=np.float64, policy: str = "mirror", backscale: str = "none",
         rescue: bool = False, nthreads: int = 0, cplx: bool | None = None) -> dict:
    """Run the oracle over a batch.

    A: (4, n) array (real or complex), element order 11, 21, 12, 22.
    dtype: np.float64 or np.float32 (the arithmetic precision).
    Returns dict(U=(4,n), V=(4,n), smax, smin, s, flagged, trains=list of output arrays).
    """
    if cplx is None:
        cplx = bool(np.iscomplexobj(A))
    dtype = np.dtype(dtype)
    if cplx and not np.iscomplexobj(A):
        A = A.astype(np.complex128 if dtype == np.float64 else np.complex64)
    n = A.shape[1]
    ins = split(A, dtype)
    nout = 19 if cplx else 11
    outs = [np.empty(n, dtype=dtype) for _ in range(nout)]
    L = lib()
    flagged = np.zeros(n, dtype=np.uint8)
    pin, pout = _ptrs(ins), _ptrs(outs)
    pol = POLICY[policy]
    bs = BACKSCALE[backscale]
    if dtype == np.float64:
        f = L.oracle_zsvd2 if cplx else L.oracle_dsvd2
        f(n, pin, pout, pol, bs, nthreads)
    elif dtype == np.float32:
        f = L.oracle_csvd2 if cplx else L.oracle_ssvd2
        f(n, pin, pout, pol, bs, int(rescue), flagged.ctypes.data, nthreads)
    else:
        raise ValueError(dtype)
    # rescue: False/0 none, True/1 FP64 tail, 2 sigma quotient only, 3 FP64 triangle + FP32 assembly
    k = 16 if cplx else 8
    return dict(U=join(outs[0:k // 2], cplx), V=join(outs[k // 2:k], cplx),
                smax=outs[k], smin=outs[k + 1], s=outs[k + 2], flagged=flagged,
                trains=outs, inputs=ins)


SINE = 16  # ORACLE_SINE: U by the sine form of eq. (31)


def run_trains(ins: list, cplx: bool, dtype, policy="mirror", backscale="none",
               rescue=False, nthreads=0, form="tangent") -> tuple:
    """Same as svd2 but on SoA trains directly; returns (outs, flagged).
    form: "tangent" (eq. (29)) or "sine" (eq. (31))."""
    dtype = np.dtype(dtype)
    n = ins[0].shape[0]
    nout = 19 if cplx else 11
    outs = [np.empty(n, dtype=dtype) for _ in range(nout)]
    flagged = np.zeros(n, dtype=np.uint8)
    L = lib()
    pin, pout = _ptrs(ins), _ptrs(outs)
    pol = POLICY[policy] | (SINE if form == "sine" else 0)
    if dtype == np.float64:
        (L.oracle_zsvd2 if cplx else L.oracle_dsvd2)(n, pin, pout, pol, BACKSCALE[backscale], nthreads)
    else:
        (L.oracle_csvd2 if cplx else L.oracle_ssvd2)(n, pin, pout, pol, BACKSCALE[backscale], int(rescue),
                                                    flagged.ctypes.data, nthreads)
    return outs, flagged


def trace(a, cplx: bool, dtype=np.float64, policy="mirror", rescue=False) -> dict:
    """Intermediates of one matrix.  a: 4 (real) or 8 (complex) components in
    the order a11[r,i], a21[r,i], a12[r,i], a22[r,i]."""
    dtype = np.dtype(dtype)
    a = np.ascontiguousarray(a, dtype=dtype)
    tr = np.zeros(len(TRACE_FIELDS), dtype=np.float64)
    L = lib()
    if dtype == np.float64:
        L.oracle_trace_d(a.ctypes.data, int(cplx), POLICY[policy], tr.ctypes.data)
    else:
        L.oracle_trace_s(a.ctypes.data, int(cplx), POLICY[policy], int(rescue), tr.ctypes.data)
    return dict(zip(TRACE_FIELDS, tr.tolist()))


def metrics(ins: list, outs: list, cplx: bool, nthreads: int = 0) -> dict:
    """kappa, rho, delta, eta of eqs. (32)-(35) per lane, in binary128."""
    n = ins[0].shape[0]
    res = {k: np.empty(n, dtype=np.float64) for k in ("kappa", "rho", "delta", "eta")}
    L = lib()
    f = L.oracle_metrics_d if ins[0].dtype == np.float64 else L.oracle_metrics_s
    f(n, int(cplx), _ptrs(ins), _ptrs(outs), res["kappa"].ctypes.data, res["rho"].ctypes.data,
      res["delta"].ctypes.data, res["eta"].ctypes.data, nthreads)
    return res


# ---------------------------------------------------------------------------
# Kogbetliantz oracle
# ---------------------------------------------------------------------------

def _kog_lib():
    L = lib()
    if not getattr(L, "_kog_ready", False):
        P, i, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
        L.oracle_kog_pairs.argtypes = [i, i, P]
        for s in ("d", "z", "s", "c"):
            getattr(L, f"oracle_kog_step_{s}").argtypes = [i, P, i, i]
            getattr(L, f"oracle_kog_solve_{s}").argtypes = [i, P, i, d, i, P, P, P]
            getattr(L, f"oracle_kog_solve_{s}").restype = i
        for s in "ds":
            getattr(L, f"oracle_kog_svd_{s}").argtypes = [i, P, i, P, i, P, i, P, i, d, i, P, P]
            getattr(L, f"oracle_kog_svd_{s}").restype = i
        L.oracle_kog_norms_d.argtypes = [i, P, i, i, P, P]
        L.oracle_kog_norms_s.argtypes = [i, P, i, i, P, P]
        L._kog_ready = True
    return L


def kog_pairs(N: int, t: int) -> np.ndarray:
    out = np.zeros((N // 2, 2), dtype=np.int32)
    _kog_lib().oracle_kog_pairs(N, t, out.ctypes.data)
    return out


def _kog_buf(A: np.ndarray):
    """column-major buffer: real -> float64/float32, complex -> interleaved float64"""
    assert A.flags.f_contiguous and A.shape[0] == A.shape[1]
    if np.iscomplexobj(A):
        flat = A.ravel(order="F")
        if A.dtype == np.complex128:
            return flat.view(np.float64), "z"
        return flat.view(np.float32), "c"
    return A, ("d" if A.dtype == np.float64 else "s")


def kog_step(A: np.ndarray, t: int) -> None:
    """One step in place (A Fortran-ordered, complex128, float64 or float32)."""
    buf, s = _kog_buf(A)
    getattr(_kog_lib(), f"oracle_kog_step_{s}")(A.shape[0], buf.ctypes.data, A.shape[0], t)


def kog_norms(A: np.ndarray):
    L = _kog_lib()
    off2, tot2 = ctypes.c_double(), ctypes.c_double()
    buf, s = _kog_buf(A)
    if s in ("s", "c"):
        L.oracle_kog_norms_s(A.shape[0], buf.ctypes.data, A.shape[0], int(s == "c"),
                             ctypes.byref(off2), ctypes.byref(tot2))
    else:
        L.oracle_kog_norms_d(A.shape[0], buf.ctypes.data, A.shape[0], int(s == "z"),
                             ctypes.byref(off2), ctypes.byref(tot2))
    return off2.value, tot2.value


def kog_svd(A: np.ndarray, tol: float = 1e-14, max_sweeps: int = 40) -> dict:
    """SVD A_0 = U diag(sigma) V^* by the Kogbetliantz method with accumulated
    transformations (at least one sweep; sigma descending, ties by index, U
    and V columns permuted alike).  A (Fortran-ordered) is replaced by the
    final iterate.  Returns status, sweeps, off_rel, U, V, sigma."""
    N = A.shape[0]
    buf, s = _kog_buf(A)
    U = np.zeros((N, N), dtype=A.dtype, order="F")
    V = np.zeros((N, N), dtype=A.dtype, order="F")
    ub, _ = _kog_buf(U)
    vb, _ = _kog_buf(V)
    rdt = np.float64 if s in "dz" else np.float32
    sig = np.zeros(N, dtype=rdt)
    sw, off = ctypes.c_int(), ctypes.c_double()
    st = getattr(_kog_lib(), f"oracle_kog_svd_{'d' if s in 'dz' else 's'}")(
        N, buf.ctypes.data, N, ub.ctypes.data, N, vb.ctypes.data, N, sig.ctypes.data, int(s in "zc"),
        tol, max_sweeps, ctypes.byref(sw), ctypes.byref(off))
    return dict(status=st, sweeps=sw.value, off_rel=off.value, U=U, V=V, sigma=sig)


def kog_solve(A: np.ndarray, tol: float = 1e-14, max_sweeps: int = 40) -> dict:
    """Full solve in place.  Returns status, sweeps, off_rel, history, sigma
    (the diagonal, sorted in descending order)."""
    buf, s = _kog_buf(A)
    sw, off = ctypes.c_int(), ctypes.c_double()
    hist = np.full(max_sweeps + 1, np.nan)
    st = getattr(_kog_lib(), f"oracle_kog_solve_{s}")(A.shape[0], buf.ctypes.data, A.shape[0], tol,
                                                      max_sweeps, ctypes.byref(sw), ctypes.byref(off),
                                                      hist.ctypes.data)
    sig = np.sort(np.abs(np.diag(A)).astype(np.float64))[::-1]
    return dict(status=st, sweeps=sw.value, off_rel=off.value, history=hist[: sw.value + 1],
                sigma=sig)


def urv(A: np.ndarray, dtype=np.float64, policy: str = "mirror", nthreads: int = 0,
        cplx: bool | None = None) -> dict:
    """Phase outputs of the URV factorization (section 2.2, eqs. (9) and (11)):
    R = [[r11, r12], [0, r22]] of the scaled matrix A^ = 2^s A and its unitary
    factors, A^ = U_+ R V_+^*.  Same pipeline and arguments as svd2().
    Returns dict(r11, r12, r22, Up=(4, n), Vp=(4, n), trains=list of the
    output arrays in the order r11, r12, r22, U_+, V_+)."""
    if cplx is None:
        cplx = bool(np.iscomplexobj(A))
    dtype = np.dtype(dtype)
    if cplx and not np.iscomplexobj(A):
        A = A.astype(np.complex128 if dtype == np.float64 else np.complex64)
    n = A.shape[1]
    ins = split(A, dtype)
    nf = 19 if cplx else 11
    outs = [np.empty(n, dtype=dtype) for _ in range(nf)]
    L = lib()
    f = L.oracle_urv_d if dtype == np.float64 else L.oracle_urv_s
    if dtype not in (np.float64, np.float32):
        raise ValueError(dtype)
    f(n, int(cplx), _ptrs(ins), _ptrs(outs), POLICY[policy], nthreads)
    k = 8 if cplx else 4
    return dict(r11=outs[0], r12=outs[1], r22=outs[2], Up=join(outs[3:3 + k], cplx),
                Vp=join(outs[3 + k:3 + 2 * k], cplx), trains=outs)
