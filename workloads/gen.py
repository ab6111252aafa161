"""Input generators.

Matrices are returned as numpy arrays of shape (4, n) in the element order
11, 21, 12, 22 (the record order of section 8 of arXiv:2005.07403), real or
complex.  ``to_trains`` splits them into the SoA "box trains" of section 3
(one contiguous array per element and per real/imaginary part).

The paper measured on random 64-bit patterns read from /dev/urandom (section
8); that private file is not available, so these seeded laws stand in for it:

* ``uniform_real``  -- entries i.i.d. U[-1, 1] (the small parity workload);
* ``scaled_law``    -- every real/imaginary part is +-m 2^e, m ~ U[1, 2),
  e ~ UniformInt[emin, emax], with a fraction of lanes replaced by special
  matrices (zero, rank one, diagonal, upper triangular, near the largest finite
  value, subnormal);
* ``random_bits``   -- the paper's own law: uniform random bit patterns,
  non-finite values redrawn.
"""
from __future__ import annotations

import numpy as np

SEED_BASE = 0x200507403

KINDS = ("zero", "rank_one", "diagonal", "upper_triangular", "near_max", "subnormal")

_FMT = {
    np.dtype(np.float64): dict(mant_bits=52, tm_exp=-1074, maxv=np.finfo(np.float64).max,
                               uint=np.uint64),
    np.dtype(np.float32): dict(mant_bits=23, tm_exp=-149, maxv=np.finfo(np.float32).max,
                               uint=np.uint32),
}


def _mant(rng, size, dtype):
    """m ~ U[1, 2) on the grid of the format (exact in dtype)."""
    f = _FMT[np.dtype(dtype)]
    k = rng.integers(0, 1 << f["mant_bits"], size=size, dtype=np.int64)
    return (1.0 + np.ldexp(k.astype(np.float64), -f["mant_bits"])).astype(dtype)


def _signed_pow2(rng, size, dtype, emin, emax):
    m = _mant(rng, size, dtype)
    e = rng.integers(emin, emax + 1, size=size)
    sign = np.where(rng.random(size) < 0.5, -1.0, 1.0).astype(dtype)
    return (sign * np.ldexp(m, e).astype(dtype)).astype(dtype)


def uniform_real(n: int, seed: int, dtype=np.float64) -> np.ndarray:
    """(4, n) entries i.i.d. uniform in [-1, 1]."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=(4, n)).astype(dtype)


def scaled_law(n: int, seed: int, cplx: bool, dtype=np.float64, emin: int | None = None,
               emax: int | None = None, special_frac: float = 0.01,
               return_kinds: bool = False):
    """(4, n) matrices with every component +-m 2^e.

    dtype float64: e in [-1000, 1000] by default; float32: e in [-120, 120].
    special_frac of the lanes (each lane independently) is replaced by one of
    KINDS, uniformly.  With return_kinds, also returns an int8 array holding
    the kind index per lane (-1 for ordinary lanes).
    """
    dtype = np.dtype(dtype)
    f = _FMT[dtype]
    if emin is None or emax is None:
        emin, emax = (-1000, 1000) if dtype == np.float64 else (-120, 120)
    rng = np.random.default_rng(seed)
    re = _signed_pow2(rng, (4, n), dtype, emin, emax)
    im = _signed_pow2(rng, (4, n), dtype, emin, emax) if cplx else None
    kinds = np.full(n, -1, dtype=np.int8)
    if special_frac > 0:
        sel = np.nonzero(rng.random(n) < special_frac)[0]
        kind = rng.integers(0, len(KINDS), size=sel.size)
        kinds[sel] = kind
        half = (emax - emin) // 4
        for kidx, name in enumerate(KINDS):
            lanes = sel[kind == kidx]
            m = lanes.size
            if m == 0:
                continue
            if name == "zero":
                re[:, lanes] = 0
                if cplx:
                    im[:, lanes] = 0
            elif name == "rank_one":
                # a_ij = u_i conj(v_j), entries of u and v from the same law with a
                # narrower exponent range, formed in the working precision
                lo, hi = -half, half
                u = _signed_pow2(rng, (2, m), dtype, lo, hi)
                v = _signed_pow2(rng, (2, m), dtype, lo, hi)
                if cplx:
                    ui = _signed_pow2(rng, (2, m), dtype, lo, hi)
                    vi = _signed_pow2(rng, (2, m), dtype, lo, hi)
                    cdt = np.complex128 if dtype == np.float64 else np.complex64
                    uc = (u + 1j * ui).astype(cdt)
                    vc = (v + 1j * vi).astype(cdt)
                    a = np.stack([uc[0] * np.conj(vc[0]), uc[1] * np.conj(vc[0]),
                                  uc[0] * np.conj(vc[1]), uc[1] * np.conj(vc[1])]).astype(cdt)
                    re[:, lanes] = a.real
                    im[:, lanes] = a.imag
                else:
                    re[:, lanes] = np.stack([u[0] * v[0], u[1] * v[0], u[0] * v[1],
                                             u[1] * v[1]]).astype(dtype)
            elif name == "diagonal":
                re[1, lanes] = 0
                re[2, lanes] = 0
                if cplx:
                    im[1, lanes] = 0
                    im[2, lanes] = 0
            elif name == "upper_triangular":
                re[1, lanes] = 0
                if cplx:
                    im[1, lanes] = 0
            elif name == "near_max":
                # |x| = MAX (1 - u 2^-4), u ~ U[0, 1), random sign
                for arr in ([re, im] if cplx else [re]):
                    u = rng.random((4, m))
                    sgn = np.where(rng.random((4, m)) < 0.5, -1.0, 1.0)
                    arr[:, lanes] = (sgn * (f["maxv"] * (1.0 - u / 16.0))).astype(dtype)
            elif name == "subnormal":
                # +-k TRUE_MIN, k ~ U[1, 2^mant_bits)
                for arr in ([re, im] if cplx else [re]):
                    k = rng.integers(1, 1 << f["mant_bits"], size=(4, m), dtype=np.int64)
                    sgn = np.where(rng.random((4, m)) < 0.5, -1.0, 1.0)
                    arr[:, lanes] = (sgn * np.ldexp(k.astype(np.float64), f["tm_exp"])).astype(dtype)
    if cplx:
        cdt = np.complex128 if dtype == np.float64 else np.complex64
        A = np.empty((4, n), dtype=cdt)
        A.real = re
        A.imag = im
    else:
        A = re
    return (A, kinds) if return_kinds else A


def random_bits(n: int, seed: int, cplx: bool, dtype=np.float64) -> np.ndarray:
    """The paper's law (section 8): uniform random bit patterns, with every
    non-finite value redrawn."""
    dtype = np.dtype(dtype)
    f = _FMT[dtype]
    rng = np.random.default_rng(seed)
    ncomp = 8 if cplx else 4
    bits = rng.integers(0, np.iinfo(f["uint"]).max, size=(ncomp, n), dtype=f["uint"],
                        endpoint=True)
    vals = bits.view(dtype)
    bad = ~np.isfinite(vals)
    while bad.any():
        nb = rng.integers(0, np.iinfo(f["uint"]).max, size=int(bad.sum()), dtype=f["uint"],
                          endpoint=True)
        vals[bad] = nb.view(dtype)
        bad = ~np.isfinite(vals)
    if cplx:
        cdt = np.complex128 if dtype == np.float64 else np.complex64
        A = np.empty((4, n), dtype=cdt)
        A.real = vals[0::2]
        A.imag = vals[1::2]
        return A
    return vals.copy()


def to_trains(A: np.ndarray, dtype=None) -> list:
    """(4, n) -> list of contiguous SoA trains (4 real, or 8 re/im interleaved
    per element: a11r, a11i, a21r, a21i, a12r, a12i, a22r, a22i)."""
    if np.iscomplexobj(A):
        rdt = dtype or (np.float64 if A.dtype == np.complex128 else np.float32)
        out = []
        for e in range(4):
            out.append(np.ascontiguousarray(A[e].real, dtype=rdt))
            out.append(np.ascontiguousarray(A[e].imag, dtype=rdt))
        return out
    rdt = dtype or A.dtype
    return [np.ascontiguousarray(A[e], dtype=rdt) for e in range(4)]


# ---------------------------------------------------------------------------
# Kogbetliantz inputs
# ---------------------------------------------------------------------------

def _haar_like(rng, N: int, cplx: bool) -> np.ndarray:
    """Orthogonal (unitary) Q as the Householder product of a QR factorisation
    of a Gaussian matrix, with the sign (phase) of diag(R) moved into Q."""
    if cplx:
        G = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    else:
        G = rng.standard_normal((N, N))
    Q, R = np.linalg.qr(G)
    d = np.diag(R)
    ph = d / np.where(np.abs(d) == 0, 1, np.abs(d))
    return Q * ph[None, :]


def kog_matrix(order: int, seed: int, cond: float = 1e12, cplx: bool = False,
               return_sigma: bool = False):
    """A = Q1 diag(s) Q2^* in FP64, s_i = cond^(-i/(order-1)) geometric from 1
    to 1/cond, Q1, Q2 seeded random orthogonal (unitary).  Column-major
    (Fortran-ordered) array of shape (order, order)."""
    rng = np.random.default_rng(seed)
    Q1 = _haar_like(rng, order, cplx)
    Q2 = _haar_like(rng, order, cplx)
    i = np.arange(order, dtype=np.float64)
    s = cond ** (-i / max(order - 1, 1))
    A = (Q1 * s[None, :]) @ np.conj(Q2.T)
    A = np.asfortranarray(A)
    return (A, s) if return_sigma else A


def kog_problem_set(nprob: int, seed: int, omin: int = 32, omax: int = 2048):
    """Uneven batch: orders 2 round(2^U[log2(omin/2), log2(omax/2)]), condition
    numbers 10^U[2, 12]; the first half complex FP64, the second half real
    (to be rounded to FP32 by the caller).  Returns a list of dicts."""
    rng = np.random.default_rng(seed)
    lo, hi = np.log2(omin / 2), np.log2(omax / 2)
    probs = []
    for p in range(nprob):
        order = 2 * int(round(2 ** rng.uniform(lo, hi)))
        cond = 10 ** rng.uniform(2, 12)
        cplx = p < nprob // 2
        A, s = kog_matrix(order, int(rng.integers(0, 2**62)), cond=cond, cplx=cplx,
                          return_sigma=True)
        probs.append(dict(order=order, cond=cond, cplx=cplx, A=A, sigma=s))
    return probs


def round_robin_pairs(N: int) -> np.ndarray:
    """Round-robin (circle method) tournament of N = 2n players: N-1 rounds of
    n disjoint pairs (p < q) covering every pair exactly once.  Returns an
    int32 array of shape (N-1, n, 2).  This is scheduling, not arithmetic of
    the method; the paper leaves the pivot ordering open (section 1)."""
    assert N % 2 == 0 and N >= 2
    n = N // 2
    players = list(range(N))
    rounds = np.empty((N - 1, n, 2), dtype=np.int32)
    for t in range(N - 1):
        for k in range(n):
            a, b = players[k], players[N - 1 - k]
            rounds[t, k] = (min(a, b), max(a, b))
        # keep players[0] fixed, rotate the rest by one
        players = [players[0]] + [players[-1]] + players[1:-1]
    return rounds


def kog_problem_set_device(nprob: int, seed: int, omin: int = 32, omax: int = 2048,
                           device: str = "cuda"):
    """The uneven batch built on the GPU (for benchmarking): orders
    2 round(2^U[log2(omin/2), log2(omax/2)]), condition numbers 10^U[2, 12],
    sigma geometric from 1 to 1/cond, A = Q1 diag(sigma) Q2^* with Q1, Q2 the
    Q factors (phase-fixed) of seeded Gaussian matrices, formed in FP64 with
    torch on the device; the first half complex FP64, the second half real and
    rounded to FP32.  Gaussians come from numpy's seeded PCG64.  Matrices are
    column-major (stride(0) == 1).  Returns a list of dicts."""
    import torch
    rng = np.random.default_rng(seed)
    lo, hi = np.log2(omin / 2), np.log2(omax / 2)
    out = []
    for p in range(nprob):
        order = 2 * int(round(2 ** rng.uniform(lo, hi)))
        cond = 10 ** rng.uniform(2, 12)
        cplx = p < nprob // 2
        qs = []
        for _ in range(2):
            G = rng.standard_normal((order, order))
            if cplx:
                G = G + 1j * rng.standard_normal((order, order))
            Q, R = torch.linalg.qr(torch.from_numpy(G).to(device))
            d = torch.diagonal(R)
            ph = d / torch.where(d.abs() == 0, torch.ones_like(d.abs()), d.abs())
            qs.append(Q * ph[None, :])
        sig = cond ** (-np.arange(order, dtype=np.float64) / max(order - 1, 1))
        s_t = torch.from_numpy(sig).to(device)
        A = (qs[0] * s_t[None, :].to(qs[0].dtype)) @ qs[1].conj().T
        if not cplx:
            A = A.real.to(torch.float32)
        A = A.t().contiguous().t()  # column-major
        out.append(dict(order=order, cond=cond, cplx=cplx, A=A, sigma=sig))
    return out
