"""Pins of the Kogbetliantz oracle (no GPU): the pair schedule, the per-step
identities of a unitary two-sided rotation, and the converged singular values
against numpy.linalg.svd (a library routine) and against the construction."""
import numpy as np
import pytest

import oracle.oracle as O
from workloads import kog_matrix

EPS = 2.0 ** -52


@pytest.mark.parametrize("N", [2, 4, 6, 8, 34, 64, 130])
def test_schedule_is_a_round_robin(N):
    seen = set()
    for t in range(N - 1):
        pr = O.kog_pairs(N, t)
        assert pr.shape == (N // 2, 2)
        assert np.all(pr[:, 0] < pr[:, 1])
        assert sorted(pr.ravel().tolist()) == list(range(N))  # perfect matching
        for p, q in pr.tolist():
            assert (p, q) not in seen
            seen.add((p, q))
    assert len(seen) == N * (N - 1) // 2  # every pair once per sweep


@pytest.mark.parametrize("cplx", [False, True])
def test_step_identities(cplx):
    """A step is A <- U^* A V with unitary U, V and diagonalised pivot blocks:
    ||A||_F is kept and off(A)^2 drops by exactly the pivots' off-diagonal mass
    (up to rounding)."""
    N = 64
    A = kog_matrix(N, 3, cond=1e6, cplx=cplx)
    for t in range(5):
        off0, tot0 = O.kog_norms(A)
        pr = O.kog_pairs(N, t)
        piv = sum(abs(A[p, q]) ** 2 + abs(A[q, p]) ** 2 for p, q in pr.tolist())
        O.kog_step(A, t)
        off1, tot1 = O.kog_norms(A)
        assert abs(tot1 - tot0) <= 64 * N * EPS * tot0
        assert abs(off1 - (off0 - piv)) <= 64 * N * EPS * tot0


def test_order_two_is_one_svd():
    """N = 2: one step is the 2x2 SVD itself."""
    rng = np.random.default_rng(4)
    for _ in range(50):
        A = np.asfortranarray(rng.standard_normal((2, 2)))
        sv = np.linalg.svd(A, compute_uv=False)
        r = O.kog_solve(A)
        assert r["status"] == 0 and r["sweeps"] <= 1
        assert np.allclose(r["sigma"], sv, rtol=4 * EPS, atol=4 * EPS * sv[0])
        assert A[0, 1] == 0 and A[1, 0] == 0


@pytest.mark.parametrize("N,cplx,cond", [(64, False, 1e12), (96, True, 1e12), (128, False, 1e3)])
def test_solve_matches_library_svd(N, cplx, cond):
    A, s = kog_matrix(N, 7, cond=cond, cplx=cplx, return_sigma=True)
    A0 = A.copy()
    r = O.kog_solve(A, tol=1e-14)
    assert r["status"] == 0, r
    sv = np.linalg.svd(A0, compute_uv=False)
    bound = 8 * N * EPS * sv[0]
    assert np.max(np.abs(r["sigma"] - sv)) <= bound
    assert np.max(np.abs(r["sigma"] - s)) <= bound
    # Frobenius invariance: sum of sigma^2 = ||A_0||_F^2
    assert abs(np.sum(r["sigma"] ** 2) - np.sum(np.abs(A0) ** 2)) <= 8 * N * EPS * np.sum(np.abs(A0) ** 2)
    # the off-norm history decreases and ends below the tolerance
    h = r["history"]
    assert h[-1] < 1e-14 and np.all(np.diff(h) < 0)


def test_fp32_solve():
    N = 64
    A, s = kog_matrix(N, 8, cond=1e4, return_sigma=True)
    A32 = np.asfortranarray(A.astype(np.float32))
    sv = np.linalg.svd(A32.astype(np.float64), compute_uv=False)
    r = O.kog_solve(A32, tol=1e-6)
    assert r["status"] == 0
    assert np.max(np.abs(r["sigma"] - sv)) <= 8 * N * 2.0 ** -23 * sv[0]



def _scaled(A, k):
    """A * 2^k, one component at a time, rounded to the nearest in A's type."""
    if np.iscomplexobj(A):
        return np.asfortranarray(_scaled(A.real, k) + 1j * _scaled(A.imag, k)).astype(A.dtype)
    return np.asfortranarray(A * A.dtype.type(2.0 ** k))


@pytest.mark.parametrize("kind,k", [("d", 600), ("d", -600), ("d", 1000), ("d", -1000), ("z", 700),
                                    ("z", -700), ("s", 100), ("s", -60), ("c", 100), ("c", -60)])
def test_solve_is_scale_equivariant(kind, k):
    """Scaling A by 2^k scales the solve's result by 2^k, rounded once, and
    leaves the sweep count unchanged: the iteration works on an exactly
    rescaled copy, so tiny or huge matrices are neither taken for zero nor
    overflow the stopping test's sums of squares."""
    dt = {"d": np.float64, "z": np.complex128, "s": np.float32, "c": np.complex64}[kind]
    A = np.asfortranarray(kog_matrix(24, 77, cond=1e3, cplx=kind in "zc").astype(dt))
    B = _scaled(A, k)
    assert np.array_equal(_scaled(B, -k), A)  # the scaled input is exact
    tol = 1e-5 if kind in "sc" else 1e-14
    ra = O.kog_solve(A, tol=tol)
    rb = O.kog_solve(B, tol=tol)
    assert ra["status"] == rb["status"] == 0
    assert ra["sweeps"] == rb["sweeps"] > 0
    assert np.array_equal(B, _scaled(A, k))
