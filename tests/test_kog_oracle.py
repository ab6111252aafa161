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


# ---------------------------------------------------------------------------
# SVD with accumulated transformations: A_0 = U diag(sigma) V^*
# ---------------------------------------------------------------------------
DT = {"d": np.float64, "z": np.complex128, "s": np.float32, "c": np.complex64}
EPSK = {"d": 2.0 ** -52, "z": 2.0 ** -52, "s": 2.0 ** -23, "c": 2.0 ** -23}


@pytest.mark.parametrize("kind", ["d", "z", "s", "c"])
@pytest.mark.parametrize("N", [2, 32, 66])
def test_svd_reconstructs_and_is_unitary(kind, N):
    """Against LAPACK and the definition of the SVD: every rotation is applied
    with O(eps) relative error, each column of U and V receives S (N - 1) of
    them in S sweeps, so ||A_0 - U S V^*||_F / ||A_0||_F and ||U^*U - I||_F
    stay below a small multiple of S N^1.5 eps; sigma is descending and
    matches LAPACK's within 8 N eps sigma_max."""
    A0 = np.asfortranarray(kog_matrix(N, 91 + N, cond=1e4, cplx=kind in "zc").astype(DT[kind]))
    A = A0.copy(order="F")
    r = O.kog_svd(A, tol=1e-14 if kind in "dz" else 1e-6)
    assert r["status"] == 0 and r["sweeps"] >= 1
    S, eps = r["sweeps"], EPSK[kind]
    U, V = r["U"].astype(np.complex128), r["V"].astype(np.complex128)
    s = r["sigma"].astype(np.float64)
    Ac = A0.astype(np.complex128)
    bound = 4 * S * N ** 1.5 * eps
    assert np.linalg.norm(Ac - (U * s) @ V.conj().T) <= bound * np.linalg.norm(Ac)
    assert np.linalg.norm(U.conj().T @ U - np.eye(N)) <= bound
    assert np.linalg.norm(V.conj().T @ V - np.eye(N)) <= bound
    assert np.all(np.diff(s) <= 0)
    sv = np.linalg.svd(Ac, compute_uv=False)
    assert np.max(np.abs(s - sv)) <= 8 * N * eps * sv[0]
    # the final iterate's diagonal holds the same values
    assert np.array_equal(np.sort(np.abs(np.diag(A)).astype(np.float64))[::-1], s)


@pytest.mark.parametrize("kind", ["d", "z"])
def test_svd_singular_vectors_match_lapack(kind):
    """With well separated singular values (geometric, ratio 1.2) each
    singular pair is unique up to a phase: |<u_i, u_i'>| and |<v_i, v_i'>|
    against LAPACK's vectors are 1 within 1e-11."""
    N = 40
    rng = np.random.default_rng(5)
    sig = 1.2 ** -np.arange(N)
    Q1 = np.linalg.qr(rng.standard_normal((N, N)) + (1j * rng.standard_normal((N, N)) if kind == "z" else 0))[0]
    Q2 = np.linalg.qr(rng.standard_normal((N, N)) + (1j * rng.standard_normal((N, N)) if kind == "z" else 0))[0]
    A0 = np.asfortranarray(((Q1 * sig) @ Q2.conj().T).astype(DT[kind]))
    r = O.kog_svd(A0.copy(order="F"))
    Ul, sl, Vlh = np.linalg.svd(A0.astype(np.complex128))
    cu = np.abs(np.sum(np.conj(Ul) * r["U"], axis=0))
    cv = np.abs(np.sum(np.conj(Vlh.conj().T) * r["V"], axis=0))
    assert np.max(np.abs(cu - 1)) <= 1e-11 and np.max(np.abs(cv - 1)) <= 1e-11


@pytest.mark.parametrize("kind", ["d", "s"])
def test_svd_of_real_diagonal_is_exact(kind):
    """A real diagonal matrix takes one sweep (the minimum), U and V come out
    as signed permutation matrices and U diag(sigma) V^T reproduces A exactly;
    sigma is |d| in descending order."""
    d = np.array([3.0, -5.0, 0.5, -0.25, 7.0, 2.0, -1.0, 4.0])
    A0 = np.asfortranarray(np.diag(d).astype(DT[kind]))
    r = O.kog_svd(A0.copy(order="F"))
    assert r["status"] == 0 and r["sweeps"] == 1
    assert set(np.unique(np.abs(r["U"]))) == {0.0, 1.0} and set(np.unique(np.abs(r["V"]))) == {0.0, 1.0}
    assert np.array_equal(r["sigma"], np.sort(np.abs(d))[::-1].astype(DT[kind]))
    assert np.array_equal((r["U"] * r["sigma"]) @ r["V"].T, A0)


@pytest.mark.parametrize("kind", ["d", "z", "s", "c"])
def test_svd_zero_matrix_and_bad_sweep_limit(kind):
    Z = np.zeros((6, 6), dtype=DT[kind], order="F")
    r = O.kog_svd(Z)
    assert r["status"] == 0 and r["sweeps"] == 1
    assert np.array_equal(r["U"], np.eye(6)) and np.array_equal(r["V"], np.eye(6))
    assert np.array_equal(r["sigma"], np.zeros(6))
    assert O.kog_svd(Z, max_sweeps=0)["status"] == 6


def test_svd_iterate_equals_solve():
    """Accumulating the transformations does not change the iterate: after
    the same sweeps, kog_svd's A equals kog_solve's bit for bit."""
    A = np.asfortranarray(kog_matrix(34, 17, cond=1e8, cplx=True))
    B = A.copy(order="F")
    r1 = O.kog_svd(A)
    r2 = O.kog_solve(B)
    assert r1["sweeps"] == r2["sweeps"]
    assert np.array_equal(A, B)
