"""GPU parity of the Kogbetliantz SVD with accumulated transformations
(A_0 = U diag(sigma) V^*) against the oracle's: U, V, sigma and the final
iterate bitwise, the same status and sweep count, for one step per pass (in
place), the hipGraph replay and two or three steps per pass (U and V
alternating with workspace copies)."""
import numpy as np
import pytest

import oracle.oracle as O
from workloads import SEED_BASE, kog_matrix

pytestmark = pytest.mark.gpu

DT = {"d": np.float64, "z": np.complex128, "s": np.float32, "c": np.complex64}
TOL = {"d": 1e-14, "z": 1e-14, "s": 1e-6, "c": 1e-6}
EPS = {"d": 2.0 ** -52, "z": 2.0 ** -52, "s": 2.0 ** -23, "c": 2.0 ** -23}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available()
    from paper_2005_07403_amd import svd2 as S
    S.lib()
    yield


def _bits(a):
    return np.ascontiguousarray(a).view(np.uint8)


def _flags(mode):
    from paper_2005_07403_amd import svd2 as S
    return {"two": S.SVD2_KOG_TWO_STEP, "three": S.SVD2_KOG_THREE_STEP, "default": 0,
            "unfused": S.SVD2_KOG_UNFUSED, "graph": S.SVD2_KOG_UNFUSED | S.SVD2_KOG_GRAPH}[mode]


def _dev(A):
    import torch
    t = torch.from_numpy(np.asfortranarray(A)).cuda()
    assert t.stride(0) == 1
    return t


def _run(A, kind, mode, max_sweeps=40, pad=0):
    """GPU SVD of A (optionally with leading dimensions N + pad); returns
    (result dict, final iterate, U, V, sigma) as host arrays."""
    import torch
    from paper_2005_07403_amd import svd2 as S
    N = A.shape[0]
    if pad:
        big = np.zeros((N + pad, N), dtype=A.dtype, order="F")
        big[:N] = A
        G = torch.from_numpy(big).cuda()[:N]
        U = torch.full((N, N + pad), np.nan, dtype=G.dtype, device="cuda").t()[:N]
        V = torch.full((N, N + pad), np.nan, dtype=G.dtype, device="cuda").t()[:N]
    else:
        G, U, V = _dev(A), None, None
    r = S.kog_svd(G, tol=TOL[kind], max_sweeps=max_sweeps, U=U, V=V, flags=_flags(mode))
    torch.cuda.synchronize()
    return r, G.cpu().numpy(), r["U"].cpu().numpy(), r["V"].cpu().numpy(), r["sigma"].cpu().numpy()


@pytest.mark.parametrize("kind", ["d", "z", "s", "c"])
@pytest.mark.parametrize("mode", ["two", "three", "unfused", "graph"])
@pytest.mark.parametrize("N", [2, 4, 6, 8, 10, 14, 64, 130])
def test_svd_bitwise(kind, mode, N):
    A = np.asfortranarray(kog_matrix(N, SEED_BASE + 500 + N, cond=1e6 if kind in "dz" else 1e3,
                                     cplx=kind in "zc").astype(DT[kind]))
    r, Ag, U, V, s = _run(A.copy(order="F"), kind, mode)
    ro = O.kog_svd(A, tol=TOL[kind])
    assert r["status"] == ro["status"] == 0
    assert r["sweeps"] == ro["sweeps"]
    assert np.array_equal(_bits(Ag), _bits(A)), "iterate"
    assert np.array_equal(_bits(s), _bits(ro["sigma"])), "sigma"
    assert np.array_equal(_bits(U), _bits(ro["U"])), "U"
    assert np.array_equal(_bits(V), _bits(ro["V"])), "V"


@pytest.mark.parametrize("kind", ["d", "z", "s", "c"])
@pytest.mark.parametrize("mode", ["two", "three"])
def test_svd_padded_leading_dimensions(kind, mode):
    N = 66
    A = np.asfortranarray(kog_matrix(N, SEED_BASE + 510, cond=1e4, cplx=kind in "zc").astype(DT[kind]))
    r, Ag, U, V, s = _run(A.copy(order="F"), kind, mode, pad=6)
    ro = O.kog_svd(A, tol=TOL[kind])
    assert r["sweeps"] == ro["sweeps"]
    assert np.array_equal(_bits(U), _bits(ro["U"])) and np.array_equal(_bits(V), _bits(ro["V"]))
    assert np.array_equal(_bits(s), _bits(ro["sigma"])) and np.array_equal(_bits(Ag), _bits(A))


@pytest.mark.parametrize("mode", ["two", "three", "unfused"])
def test_svd_not_converged_tiny_and_diagonal(mode):
    """max_sweeps = 1 stops with status 7 and the oracle's outputs after one
    sweep; a matrix scaled by 2^-600 gives the oracle's result; a real
    diagonal matrix gives signed permutations, reproducing A exactly."""
    A = np.asfortranarray(kog_matrix(64, SEED_BASE + 520, cond=1e10))
    r, Ag, U, V, s = _run(A.copy(order="F"), "d", mode, max_sweeps=1)
    ro = O.kog_svd(A, tol=1e-14, max_sweeps=1)
    assert r["status"] == ro["status"] == 7 and r["sweeps"] == 1
    assert np.array_equal(_bits(U), _bits(ro["U"])) and np.array_equal(_bits(s), _bits(ro["sigma"]))
    T = np.asfortranarray(kog_matrix(34, SEED_BASE + 521, cond=1e3, cplx=True) * 2.0 ** -600)
    r, Ag, U, V, s = _run(T.copy(order="F"), "z", mode)
    ro = O.kog_svd(T)
    assert r["sweeps"] == ro["sweeps"] > 1
    assert np.array_equal(_bits(U), _bits(ro["U"])) and np.array_equal(_bits(s), _bits(ro["sigma"]))
    d = np.array([3.0, -5.0, 0.5, -0.25, 7.0, 2.0, -1.0, 4.0])
    D = np.asfortranarray(np.diag(d))
    r, Ag, U, V, s = _run(D.copy(order="F"), "d", mode)
    assert r["sweeps"] == 1 and np.array_equal(s, np.sort(np.abs(d))[::-1])
    assert np.array_equal((U * s) @ V.T, D)


@pytest.mark.parametrize("kind", ["d", "c"])
@pytest.mark.parametrize("mode", ["two", "three"])
def test_svd_order_1030_multi_step_equals_one_step(kind, mode):
    """At an order with many segments and row blocks, two or three steps per
    pass give bitwise the one-step-per-pass result (the accumulation walks of
    2, 3, 4 or 6 steps are single steps), and U diag(sigma) V^* reproduces
    A_0."""
    import torch
    N = 1030
    A = np.asfortranarray(kog_matrix(N, SEED_BASE + 530, cond=1e6 if kind == "d" else 1e3,
                                     cplx=kind in "zc").astype(DT[kind]))
    r1, A1, U1, V1, s1 = _run(A.copy(order="F"), kind, mode)
    r2, A2, U2, V2, s2 = _run(A.copy(order="F"), kind, "unfused")
    assert r1["status"] == r2["status"] == 0 and r1["sweeps"] == r2["sweeps"]
    for x, y in ((A1, A2), (U1, U2), (V1, V2), (s1, s2)):
        assert np.array_equal(_bits(x), _bits(y))
    cd = torch.complex128
    Ug, Vg, sg = (torch.from_numpy(np.ascontiguousarray(x)).cuda().to(cd) for x in (U1, V1, s1))
    A0 = torch.from_numpy(np.ascontiguousarray(A)).cuda().to(cd)
    rec = torch.linalg.norm(A0 - (Ug * sg) @ Vg.conj().t().contiguous()) / torch.linalg.norm(A0)
    orth = torch.linalg.norm(Ug.conj().t().contiguous() @ Ug - torch.eye(N, dtype=cd, device="cuda"))
    bound = 4 * r1["sweeps"] * N ** 1.5 * EPS[kind]
    assert float(rec) <= bound and float(orth) <= bound
    assert np.all(np.diff(s1) <= 0)


def test_svd_caller_outputs_checked():
    """U, V and sigma supplied by the caller must have A's order, element type
    and device, since the library writes N x N and N elements of that type;
    a mismatch raises before anything is launched and leaves A as it was.
    The same holds for kog_sigma's and svd2's output tensors."""
    import torch
    from paper_2005_07403_amd import svd2 as S
    N = 16
    A = np.asfortranarray(kog_matrix(N, SEED_BASE + 370, cond=1e4))
    G = _dev(A)
    bad = [dict(U=torch.empty((N, N), dtype=torch.float32, device="cuda").t()),
           dict(V=torch.empty((N - 2, N - 2), dtype=torch.float64, device="cuda").t()),
           dict(sigma=torch.empty(N - 1, dtype=torch.float64, device="cuda")),
           dict(sigma=torch.empty(N, dtype=torch.float32, device="cuda"))]
    for kw in bad:
        with pytest.raises(ValueError):
            S.kog_svd(G, **kw)
    torch.cuda.synchronize()
    assert np.array_equal(G.cpu().numpy(), A)
    with pytest.raises(ValueError):
        S.kog_sigma(G, out=torch.empty(N - 1, dtype=torch.float64, device="cuda"))
    trains = [torch.zeros(64, dtype=torch.float64, device="cuda") for _ in range(4)]
    outs = [torch.empty(64, dtype=torch.float64, device="cuda") for _ in range(10)]
    with pytest.raises(ValueError):
        S.svd2(trains, out=outs + [torch.empty(32, dtype=torch.float64, device="cuda")])
    with pytest.raises(ValueError):
        S.svd2(trains, out=outs + [torch.empty(64, dtype=torch.float32, device="cuda")])


@pytest.mark.slow
def test_svd_full_order_4096():
    """The benchmark's SVD (order 4096, real FP64, sigma from 1 to 1e-12, tuned
    launch shapes): two steps per pass (U and V four steps per pass) and three
    (U and V six steps per pass) bitwise equal to one step per pass, which
    matches the oracle bitwise at the orders
    the oracle can run; U diag(sigma) V^T reproduces A_0 and U, V are
    orthogonal within 4 S N^1.5 eps; sigma matches the construction within
    8 N eps."""
    import torch
    from paper_2005_07403_amd import svd2 as S
    S.apply_tuning()
    N = 4096
    A, sig0 = kog_matrix(N, SEED_BASE + 3, cond=1e12, return_sigma=True)
    A = np.asfortranarray(A)
    r1, A1, U1, V1, s1 = _run(A.copy(order="F"), "d", "two", max_sweeps=60)
    r2, A2, U2, V2, s2 = _run(A.copy(order="F"), "d", "unfused", max_sweeps=60)
    assert r1["status"] == r2["status"] == 0 and r1["sweeps"] == r2["sweeps"]
    for x, y in ((A1, A2), (U1, U2), (V1, V2), (s1, s2)):
        assert np.array_equal(_bits(x), _bits(y))
    del A2, U2, V2, s2
    r3, A3, U3, V3, s3 = _run(A.copy(order="F"), "d", "three", max_sweeps=60)
    assert r3["status"] == 0 and r3["sweeps"] == r1["sweeps"]
    for x, y in ((A1, A3), (U1, U3), (V1, V3), (s1, s3)):
        assert np.array_equal(_bits(x), _bits(y))
    del A3, U3, V3, s3
    eps, S_ = 2.0 ** -52, r1["sweeps"]
    Ug, Vg, sg = (torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in (U1, V1, s1))
    A0 = torch.from_numpy(np.ascontiguousarray(A)).cuda()
    rec = float(torch.linalg.norm(A0 - (Ug * sg) @ Vg.t().contiguous()) / torch.linalg.norm(A0))
    I = torch.eye(N, dtype=torch.float64, device="cuda")
    bound = 4 * S_ * N ** 1.5 * eps
    assert rec <= bound
    assert float(torch.linalg.norm(Ug.t().contiguous() @ Ug - I)) <= bound
    assert float(torch.linalg.norm(Vg.t().contiguous() @ Vg - I)) <= bound
    assert np.max(np.abs(s1 - sig0)) <= 8 * N * eps * sig0[0]
