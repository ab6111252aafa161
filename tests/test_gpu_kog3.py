"""GPU parity of the three-step Kogbetliantz passes (SVD2_KOG_THREE_STEP):
steps t, t+1, t+2 in one pass over the matrix, bitwise equal to three of the
oracle's single steps (section 1's step, under the circle ordering), for
every element type, at small, ragged and full orders, through the step,
sweep and solve entry points and over the workgroup shapes."""
import numpy as np
import pytest

import oracle.oracle as O
from workloads import SEED_BASE, kog_matrix

pytestmark = pytest.mark.gpu

DT = {"d": np.float64, "z": np.complex128, "s": np.float32, "c": np.complex64}


def _make(N, kind, seed, cond=1e8):
    A = kog_matrix(N, seed, cond=cond, cplx=kind in "zc")
    return np.asfortranarray(A.astype(DT[kind]))


def _dev(A):
    import torch
    t = torch.from_numpy(A).cuda()
    assert t.stride(0) == 1
    return t


def _same(a, b):
    return np.array_equal(np.ascontiguousarray(a).view(np.uint8), np.ascontiguousarray(b).view(np.uint8))


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available()
    from paper_2005_07403_amd import svd2 as S
    S.lib()
    yield
    S.kog_set_three_step_tiles([])


@pytest.mark.parametrize("kind", ["d", "z", "s", "c"])
@pytest.mark.parametrize("N", [4, 6, 8, 66, 130, 1030])
def test_three_step_single_pass_bitwise(kind, N):
    """One three-step pass through the step entry point, at the first and the
    last three steps of a sweep, bitwise equal to three oracle steps."""
    import torch
    from paper_2005_07403_amd import svd2 as S
    A = _make(N, kind, SEED_BASE + 1360 + N)
    G = _dev(A)
    f = S.SVD2_KOG_THREE_STEP
    ws = S.kog_workspace(G, f)
    for t in sorted({0, N - 4}):
        S.kog_step(G, t, ws=ws, flags=f)
        for u in range(t, t + 3):
            O.kog_step(A, u)
        torch.cuda.synchronize()
        assert _same(G.cpu().numpy(), A), (kind, N, t)


@pytest.mark.parametrize("kind", ["d", "z", "s", "c"])
@pytest.mark.parametrize("N", [2, 4, 6, 8, 10, 64, 130, 1030])
def test_three_step_sweep_bitwise(kind, N):
    """Two sweeps (N-1 steps each: three-step passes, then a two-step pass or
    a single step where 3 does not divide N-1), each bitwise equal to N-1
    oracle steps."""
    import torch
    from paper_2005_07403_amd import svd2 as S
    A = _make(N, kind, SEED_BASE + 1330 + N)
    G = _dev(A)
    f = S.SVD2_KOG_THREE_STEP
    ws = S.kog_workspace(G, f)
    for _ in range(2):
        S.kog_sweep(G, ws=ws, flags=f)
        for t in range(N - 1):
            O.kog_step(A, t)
        torch.cuda.synchronize()
        assert _same(G.cpu().numpy(), A), (kind, N)


@pytest.mark.parametrize("wpg,lc", [(1, 2), (1, 3), (2, 5), (4, 7), (4, 16), (2, 64), (1, 128)])
@pytest.mark.parametrize("kind", ["d", "c"])
def test_three_step_tile_shapes(kind, wpg, lc):
    """Workgroup shapes: wavefronts per workgroup and column pairs per tile,
    down to tiles narrower than the two-pair halo on either side."""
    import torch
    from paper_2005_07403_amd import svd2 as S
    N = 254
    S.kog_set_three_step_tiles([(1 << 20, wpg, lc)])
    try:
        A = _make(N, kind, SEED_BASE + 1390 + lc)
        G = _dev(A)
        S.kog_sweep(G, flags=S.SVD2_KOG_THREE_STEP)
        for t in range(N - 1):
            O.kog_step(A, t)
        torch.cuda.synchronize()
        assert _same(G.cpu().numpy(), A), (kind, wpg, lc)
    finally:
        S.kog_set_three_step_tiles([])


@pytest.mark.parametrize("kind", ["d", "z", "s", "c"])
def test_three_step_padded_lda(kind):
    """A with lda > N: the padding rows stay untouched."""
    import torch
    from paper_2005_07403_amd import svd2 as S
    N, pad = 66, 5
    A = _make(N, kind, SEED_BASE + 1340)
    big = np.asfortranarray(np.full((N + pad, N), 7, dtype=DT[kind]))
    big[:N, :] = A
    Gbig = _dev(big)
    G = Gbig[:N, :]
    assert G.stride(1) == N + pad
    S.kog_sweep(G, flags=S.SVD2_KOG_THREE_STEP)
    for t in range(N - 1):
        O.kog_step(A, t)
    torch.cuda.synchronize()
    out = Gbig.cpu().numpy()
    assert _same(out[:N, :], A)
    assert np.all(out[N:, :] == 7)


@pytest.mark.parametrize("kind", ["d", "z", "s", "c"])
@pytest.mark.parametrize("N", [64, 130])
def test_three_step_solve_bitwise(kind, N):
    """Full solve: same status, sweep count and final matrix as the oracle."""
    from paper_2005_07403_amd import svd2 as S
    tol = 1e-14 if kind in "dz" else 1e-6
    A = _make(N, kind, SEED_BASE + 1350 + N, cond=1e10 if kind in "dz" else 1e4)
    G = _dev(A)
    r = S.kog_solve(G, tol=tol, flags=S.SVD2_KOG_THREE_STEP)
    ro = O.kog_solve(A, tol=tol)
    assert r["status"] == ro["status"] == 0
    assert r["sweeps"] == ro["sweeps"]
    assert _same(G.cpu().numpy(), A)


def test_three_step_full_order_4096_first_pass():
    """The one-problem workload (real FP64, N = 4096): the first three-step
    pass in the launch configuration the benchmark uses, bitwise equal to
    three oracle steps, and a whole sweep bitwise equal to the unfused
    single-step sweep on the GPU."""
    import torch
    from paper_2005_07403_amd import svd2 as S
    S.apply_tuning()
    N = 4096
    A = kog_matrix(N, SEED_BASE + 3, cond=1e12)
    A = np.asfortranarray(A)
    G = _dev(A)
    f = S.SVD2_KOG_THREE_STEP
    S.kog_step(G, 0, flags=f)
    B = A.copy(order="F")
    for t in range(3):
        O.kog_step(B, t)
    torch.cuda.synchronize()
    assert _same(G.cpu().numpy(), B)
    G1, G2 = _dev(A), _dev(A)
    S.kog_sweep(G1, flags=S.SVD2_KOG_UNFUSED)
    S.kog_sweep(G2, flags=f)
    torch.cuda.synchronize()
    assert torch.equal(G1.view(torch.int64), G2.view(torch.int64))
