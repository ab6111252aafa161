"""GPU parity of the Kogbetliantz solver (fused persistent kernel, unfused
chain, hipGraph replay) against the CPU oracle.  The GPU uses the oracle's
pivot SVD (bitwise identical lanes) and the same rounding order in the block
update, so the iterates are compared bitwise."""
import numpy as np
import pytest

import oracle.oracle as O
from workloads import SEED_BASE, kog_matrix

pytestmark = pytest.mark.gpu

DT = {"d": np.float64, "z": np.complex128, "s": np.float32, "c": np.complex64}
EPS = {"d": 2.0 ** -52, "z": 2.0 ** -52, "s": 2.0 ** -23, "c": 2.0 ** -23}
MODES = {"fused": 0, "unfused": 1, "graph": 3}


def _make(N, kind, seed, cond=1e8):
    A = kog_matrix(N, seed, cond=cond, cplx=kind in "zc")
    return np.asfortranarray(A.astype(DT[kind]))


def _dev(A):
    import torch
    t = torch.from_numpy(A).cuda()
    assert t.stride(0) == 1
    return t


def _same(a, b):
    a = np.ascontiguousarray(a).view(np.uint8)
    b = np.ascontiguousarray(b).view(np.uint8)
    return np.array_equal(a, b)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available()
    from paper_2005_07403_amd import svd2 as S
    S.lib()
    yield


@pytest.mark.parametrize("kind", ["d", "z", "s", "c"])
@pytest.mark.parametrize("mode", ["fused", "unfused"])
@pytest.mark.parametrize("N", [2, 6, 64, 130, 1030])
def test_steps_bitwise(kind, mode, N):
    import torch
    from paper_2005_07403_amd import svd2 as S
    A = _make(N, kind, SEED_BASE + 300 + N)
    G = _dev(A)
    ws = S.kog_workspace(G)
    for t in range(min(N - 1, 4)):
        S.kog_step(G, t, ws=ws, flags=MODES[mode])
        O.kog_step(A, t)
        torch.cuda.synchronize()
        assert _same(G.cpu().numpy(), A), (kind, mode, N, t)


@pytest.mark.parametrize("kind", ["d", "z", "s"])
@pytest.mark.parametrize("mode", ["fused", "unfused", "graph"])
def test_solve_bitwise(kind, mode):
    """Full solve at N = 64: same sweep count, bitwise the same final matrix."""
    from paper_2005_07403_amd import svd2 as S
    N = 64
    tol = 1e-14 if kind in "dz" else 1e-6
    A = _make(N, kind, SEED_BASE + 310, cond=1e10 if kind in "dz" else 1e4)
    A0 = A.copy()
    G = _dev(A)
    r = S.kog_solve(G, tol=tol, flags=MODES[mode])
    ro = O.kog_solve(A, tol=tol)
    assert r["status"] == ro["status"] == 0
    assert r["sweeps"] == ro["sweeps"]
    assert _same(G.cpu().numpy(), A)
    sv = np.linalg.svd(A0.astype(np.complex128 if kind in "zc" else np.float64), compute_uv=False)
    sig = np.sort(np.abs(np.diag(G.cpu().numpy())).astype(np.float64))[::-1]
    assert np.max(np.abs(sig - sv)) <= 8 * N * EPS[kind] * sv[0]


def test_sweep_entry_point_and_norms():
    import torch
    from paper_2005_07403_amd import svd2 as S
    N = 130
    A = _make(N, "d", SEED_BASE + 320)
    G = _dev(A)
    S.kog_sweep(G)
    for t in range(N - 1):
        O.kog_step(A, t)
    torch.cuda.synchronize()
    assert _same(G.cpu().numpy(), A)
    off2, tot2 = S.kog_norms(G)
    o2, t2 = O.kog_norms(A)
    assert abs(off2 - o2) <= 1e-12 * t2 and abs(tot2 - t2) <= 1e-12 * t2


@pytest.mark.parametrize("mode", ["two_step", "unfused", "fused"])
def test_full_order_4096_first_steps(mode):
    """The one-problem workload (real FP64, N = 4096, sigma geometric from 1
    to 1e-12) in the tile shapes the benchmark times (the autotuner's table):
    steps 0-3 as two two-step passes, or as four unfused or fused steps, are
    bitwise the oracle's after steps 1 and 3."""
    import torch
    from paper_2005_07403_amd import svd2 as S
    S.apply_tuning()
    N = 4096
    A = kog_matrix(N, SEED_BASE + 3, cond=1e12)
    G = _dev(A)
    flags = {"two_step": S.SVD2_KOG_TWO_STEP, "unfused": S.SVD2_KOG_UNFUSED, "fused": 0}[mode]
    ws = S.kog_workspace(G, flags)
    for t0 in (0, 2):
        if mode == "two_step":
            S.kog_step(G, t0, ws=ws, flags=flags)
        else:
            for t in (t0, t0 + 1):
                S.kog_step(G, t, ws=ws, flags=flags)
        for t in (t0, t0 + 1):
            O.kog_step(A, t)
        torch.cuda.synchronize()
        assert _same(G.cpu().numpy(), A), (mode, t0)


@pytest.mark.slow
def test_full_order_4096_solve():
    """Full fused solve of the one-problem workload; sigma against the
    construction."""
    from paper_2005_07403_amd import svd2 as S
    N = 4096
    A, s = kog_matrix(N, SEED_BASE + 3, cond=1e12, return_sigma=True)
    G = _dev(A)
    r = S.kog_solve(G, tol=1e-14, max_sweeps=60)
    assert r["status"] == 0, r
    sig = np.sort(np.diag(G.cpu().numpy()))[::-1]
    assert np.all(sig >= 0)
    assert np.max(np.abs(sig - s)) <= 8 * N * EPS["d"] * s[0]
    print(f"N=4096 solve: {r['sweeps']} sweeps, off/||A|| = {r['off_rel']:.3e}")


@pytest.mark.parametrize("kind", ["d", "z", "s", "c"])
@pytest.mark.parametrize("N", [2, 4, 6, 8, 64, 130, 1030])
def test_two_step_sweep_bitwise(kind, N):
    """Two steps per pass (out of place, ping-pong with the workspace matrix):
    one sweep, then a second, each bitwise equal to N-1 oracle steps.  The
    sweep count of passes is odd or even depending on N, so both the result
    left in the workspace (copied back) and in A are covered."""
    import torch
    from paper_2005_07403_amd import svd2 as S
    A = _make(N, kind, SEED_BASE + 330 + N)
    G = _dev(A)
    ws = S.kog_workspace(G, S.SVD2_KOG_TWO_STEP)
    for _ in range(2):
        S.kog_sweep(G, ws=ws, flags=S.SVD2_KOG_TWO_STEP)
        for t in range(N - 1):
            O.kog_step(A, t)
        torch.cuda.synchronize()
        assert _same(G.cpu().numpy(), A), (kind, N)


@pytest.mark.parametrize("kind", ["d", "z", "s", "c"])
@pytest.mark.parametrize("N", [4, 6, 130])
def test_two_step_single_pass_bitwise(kind, N):
    """One two-step pass through the step entry point (steps t, t+1, copied
    back into A), at the first and the last pair of steps of a sweep,
    bitwise equal to two oracle steps each."""
    import torch
    from paper_2005_07403_amd import svd2 as S
    A = _make(N, kind, SEED_BASE + 360 + N)
    G = _dev(A)
    ws = S.kog_workspace(G, S.SVD2_KOG_TWO_STEP)
    for t in sorted({0, N - 3}):
        S.kog_step(G, t, ws=ws, flags=S.SVD2_KOG_TWO_STEP)
        O.kog_step(A, t)
        O.kog_step(A, t + 1)
        torch.cuda.synchronize()
        assert _same(G.cpu().numpy(), A), (kind, N, t)


@pytest.mark.parametrize("kind", ["d", "z", "s", "c"])
def test_two_step_padded_lda(kind):
    """A with lda > N (a view into a larger column-major buffer): the
    workspace matrix uses lda = N, the padding rows stay untouched."""
    import torch
    from paper_2005_07403_amd import svd2 as S
    N, pad = 66, 5
    A = _make(N, kind, SEED_BASE + 340)
    big = np.asfortranarray(np.full((N + pad, N), 7, dtype=DT[kind]))
    big[:N, :] = A
    Gbig = _dev(big)
    G = Gbig[:N, :]
    assert G.stride(1) == N + pad
    S.kog_sweep(G, flags=S.SVD2_KOG_TWO_STEP)
    for t in range(N - 1):
        O.kog_step(A, t)
    torch.cuda.synchronize()
    out = Gbig.cpu().numpy()
    assert _same(out[:N, :], A)
    assert np.all(out[N:, :] == 7)


@pytest.mark.parametrize("kind", ["d", "z", "s", "c"])
@pytest.mark.parametrize("N", [64, 130])
def test_two_step_solve_bitwise(kind, N):
    """Full solve in the two-step mode: same sweep count, status and final
    matrix as the oracle."""
    from paper_2005_07403_amd import svd2 as S
    tol = 1e-14 if kind in "dz" else 1e-6
    A = _make(N, kind, SEED_BASE + 350 + N, cond=1e10 if kind in "dz" else 1e4)
    G = _dev(A)
    r = S.kog_solve(G, tol=tol, flags=S.SVD2_KOG_TWO_STEP)
    ro = O.kog_solve(A, tol=tol)
    assert r["status"] == ro["status"] == 0
    assert r["sweeps"] == ro["sweeps"]
    assert abs(r["off_rel"] - ro["off_rel"]) <= 1e-12 + 1e-10 * ro["off_rel"]
    assert _same(G.cpu().numpy(), A)


def test_two_step_full_order_4096_sweep():
    """One two-step sweep of the one-problem workload (real FP64, N = 4096)
    against the single-step unfused sweep on the GPU (bitwise)."""
    import torch
    from paper_2005_07403_amd import svd2 as S
    N = 4096
    A = kog_matrix(N, SEED_BASE + 3, cond=1e12)
    G1, G2 = _dev(A), _dev(A)
    S.kog_sweep(G1, flags=S.SVD2_KOG_UNFUSED)
    S.kog_sweep(G2, flags=S.SVD2_KOG_TWO_STEP)
    torch.cuda.synchronize()
    assert torch.equal(G1.view(torch.int64), G2.view(torch.int64))


@pytest.mark.slow
def test_two_step_full_order_4096_solve_equals_unfused():
    """The one-problem workload solved to 1e-14 by the two-step driver ends
    bitwise equal to the unfused single-step solve (same sweep count), and its
    sigma matches the construction."""
    import torch
    from paper_2005_07403_amd import svd2 as S
    N = 4096
    A, s = kog_matrix(N, SEED_BASE + 3, cond=1e12, return_sigma=True)
    G1, G2 = _dev(A), _dev(A)
    r1 = S.kog_solve(G1, tol=1e-14, max_sweeps=60, flags=S.SVD2_KOG_UNFUSED)
    r2 = S.kog_solve(G2, tol=1e-14, max_sweeps=60, flags=S.SVD2_KOG_TWO_STEP)
    torch.cuda.synchronize()
    assert r1["status"] == r2["status"] == 0
    assert r1["sweeps"] == r2["sweeps"]
    assert torch.equal(G1.view(torch.int64), G2.view(torch.int64))
    sig = np.sort(np.diag(G2.cpu().numpy()))[::-1]
    assert np.max(np.abs(sig - s)) <= 8 * N * EPS["d"] * s[0]


@pytest.mark.parametrize("kind", ["d", "z", "s", "c"])
def test_sigma_extraction(kind):
    """kog_sigma after a solve: the diagonal magnitudes in descending order,
    bitwise (the converged diagonal is real and non-negative), equal to the
    oracle's sorted diagonal; also for an order that is not a power of two."""
    from paper_2005_07403_amd import svd2 as S
    N = 130
    tol = 1e-14 if kind in "dz" else 1e-6
    A = _make(N, kind, SEED_BASE + 360, cond=1e8 if kind in "dz" else 1e3)
    G = _dev(A)
    S.kog_solve(G, tol=tol)
    O.kog_solve(A, tol=tol)
    sig = S.kog_sigma(G).cpu().numpy()
    d = np.diag(A)
    assert np.all(np.imag(d) == 0) and np.all(np.real(d) >= 0)
    want = np.sort(np.real(d))[::-1].astype(sig.dtype)
    assert _same(sig, want)


def test_sigma_extraction_general_input():
    """On an arbitrary real matrix (signed diagonal, order 1..300) the
    result is |diag| sorted descending, bitwise."""
    import torch
    from paper_2005_07403_amd import svd2 as S
    rng = np.random.default_rng(SEED_BASE + 370)
    for N in (1, 2, 3, 7, 64, 255, 256, 257, 300):
        A = np.asfortranarray(rng.standard_normal((N, N)))
        sig = S.kog_sigma(_dev(A)).cpu().numpy()
        assert _same(sig, np.sort(np.abs(np.diag(A)))[::-1]), N


def _scaled(A, k):
    """A * 2^k, one component at a time, rounded to the nearest in A's type."""
    if np.iscomplexobj(A):
        return np.asfortranarray(_scaled(A.real, k) + 1j * _scaled(A.imag, k)).astype(A.dtype)
    return np.asfortranarray(A * A.dtype.type(2.0 ** k))


SCALES = [("d", 600), ("d", -600), ("d", -1000), ("z", 700), ("z", -700), ("s", 100), ("s", -60),
          ("c", 100), ("c", -60)]


@pytest.mark.parametrize("kind,k", SCALES)
@pytest.mark.parametrize("mode", ["fused", "unfused", "graph", "two"])
def test_solve_tiny_and_huge_matrices(kind, k, mode):
    """A matrix scaled by 2^k far from 1 takes the sweeps of the unscaled one
    and ends bitwise equal to the oracle's solve of it (both scale the matrix
    exactly by a power of two around the iteration)."""
    from paper_2005_07403_amd import svd2 as S
    N = 64
    tol = 1e-14 if kind in "dz" else 1e-6
    A1 = _make(N, kind, SEED_BASE + 360, cond=1e6 if kind in "dz" else 1e3)
    A = _scaled(A1, k)
    assert _same(_scaled(A, -k), A1)
    flags = S.SVD2_KOG_TWO_STEP if mode == "two" else MODES[mode]
    G = _dev(A)
    r = S.kog_solve(G, tol=tol, flags=flags)
    ro = O.kog_solve(A, tol=tol)
    r1 = O.kog_solve(A1, tol=tol)
    assert r["status"] == ro["status"] == r1["status"] == 0
    assert r["sweeps"] == ro["sweeps"] == r1["sweeps"] > 0
    assert _same(G.cpu().numpy(), A)


@pytest.mark.parametrize("kind", ["d", "c"])
def test_caller_workspace_in_bytes(kind):
    """The binding passes a caller's workspace at its size in bytes whatever
    its dtype: 8 bytes short of kog_workspace_bytes is refused before any
    launch (the matrix untouched), and the exact size gives the solve of a
    workspace the binding allocates, bit for bit."""
    import torch
    from paper_2005_07403_amd import svd2 as S
    N, flags = 64, S.SVD2_KOG_TWO_STEP
    A = _make(N, kind, SEED_BASE + 360)
    need = S.kog_workspace_bytes(N, kind, flags)
    assert need % 8 == 0
    G = _dev(A)
    with pytest.raises(S.Svd2Error) as err:
        S.kog_solve(G, ws=torch.empty(need // 8 - 1, dtype=torch.float64, device="cuda"), flags=flags)
    assert err.value.status == 6
    assert _same(G.cpu().numpy(), A)
    r1 = S.kog_solve(G, flags=flags)
    G2 = _dev(A)
    r2 = S.kog_solve(G2, ws=torch.empty(need // 8, dtype=torch.float64, device="cuda"), flags=flags)
    torch.cuda.synchronize()
    assert r1["sweeps"] == r2["sweeps"] and _same(G.cpu().numpy(), G2.cpu().numpy())


def test_barrier_probe_epochs():
    """The fused kernel's grid barrier, checked by its epoch counters in the
    barrier probe: after each of 200 barriers every workgroup sees every
    other's epoch at the barrier's (no workgroup released early, no wait
    aborted), for 1, 2 and 4 workgroups per CU; a barrier-free launch and a
    grid larger than the barrier's slots are handled."""
    import torch
    from paper_2005_07403_amd import svd2 as S
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    ws = torch.empty(256 + 4096 * 64, dtype=torch.uint8, device="cuda")
    viol = torch.zeros(1, dtype=torch.int32, device="cuda")
    for blocks in (cus, 2 * cus, 4 * cus):
        viol.zero_()
        S.kog_barrier_probe(200, blocks, ws, violations=viol)
        torch.cuda.synchronize()
        assert int(viol.item()) == 0, blocks
    S.kog_barrier_probe(0, cus, ws, violations=viol)
    torch.cuda.synchronize()
    assert int(viol.item()) == 0
    with pytest.raises(S.Svd2Error):
        S.kog_barrier_probe(1, 4096 + 1, ws)
