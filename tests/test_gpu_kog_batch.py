"""GPU parity of the uneven multi-problem Kogbetliantz solve: every problem of
a mixed batch (orders 2..130, real/complex FP64 and FP32) must end bitwise
equal to the oracle's single-problem solve, with the same sweep count, with
one, two or three steps per pass."""
import numpy as np
import pytest

import oracle.oracle as O
from workloads import SEED_BASE, kog_matrix

pytestmark = pytest.mark.gpu

DT = {"d": np.float64, "z": np.complex128, "s": np.float32, "c": np.complex64}
TOL = {"d": 1e-14, "z": 1e-14, "s": 1e-7, "c": 1e-7}


def _bits(a):
    return np.ascontiguousarray(a).view(np.uint8)


def _mode_flags(S, mode):
    """batch flags for one, two or three steps per pass"""
    return {1: 0, 2: S.SVD2_KOG_TWO_STEP, 3: S.SVD2_KOG_THREE_STEP}[mode]


def _single_flags(S, mode):
    """the single-problem solver's flags for the same steps per pass"""
    return {1: S.SVD2_KOG_UNFUSED, 2: S.SVD2_KOG_TWO_STEP, 3: S.SVD2_KOG_THREE_STEP}[mode]


def _batch(specs, seed):
    mats = []
    for i, (N, kind, cond) in enumerate(specs):
        A = kog_matrix(N, seed + i, cond=cond, cplx=kind in "zc")
        mats.append(np.asfortranarray(A.astype(DT[kind])))
    return mats


@pytest.mark.parametrize("graph", [False, True])
@pytest.mark.parametrize("mode", [1, 2, 3])
def test_mixed_batch_bitwise(graph, mode):
    import torch
    from paper_2005_07403_amd import svd2 as S
    flags = (S.SVD2_KOG_GRAPH if graph else 0) | _mode_flags(S, mode)
    specs = [(2, "d", 10.0), (4, "z", 1e3), (6, "s", 1e2), (32, "d", 1e12), (34, "z", 1e8),
             (64, "s", 1e4), (66, "c", 1e3), (128, "d", 1e6), (130, "z", 1e10), (96, "c", 1e2),
             (40, "s", 1e5), (2, "z", 1.0)]
    mats = _batch(specs, SEED_BASE + 400)
    dev = [torch.from_numpy(m).cuda() for m in mats]
    tols = [TOL[k] for _, k, _ in specs]
    res = S.kog_batch_solve(dev, tols, max_sweeps=40, flags=flags)
    torch.cuda.synchronize()
    for i, ((N, kind, cond), A) in enumerate(zip(specs, mats)):
        ro = O.kog_solve(A, tol=TOL[kind], max_sweeps=40)
        assert res[i]["status"] == 0 == ro["status"], (i, res[i], ro["status"])
        assert res[i]["sweeps"] == ro["sweeps"], (i, res[i], ro["sweeps"])
        got = dev[i].cpu().numpy()
        assert np.array_equal(_bits(got), _bits(A)), (i, N, kind)


@pytest.mark.parametrize("mode", [1, 2, 3])
def test_batch_equals_single_problem_solver(mode):
    """A problem solved inside a batch ends bitwise equal to the same problem
    solved alone by the single-problem entry point (tile shape and batching do
    not change the arithmetic)."""
    import torch
    from paper_2005_07403_amd import svd2 as S
    specs = [(256, "d", 1e12), (200, "z", 1e6), (128, "s", 1e3), (150, "c", 1e3)]
    mats = _batch(specs, SEED_BASE + 410)
    dev = [torch.from_numpy(m).cuda() for m in mats]
    alone = [torch.from_numpy(m).cuda() for m in mats]
    res = S.kog_batch_solve(dev, [TOL[k] for _, k, _ in specs], flags=_mode_flags(S, mode))
    for i, (_, kind, _) in enumerate(specs):
        r = S.kog_solve(alone[i], tol=TOL[kind], flags=_single_flags(S, mode))
        assert r["sweeps"] == res[i]["sweeps"]
        a, b = alone[i].cpu().numpy(), dev[i].cpu().numpy()
        assert np.array_equal(_bits(a), _bits(b))


@pytest.mark.parametrize("mode", [1, 2, 3])
def test_batch_not_converged_and_already_diagonal(mode):
    """A problem stopped by max_sweeps keeps the iterate of its last sweep
    (bitwise the oracle's after that many sweeps; in the two-step mode the
    iterate of order 64 ends a sweep in the second matrix and is copied
    back, in the three-step mode in the caller's); a diagonal input is left
    untouched."""
    import torch
    from paper_2005_07403_amd import svd2 as S
    A = np.asfortranarray(kog_matrix(64, SEED_BASE + 420, cond=1e12))
    D = np.asfortranarray(np.diag(np.arange(1.0, 33.0)))
    dev = [torch.from_numpy(A).cuda(), torch.from_numpy(D).cuda()]
    res = S.kog_batch_solve(dev, [1e-14, 1e-14], max_sweeps=[1, 5], flags=_mode_flags(S, mode))
    assert res[0]["status"] == 7 and res[0]["sweeps"] == 1
    assert res[1]["status"] == 0 and res[1]["sweeps"] == 0
    assert torch.equal(dev[1].cpu(), torch.from_numpy(D))
    ro = O.kog_solve(A, tol=1e-14, max_sweeps=1)
    assert ro["status"] == 7 and ro["sweeps"] == 1
    assert np.array_equal(_bits(dev[0].cpu().numpy()), _bits(A))


@pytest.mark.parametrize("mode", [2, 3])
def test_multi_step_batch_large_orders(mode):
    """Orders up to 1026 (several multi-step tiles per problem in both
    directions, a partial last column tile; orders whose sweeps leave 0, 1
    and 2 steps after the last three-step pass) in the two- and three-step
    batch: each problem bitwise equal to its single-problem solve."""
    import torch
    from paper_2005_07403_amd import svd2 as S
    specs = [(1026, "d", 1e10), (514, "z", 1e6), (770, "s", 1e3), (390, "c", 1e3), (258, "d", 1e2)]
    mats = _batch(specs, SEED_BASE + 430)
    dev = [torch.from_numpy(m).cuda() for m in mats]
    alone = [torch.from_numpy(m).cuda() for m in mats]
    tols = [TOL[k] for _, k, _ in specs]
    res = S.kog_batch_solve(dev, tols, flags=_mode_flags(S, mode) | S.SVD2_KOG_GRAPH)
    for i, (N, kind, _) in enumerate(specs):
        r = S.kog_solve(alone[i], tol=tols[i], flags=_single_flags(S, mode))
        assert r["status"] == res[i]["status"] == 0
        assert r["sweeps"] == res[i]["sweeps"], (N, kind)
        assert np.array_equal(_bits(alone[i].cpu().numpy()), _bits(dev[i].cpu().numpy())), (N, kind)


@pytest.mark.slow
@pytest.mark.parametrize("mode", [2, 3])
def test_full_uneven_batch_multi_step(mode):
    """The 256-problem uneven workload (orders 32..2048, half complex FP64 at
    tol 1e-14, half FP32 at tol 1e-7), solved two or three steps per pass with
    graph replay as the benchmark times it: every problem converges, its
    singular values match the construction within 8 N eps sigma_max, and the
    six smallest problems end bitwise equal to the oracle's single-problem
    solve."""
    from paper_2005_07403_amd import svd2 as S
    from workloads import kog_problem_set_device
    probs = kog_problem_set_device(256, SEED_BASE + 5)
    mats = [p["A"] for p in probs]
    tols = [1e-14 if p["cplx"] else 1e-7 for p in probs]
    small = sorted(range(len(probs)), key=lambda i: probs[i]["order"])[:6]
    host = {i: np.asfortranarray(mats[i].cpu().numpy()) for i in small}
    res = S.kog_batch_solve(mats, tols, max_sweeps=40, flags=S.SVD2_KOG_GRAPH | _mode_flags(S, mode))
    for i, (p, r) in enumerate(zip(probs, res)):
        assert r["status"] == 0 and r["off_rel"] < tols[i], (i, p["order"], r)
        sig = S.kog_sigma(mats[i]).cpu().numpy().astype(np.float64)
        eps = 2.0 ** -52 if p["cplx"] else 2.0 ** -23
        assert np.max(np.abs(sig - p["sigma"])) <= 8 * p["order"] * eps * p["sigma"][0], (i, p["order"])
    for i in small:
        ro = O.kog_solve(host[i], tol=tols[i], max_sweeps=40)
        assert ro["status"] == 0 and ro["sweeps"] == res[i]["sweeps"], (i, probs[i]["order"])
        assert np.array_equal(_bits(mats[i].cpu().numpy()), _bits(host[i])), (i, probs[i]["order"])


def _scaled(A, k):
    """A * 2^k, one component at a time, rounded to the nearest in A's type."""
    if np.iscomplexobj(A):
        return np.asfortranarray(_scaled(A.real, k) + 1j * _scaled(A.imag, k)).astype(A.dtype)
    return np.asfortranarray(A * A.dtype.type(2.0 ** k))


@pytest.mark.parametrize("mode", [1, 2, 3])
def test_batch_tiny_and_huge_matrices(mode):
    """Problems scaled far from 1 (2^+-600 and beyond in FP64, 2^100 and 2^-60
    in FP32) each take the sweeps the oracle takes and end bitwise equal to
    its solve; each problem is scaled by its own power of two."""
    import torch
    from paper_2005_07403_amd import svd2 as S
    specs = [(64, "d", 1e6, 600), (66, "d", 1e6, -1000), (34, "z", 1e4, 700), (32, "z", 1e4, -700),
             (64, "s", 1e3, 100), (40, "c", 1e2, -60), (6, "c", 1e2, 100), (130, "d", 1e8, 0)]
    mats = [_scaled(m, k) for m, (_, _, _, k) in zip(_batch([s[:3] for s in specs], SEED_BASE + 430), specs)]
    dev = [torch.from_numpy(m).cuda() for m in mats]
    res = S.kog_batch_solve(dev, [TOL[s[1]] for s in specs], max_sweeps=40, flags=_mode_flags(S, mode))
    torch.cuda.synchronize()
    for i, ((N, kind, _, k), A) in enumerate(zip(specs, mats)):
        ro = O.kog_solve(A, tol=TOL[kind], max_sweeps=40)
        assert res[i]["status"] == 0 == ro["status"], (i, res[i], ro["status"])
        assert res[i]["sweeps"] == ro["sweeps"] > 0, (i, res[i], ro["sweeps"])
        assert np.array_equal(_bits(dev[i].cpu().numpy()), _bits(A)), (i, N, kind, k)


@pytest.mark.parametrize("mode", [1, 2, 3])
def test_batch_padded_leading_dimensions(mode):
    """Problems stored with lda > N (views into taller matrices) in every
    mode: each ends bitwise equal to the oracle's solve, with the oracle's
    sweep count, and the padding rows stay untouched (in the multi-step modes
    the iterate passes through the workspace's matrix, whose lda is N)."""
    import torch
    from paper_2005_07403_amd import svd2 as S
    specs = [(66, "d", 1e6), (40, "z", 1e4), (70, "s", 1e3), (34, "c", 1e2)]
    mats = _batch(specs, SEED_BASE + 440)
    pads = [3, 5, 1, 8]
    bigs, views = [], []
    for A, pad, (N, kind, _) in zip(mats, pads, specs):
        big = np.asfortranarray(np.full((N + pad, N), 7, dtype=DT[kind]))
        big[:N, :] = A
        g = torch.from_numpy(big).cuda()
        bigs.append(g)
        views.append(g[:N, :])
        assert views[-1].stride(1) == N + pad
    res = S.kog_batch_solve(views, [TOL[k] for _, k, _ in specs], max_sweeps=40,
                            flags=S.SVD2_KOG_GRAPH | _mode_flags(S, mode))
    torch.cuda.synchronize()
    for i, ((N, kind, _), A) in enumerate(zip(specs, mats)):
        ro = O.kog_solve(A, tol=TOL[kind], max_sweeps=40)
        assert res[i]["status"] == 0 == ro["status"], (i, res[i])
        assert res[i]["sweeps"] == ro["sweeps"], (i, res[i], ro["sweeps"])
        out = bigs[i].cpu().numpy()
        assert np.array_equal(_bits(np.asfortranarray(out[:N, :])), _bits(A)), (i, N, kind)
        assert np.all(out[N:, :] == 7), (i, N, kind)
