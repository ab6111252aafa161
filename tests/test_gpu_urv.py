"""GPU parity of the phase outputs of the URV factorization (section 2.2: R of
eq. (9), U_+ and V_+ of eq. (11)), written by the *_batch_urv entry points
beside the final results: byte for byte the oracle's (signed zeros included),
and the main outputs byte for byte those of the plain entry point, in every
flag combination the entry points accept."""
import numpy as np
import pytest

import oracle.oracle as O
from tests.gpu_util import to_dev
from workloads import SEED_BASE, random_bits, scaled_law, to_trains, uniform_real

pytestmark = pytest.mark.gpu

KINDS = {"d": (np.float64, False), "z": (np.float64, True), "s": (np.float32, False), "c": (np.float32, True)}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2005_07403_amd import svd2 as S
    S.lib()
    yield
    S.svd2_set_launch(256, 1)


def _hand(cplx, dt):
    """the hand cases of the oracle's pins (diagonal with signs, each swap,
    a phase), as columns in element order 11, 21, 12, 22"""
    cols = [[3, 0, 0, -2], [-1, 0, 0, 4], [0, -2, 0, 0], [2, 0, 1, 1], [0, 0, 0, 0]]
    if cplx:
        cols += [[1j, 0, 0, 1], [2, 0, 1j, 1]]
    A = np.array(cols).T
    return A.astype((np.complex128 if dt == np.float64 else np.complex64) if cplx else dt)


def _inputs(kind, n, seed):
    dt, cplx = KINDS[kind]
    A = scaled_law(n, seed, cplx, dtype=dt, special_frac=0.05)
    B = random_bits(n // 8, seed + 1, cplx, dtype=dt)
    C = uniform_real(n // 8, seed + 2, dtype=dt)
    if cplx:
        C = C.astype(np.complex128 if dt == np.float64 else np.complex64)
    return np.concatenate([_hand(cplx, dt), A, B, C], axis=1), dt, cplx


def _bytes(t):
    return np.ascontiguousarray(t).view(np.uint8)


MODES = {"plain": 0, "no_uv": "NO_UV", "sine": "SINE_FORM", "tail": "RESCUE_FP64",
         "sigma": "RESCUE_FP64|RESCUE_SIGMA", "tri": "RESCUE_FP64|RESCUE_TRI",
         "queue": "RESCUE_FP64|RESCUE_QUEUE", "queue_nouv": "RESCUE_FP64|RESCUE_QUEUE|NO_UV"}


def _flags(S, mode):
    v = MODES[mode]
    if v == 0:
        return 0
    f = 0
    for name in v.split("|"):
        f |= getattr(S, "SVD2_" + name)
    return f


@pytest.mark.parametrize("upv", [True, False], ids=["r_u_v", "r_only"])
@pytest.mark.parametrize("mode", list(MODES))
@pytest.mark.parametrize("kind", ["d", "z", "s", "c"])
def test_phase_outputs_bitwise(kind, mode, upv):
    import torch
    from paper_2005_07403_amd import svd2 as S
    dt, cplx = KINDS[kind]
    if dt == np.float64 and (mode.startswith("queue") or mode in ("tail", "sigma", "tri")):
        pytest.skip("rescue flags are FP32 only")
    flags = _flags(S, mode)
    A, dt, cplx = _inputs(kind, 20000 + 37, SEED_BASE + 800 + ord(kind))
    n = A.shape[1]
    tr = to_trains(A, dt)
    dev = to_dev(tr)
    tdt = torch.float64 if dt == np.float64 else torch.float32
    nf = (19 if cplx else 11) if upv else 3
    f = [torch.full((n,), float("nan"), dtype=tdt, device="cuda") for _ in range(nf)]
    c1 = torch.zeros(1, dtype=torch.int32, device="cuda")
    c2 = torch.zeros(1, dtype=torch.int32, device="cuda")
    fp32 = dt == np.float32
    plain = S.svd2(dev, flags=flags, nrescued=c1 if fp32 else None)
    out, f = S.svd2(dev, flags=flags, nrescued=c2 if fp32 else None, urv=f)
    torch.cuda.synchronize()
    assert len(out) == len(plain)
    for a, b in zip(out, plain):
        assert np.array_equal(_bytes(a.cpu().numpy()), _bytes(b.cpu().numpy()))
    if fp32:
        assert int(c1.item()) == int(c2.item())
        assert (int(c1.item()) > 0) == bool(flags & S.SVD2_RESCUE_FP64)
    ora = O.urv(A, dtype=dt)["trains"]
    for i in range(nf):
        g = f[i].cpu().numpy()
        same = _bytes(g).reshape(n, -1) == _bytes(ora[i]).reshape(n, -1)
        bad = np.nonzero(~same.all(axis=1))[0]
        assert bad.size == 0, (kind, mode, i, bad[:5], g[bad[:5]], ora[i][bad[:5]])


@pytest.mark.parametrize("kind", ["d", "c"])
@pytest.mark.parametrize("n", [1, 63, 65, 257])
def test_phase_outputs_small_and_ragged(kind, n):
    """batches of one lane, and ragged against the wavefront and workgroup"""
    import torch
    from paper_2005_07403_amd import svd2 as S
    dt, cplx = KINDS[kind]
    A = scaled_law(n, SEED_BASE + 850 + n, cplx, dtype=dt, special_frac=0.1)
    tr = to_trains(A, dt)
    tdt = torch.float64 if dt == np.float64 else torch.float32
    f = [torch.empty(n, dtype=tdt, device="cuda") for _ in range(19 if cplx else 11)]
    _, f = S.svd2(to_dev(tr), flags=S.SVD2_RESCUE_FP64 if dt == np.float32 else 0, urv=f)
    torch.cuda.synchronize()
    ora = O.urv(A, dtype=dt)["trains"]
    for g, o in zip(f, ora):
        assert np.array_equal(_bytes(g.cpu().numpy()), _bytes(o))


def test_phase_outputs_over_several_launches():
    """A batch longer than one launch's span (2^30 bytes per array): n = 2^28
    + 3 real FP32 matrices, singular values and R only.  R at the lanes around
    the boundary between launches and a random sample elsewhere is the
    oracle's; smax, smin and s are those of the plain call."""
    import torch
    from paper_2005_07403_amd import svd2 as S
    n = (1 << 28) + 3
    A = scaled_law(n, SEED_BASE + 861, False, dtype=np.float32)
    tr = to_trains(A)
    del A
    dev = [torch.from_numpy(t).cuda() for t in tr]
    flags = S.SVD2_RESCUE_FP64 | S.SVD2_RESCUE_SIGMA | S.SVD2_NO_UV
    plain = S.svd2(dev, flags=flags)
    f = [torch.empty(n, dtype=torch.float32, device="cuda") for _ in range(3)]
    out, f = S.svd2(dev, flags=flags, urv=f)
    torch.cuda.synchronize()
    for a, b in zip(out, plain):
        assert torch.equal(a.view(torch.int32), b.view(torch.int32))
    del plain, out
    rng = np.random.default_rng(SEED_BASE + 862)
    idx = np.unique(np.concatenate([np.arange((1 << 28) - 300, n), np.arange(0, 64),
                                    rng.choice(n, 1 << 18, replace=False)]))
    tidx = torch.from_numpy(idx).cuda()
    sub = np.stack([t[idx] for t in tr])
    ora = O.urv(sub, dtype=np.float32)["trains"]
    for g, o in zip(f, ora):
        assert np.array_equal(_bytes(g[tidx].cpu().numpy()), _bytes(o))
