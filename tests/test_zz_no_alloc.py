"""dkog_solve_noalloc (the Kogbetliantz solve on the library's fixed device
workspace) against dkog_solve with a caller workspace, through the C ABI:
bitwise the same iterate, sweep count, status and off-norm, on two calls in a
row (the second on a smaller matrix, so it runs on what the first left in the
fixed workspace), in the fused and the unfused mode."""
import ctypes

import numpy as np
import pytest

import oracle.oracle as O
from workloads import SEED_BASE, kog_matrix

pytestmark = pytest.mark.gpu


def _bits(a):
    return np.ascontiguousarray(a).view(np.uint8)


def _solve_pair(N, seed, flags):
    import torch
    from paper_2005_07403_amd import svd2 as S
    L = S._kog()
    A = np.asfortranarray(kog_matrix(N, seed, cond=1e8))
    G0 = torch.from_numpy(A).cuda()
    G1 = torch.from_numpy(A).cuda()
    assert G0.stride(0) == 1 and G1.stride(0) == 1
    ws = S.kog_workspace(G0, flags)
    st = torch.cuda.current_stream().cuda_stream
    sw0, off0 = ctypes.c_int(-1), ctypes.c_double(-1.0)
    sw1, off1 = ctypes.c_int(-1), ctypes.c_double(-1.0)
    print(f"[no_alloc] N={N} seed={seed} flags={flags}: dkog_solve", flush=True)
    r0 = L.dkog_solve(N, G0.data_ptr(), N, 1e-14, 40, ctypes.byref(sw0), ctypes.byref(off0), ws.data_ptr(),
                      ws.numel(), flags, st)
    print(f"[no_alloc] N={N} seed={seed} flags={flags}: dkog_solve_noalloc", flush=True)
    r1 = L.dkog_solve_noalloc(N, G1.data_ptr(), N, 1e-14, 40, ctypes.byref(sw1), ctypes.byref(off1), flags, st)
    torch.cuda.synchronize()
    assert r0 == 0 and r1 == 0, (r0, r1)
    assert sw1.value == sw0.value and sw0.value > 0
    assert _bits(np.array([off1.value])).tolist() == _bits(np.array([off0.value])).tolist()
    M0, M1 = G0.cpu().numpy(), G1.cpu().numpy()
    assert np.array_equal(_bits(M1), _bits(M0)), f"N={N}: the iterates differ"
    return A, M1, sw1.value


@pytest.mark.parametrize("flags", [0, 1], ids=["fused", "unfused"])
def test_noalloc_solve_matches_the_workspace_solve(flags):
    import torch
    assert torch.cuda.is_available()
    # first call: order 130 (a ragged last tile); second: order 66, smaller,
    # on the fixed workspace as the first call left it
    _solve_pair(130, SEED_BASE + 701, flags)
    A, M, sweeps = _solve_pair(66, SEED_BASE + 702, flags)
    # and both against the oracle, which solves its copy in place
    B = np.array(A, order="F")
    ro = O.kog_solve(B, tol=1e-14)
    assert ro["status"] == 0 and ro["sweeps"] == sweeps
    assert np.array_equal(_bits(M), _bits(B)), "the iterate differs from the oracle's"
