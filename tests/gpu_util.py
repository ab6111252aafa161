"""Helpers shared by the GPU tests: upload SoA trains, run the HIP path through
the C ABI, compare with the oracle."""
import numpy as np

import oracle.oracle as O


def to_dev(trains):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(t)).cuda() for t in trains]


def run_gpu(trains_np, flags=0, nrescued=False, queue=False):
    import torch
    from paper_2005_07403_amd import svd2 as S
    dev = to_dev(trains_np)
    cnt = torch.zeros(1, dtype=torch.int32, device="cuda") if nrescued else None
    out = S.svd2(dev, flags=flags, nrescued=cnt)
    torch.cuda.synchronize()
    res = [o.cpu().numpy() for o in out]
    if nrescued:
        return res, int(cnt.item())
    return res


def ulp_diff(a, b):
    """ulps between same-dtype arrays (sign-magnitude ordering; +0 == -0)."""
    it = np.int64 if a.dtype == np.float64 else np.int32
    ia = a.view(it).astype(np.int64)
    ib = b.view(it).astype(np.int64)
    m = np.int64(0x7FFFFFFFFFFFFFFF) if a.dtype == np.float64 else np.int64(0x7FFFFFFF)
    ia = np.where(ia < 0, -(ia & m), ia)
    ib = np.where(ib < 0, -(ib & m), ib)
    return np.abs(ia - ib)


def same_bits(a, b):
    a = np.where(a == 0, 0, a).astype(a.dtype)
    b = np.where(b == 0, 0, b).astype(b.dtype)
    it = np.uint64 if a.dtype == np.float64 else np.uint32
    return a.view(it) == b.view(it)


def compare(gpu, ora, cplx, eps, lanes=None):
    """Parity of one batch.  Returns a dict of statistics; asserts the bar:
    s exact, sigma' within 4 ulp, U and V within 4 eps absolute (their entries
    are bounded by one), and reports the count of bitwise-identical lanes."""
    k = 16 if cplx else 8
    n = gpu[0].shape[0]
    sel = slice(None) if lanes is None else lanes
    g = [x[sel] for x in gpu]
    o = [x[sel] for x in ora]
    s_ok = same_bits(g[k + 2], o[k + 2])
    assert s_ok.all(), f"s differs on {np.count_nonzero(~s_ok)} lanes"
    umax = max(int(ulp_diff(g[k], o[k]).max()), int(ulp_diff(g[k + 1], o[k + 1]).max()))
    assert umax <= 4, f"sigma' differs by {umax} ulp"
    uv = max(float(np.max(np.abs(g[i].astype(np.float64) - o[i]))) for i in range(k))
    assert uv <= 4 * eps, f"U/V differ by {uv / eps} eps"
    exact = np.ones(g[0].shape[0], dtype=bool)
    for i in range(len(g)):
        exact &= same_bits(g[i], o[i])
    return dict(n=n, sigma_max_ulp=umax, uv_max_abs_eps=uv / eps,
                bitwise_lanes=int(exact.sum()), lanes=int(exact.size))


def oracle_outs(trains_np, cplx, dtype, rescue=False, backscale="none"):
    outs, flagged = O.run_trains(trains_np, cplx, dtype, policy="mirror", backscale=backscale,
                                 rescue=rescue)
    return outs, flagged
