"""Accuracy of the two assemblies of U on the GPU: the tangent form of
eq. (29) (the default) against the sine form of eq. (31) (SVD2_SINE_FORM),
the comparison of section 8 (Figs. 12-14), there between the vectorized
routine and a pointwise one that assembles by eq. (31).  Per batch the
maxima of rho, delta and eta (eqs. (33)-(35)) are computed in binary128 by
the oracle; both forms must stay within 16 eps, and the table of maxima is
printed (run with -s to see it)."""
import numpy as np
import pytest

import oracle.oracle as O
from workloads import SEED_BASE, random_bits, scaled_law, to_trains

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available()
    from paper_2005_07403_amd import svd2 as S
    S.lib()
    yield


@pytest.mark.parametrize("law", ["bits", "scaled"])
@pytest.mark.parametrize("cplx", [False, True])
def test_tangent_and_sine_form_accuracy(cplx, law):
    import torch
    from paper_2005_07403_amd import svd2 as S
    eps = 2.0 ** -52
    n, batches = 1 << 18, 8
    rows = []
    for b in range(batches):
        seed = SEED_BASE + 900 + 16 * b + (1 if cplx else 0)
        A = random_bits(n, seed, cplx) if law == "bits" else scaled_law(n, seed, cplx)
        tr = to_trains(A, np.float64)
        dev = [torch.from_numpy(t).cuda() for t in tr]
        row = []
        for flags in (0, S.SVD2_SINE_FORM):
            out = [o.cpu().numpy() for o in S.svd2(dev, flags=flags)]
            torch.cuda.synchronize()
            met = O.metrics(tr, out, cplx)
            vals = [float(np.nanmax(met[k])) / eps for k in ("rho", "delta", "eta")]
            assert max(vals) <= 16, (b, flags, vals)
            row += vals
        rows.append(row)
    r = np.array(rows)
    name = ("complex" if cplx else "real") + f" FP64, {law}, {batches} batches of {n}"
    print(f"\n{name}: max over each batch, in eps (tangent | sine)")
    print("batch   rho_t  rho_s   delta_t delta_s   eta_t  eta_s")
    for b, x in enumerate(r):
        print(f"{b:5d}  {x[0]:6.3f} {x[3]:6.3f}   {x[1]:6.3f}  {x[4]:6.3f}   {x[2]:6.3f} {x[5]:6.3f}")
    wins = [(int((r[:, i] < r[:, i + 3]).sum()), int((r[:, i] > r[:, i + 3]).sum())) for i in range(3)]
    print(f"tangent smaller / sine smaller: rho {wins[0]}, delta {wins[1]}, eta {wins[2]}")


@pytest.mark.parametrize("mode", ["none", "fp64_tail", "sigma_quotient", "fp64_triangle"])
@pytest.mark.parametrize("cplx", [False, True])
def test_fp32_form_error_against_fp64(cplx, mode):
    """The FP32 form on the GPU against the FP64 oracle run on the exact
    upcast inputs (the +-m 2^e law in FP32, 2^18 matrices), in units of
    eps32 = 2^-23: the relative error of sigma'_max, that of sigma'_min on the
    lanes where the FP64 value, brought exactly to the FP32 lane's scale
    (times 2^(s32 - s64)), is a normal FP32 number, and rho, delta, eta of the
    FP32 outputs in binary128.  sigma'_max within 8 eps32 and rho, delta, eta
    within 16 eps32 in every mode.  sigma'_min: on the lanes the FP32 path
    flags as near-degenerate (sigma'_min < 2^-20 sigma'_max) within 8 eps32
    relative with either rescue, on the others within 8 kappa eps32 (kappa =
    sigma_max / sigma_min < 2^20 there: the FP32 triangular factor is only
    normwise accurate); normwise within 8 eps32 everywhere; and within one
    subnormal step (2^-149) of the scaled FP64 value where that is below the
    normal range (a matrix whose singular values span more than the FP32
    range has no closer FP32 sigma'_min).  Run with -s for the table."""
    import torch
    from paper_2005_07403_amd import svd2 as S
    e32 = 2.0 ** -23
    n = 1 << 18
    A = scaled_law(n, SEED_BASE + 950 + (1 if cplx else 0), cplx, dtype=np.float32)
    tr32 = to_trains(A, np.float32)
    flags = {"none": 0, "fp64_tail": S.SVD2_RESCUE_FP64,
             "sigma_quotient": S.SVD2_RESCUE_FP64 | S.SVD2_RESCUE_SIGMA,
             "fp64_triangle": S.SVD2_RESCUE_FP64 | S.SVD2_RESCUE_TRI}[mode]
    dev = [torch.from_numpy(t).cuda() for t in tr32]
    out = [o.cpu().numpy() for o in S.svd2(dev, flags=flags)]
    torch.cuda.synchronize()
    tr64 = [t.astype(np.float64) for t in tr32]
    o64, _ = O.run_trains(tr64, cplx, np.float64)
    # the lanes the FP32 path flags (the GPU's outputs are bitwise the oracle's)
    _, flagged = O.run_trains(tr32, cplx, np.float32, rescue=1)
    k = 16 if cplx else 8
    nz = o64[k] > 0  # the zero matrix has sigma' = 0 on both sides
    fl = flagged.astype(bool)[nz]
    shift = (out[k + 2][nz].astype(np.int64) - o64[k + 2][nz].astype(np.int64))
    smax32, smin32 = out[k][nz].astype(np.float64), out[k + 1][nz].astype(np.float64)
    smax64, smin64 = np.ldexp(o64[k][nz], shift), np.ldexp(o64[k + 1][nz], shift)
    rmax = np.max(np.abs(smax32 - smax64) / smax64) / e32
    normal = smin64 >= 2.0 ** -126
    relmin = np.abs(smin32 - smin64) / np.where(normal, smin64, 1.0) / e32
    rmin = np.max(relmin[normal & fl], initial=0.0)
    kappa = smax64 / np.where(normal, smin64, 1.0)
    rkap = np.max((relmin / kappa)[normal & ~fl], initial=0.0)
    sub = np.max(np.abs(smin32[~normal] - smin64[~normal]), initial=0.0) / 2.0 ** -149
    nmin = np.max(np.abs(smin32 - smin64) / smax64) / e32
    met = O.metrics(tr32, out, cplx)
    rho, dlt, eta = (float(np.nanmax(met[x])) / e32 for x in ("rho", "delta", "eta"))
    print(f"\nFP32 {'complex' if cplx else 'real'}, rescue {mode}: sigma_max rel {rmax:.2f}; sigma_min rel "
          f"{rmin:.3g} on {int((normal & fl).sum())} flagged lanes, {rkap:.2f} kappa on the other "
          f"{int((normal & ~fl).sum())}, normwise {nmin:.2f}, {int((~normal).sum())} lanes below the normal "
          f"range within {sub:.2f} subnormal steps; rho {rho:.2f}, delta {dlt:.2f}, eta {eta:.2f} (eps32)")
    assert rmax <= 8 and nmin <= 8 and rkap <= 8
    assert max(rho, dlt, eta) <= 16
    if mode != "none":
        assert rmin <= 8 and sub <= 1
