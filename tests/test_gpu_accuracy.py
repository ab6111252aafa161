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
