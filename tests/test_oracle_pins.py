"""Pins of the CPU oracle against what the mathematics fixes (no GPU).

Each test checks the oracle against something other than itself:
closed-form singular values in exact/50-digit arithmetic, exact rational
residuals, invariants of Theorem 1, identities of section 2 (power-of-two
scaling, real = complex with zero imaginary parts), hand cases and the
constants printed in the paper.
"""
import itertools
import os
from fractions import Fraction

import mpmath as mp
import numpy as np
import pytest

import oracle.oracle as O
from workloads import random_bits, scaled_law, uniform_real

EPS64 = 2.0 ** -52
EPS32 = 2.0 ** -23
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
mp.mp.dps = 60


# ---------------------------------------------------------------------------
# helpers (independent of the oracle's arithmetic)
# ---------------------------------------------------------------------------

def exact_sigma(entries):
    """Closed-form singular values of a 2x2 matrix with exactly representable
    entries: sigma_max,min = (sqrt(F+2D) +- sqrt(F-2D))/2, F = ||A||_F^2,
    D = |det A|, with F and D^2 formed exactly in rationals."""
    a11, a21, a12, a22 = [Fraction(complex(x).real) + 0 for x in entries]
    i11, i21, i12, i22 = [Fraction(complex(x).imag) for x in entries]
    F = sum(v * v for v in (a11, a21, a12, a22, i11, i21, i12, i22))
    # det = a11 a22 - a12 a21 (complex)
    dr = (a11 * a22 - i11 * i22) - (a12 * a21 - i12 * i21)
    di = (a11 * i22 + i11 * a22) - (a12 * i21 + i12 * a21)
    D2 = dr * dr + di * di
    Fm = mp.mpf(F.numerator) / F.denominator
    D = mp.sqrt(mp.mpf(D2.numerator) / D2.denominator)
    p, q = mp.sqrt(Fm + 2 * D), mp.sqrt(max(Fm - 2 * D, mp.mpf(0)))
    smax = (p + q) / 2
    smin = (2 * D) / (p + q) if D != 0 else mp.mpf(0)
    return smax, smin


def backscaled(r, k):
    """sigma = 2^-s sigma' as exact mp numbers."""
    s = r["s"][k]
    big = np.finfo(r["smax"].dtype).max
    if s == big:
        return mp.mpf(float(r["smax"][k])), mp.mpf(float(r["smin"][k]))
    return (mp.ldexp(mp.mpf(float(r["smax"][k])), -int(s)),
            mp.ldexp(mp.mpf(float(r["smin"][k])), -int(s)))


def int_matrices_real():
    v = range(-4, 5)
    return np.array(list(itertools.product(v, repeat=4)), dtype=np.float64).T


def int_matrices_complex():
    v = (-1.0, 0.0, 1.0)
    c = np.array(list(itertools.product(v, repeat=8)), dtype=np.float64).T
    return c[0::2] + 1j * c[1::2]


def as_trains(r):
    return r["inputs"], r["trains"]


# ---------------------------------------------------------------------------
# paper constants (golden fixture)
# ---------------------------------------------------------------------------

def test_golden_constants():
    """The tan(2 phi) clamp printed in Fig. 10 and h of section 2.1."""
    vals = {}
    with open(os.path.join(GOLDEN, "paper_constants.txt")) as fh:
        for line in fh:
            line = line.split("#")[0].strip()
            if line:
                k, v = line.split("=")
                vals[k.strip()] = v.strip()
    f = float(vals["sqrt_dbl_max_fig10"])
    assert f == float.fromhex("0x1.fffffffffffffp+511")
    assert f * f < np.finfo(np.float64).max
    assert int(vals["h_double"]) == 1024 - 3
    # A matrix whose single entry has exponent h+1 forces s = -2 (section 2.1: -2 <= s)
    r = O.svd2(np.array([[np.finfo(np.float64).max], [0.0], [0.0], [0.0]]))
    assert r["s"][0] == -2.0
    r = O.svd2(np.array([[2.0 ** 1022], [0.0], [0.0], [0.0]]))
    assert r["s"][0] == -1.0


# ---------------------------------------------------------------------------
# closed-form singular values, exhaustive small integers
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("policy", ["mirror", "ref"])
@pytest.mark.parametrize("k", [0, -1070, -600, 600, 1020])
def test_exhaustive_real_closed_form(policy, k):
    M = int_matrices_real()
    A = np.ldexp(M, k)
    r = O.svd2(A, policy=policy)
    worst_max = worst_min = 0.0
    for j in range(M.shape[1]):
        if not M[:, j].any():
            continue
        xs, ns = exact_sigma(M[:, j])
        smax, smin = backscaled(r, j)
        smax, smin = mp.ldexp(smax, -k), mp.ldexp(smin, -k)
        worst_max = max(worst_max, float(abs(smax - xs) / xs))
        worst_min = max(worst_min, float(abs(smin - ns) / xs))
    # sigma_max relatively, sigma_min normwise (relative to sigma_max)
    assert worst_max <= 4 * EPS64, worst_max / EPS64
    assert worst_min <= 4 * EPS64, worst_min / EPS64


@pytest.mark.parametrize("policy", ["mirror", "ref"])
def test_exhaustive_complex_closed_form(policy):
    M = int_matrices_complex()
    r = O.svd2(M, policy=policy)
    worst_max = worst_min = 0.0
    for j in range(M.shape[1]):
        if not np.any(M[:, j]):
            continue
        xs, ns = exact_sigma(M[:, j])
        smax, smin = backscaled(r, j)
        worst_max = max(worst_max, float(abs(smax - xs) / xs))
        worst_min = max(worst_min, float(abs(smin - ns) / xs))
    assert worst_max <= 4 * EPS64, worst_max / EPS64
    assert worst_min <= 4 * EPS64, worst_min / EPS64


# ---------------------------------------------------------------------------
# residual / orthogonality metrics: pin the binary128 metric code with exact
# rational arithmetic, then use it
# ---------------------------------------------------------------------------

def _frac_metrics(ins, outs, k, cplx):
    F = lambda x: Fraction(float(x))
    if cplx:
        A = [[(F(ins[0][k]), F(ins[1][k])), (F(ins[4][k]), F(ins[5][k]))],
             [(F(ins[2][k]), F(ins[3][k])), (F(ins[6][k]), F(ins[7][k]))]]
        U = [[(F(outs[0][k]), F(outs[1][k])), (F(outs[4][k]), F(outs[5][k]))],
             [(F(outs[2][k]), F(outs[3][k])), (F(outs[6][k]), F(outs[7][k]))]]
        V = [[(F(outs[8][k]), F(outs[9][k])), (F(outs[12][k]), F(outs[13][k]))],
             [(F(outs[10][k]), F(outs[11][k])), (F(outs[14][k]), F(outs[15][k]))]]
        smax, smin, s = outs[16][k], outs[17][k], outs[18][k]
    else:
        A = [[(F(ins[0][k]), 0), (F(ins[2][k]), 0)], [(F(ins[1][k]), 0), (F(ins[3][k]), 0)]]
        U = [[(F(outs[0][k]), 0), (F(outs[2][k]), 0)], [(F(outs[1][k]), 0), (F(outs[3][k]), 0)]]
        V = [[(F(outs[4][k]), 0), (F(outs[6][k]), 0)], [(F(outs[5][k]), 0), (F(outs[7][k]), 0)]]
        smax, smin, s = outs[8][k], outs[9][k], outs[10][k]
    sig = [F(smax) * Fraction(2) ** (-int(s)), F(smin) * Fraction(2) ** (-int(s))]
    mul = lambda a, b: (a[0] * b[0] - a[1] * b[1], a[0] * b[1] + a[1] * b[0])
    cj = lambda a: (a[0], -a[1])
    num = den = Fraction(0)
    for i in range(2):
        for j in range(2):
            acc = (Fraction(0), Fraction(0))
            for l in range(2):
                t = mul(U[i][l], cj(V[j][l]))
                acc = (acc[0] + sig[l] * t[0], acc[1] + sig[l] * t[1])
            d = (acc[0] - A[i][j][0], acc[1] - A[i][j][1])
            num += d[0] ** 2 + d[1] ** 2
            den += A[i][j][0] ** 2 + A[i][j][1] ** 2

    def orth(X):
        acc = Fraction(0)
        for i in range(2):
            for j in range(2):
                g = (Fraction(0), Fraction(0))
                for l in range(2):
                    t = mul(cj(X[l][i]), X[l][j])
                    g = (g[0] + t[0], g[1] + t[1])
                if i == j:
                    g = (g[0] - 1, g[1])
                acc += g[0] ** 2 + g[1] ** 2
        return acc

    rho2 = num / den
    return (float(mp.sqrt(mp.mpf(rho2.numerator) / rho2.denominator)),
            float(mp.sqrt(mp.mpf(orth(U).numerator) / orth(U).denominator)),
            float(mp.sqrt(mp.mpf(orth(V).numerator) / orth(V).denominator)))


@pytest.mark.parametrize("cplx", [False, True])
def test_metric_code_matches_exact_rationals(cplx):
    A = scaled_law(200, 11, cplx, emin=-60, emax=60, special_frac=0.0)
    r = O.svd2(A)
    ins, outs = as_trains(r)
    met = O.metrics(ins, outs, cplx)
    for k in range(0, 200, 7):
        rho, delta, eta = _frac_metrics(ins, outs, k, cplx)
        for got, want in ((met["rho"][k], rho), (met["delta"][k], delta), (met["eta"][k], eta)):
            assert abs(got - want) <= 1e-25 + 1e-20 * want, (k, got, want)


@pytest.mark.parametrize("policy", ["mirror", "ref"])
@pytest.mark.parametrize("law", ["uniform", "scaled", "bits"])
@pytest.mark.parametrize("cplx", [False, True])
def test_residual_orthogonality_bound(policy, law, cplx):
    n = 20000
    if law == "uniform":
        A = uniform_real(n, 1)
        if cplx:
            A = A + 1j * uniform_real(n, 2)
    elif law == "scaled":
        A = scaled_law(n, 3, cplx)
    else:
        A = random_bits(n, 4, cplx)
    r = O.svd2(A, policy=policy)
    met = O.metrics(*as_trains(r), cplx)
    for key in ("rho", "delta", "eta"):
        assert np.all(met[key] <= 16 * EPS64), (key, met[key].max() / EPS64)


# ---------------------------------------------------------------------------
# identities of section 2
# ---------------------------------------------------------------------------

def _same_bits(a, b):
    """bitwise equality up to the sign of zero"""
    a = np.where(a == 0, 0.0, a)
    b = np.where(b == 0, 0.0, b)
    return np.array_equal(a.view(np.uint64), b.view(np.uint64)) if a.dtype == np.float64 else \
        np.array_equal(a.view(np.uint32), b.view(np.uint32))


@pytest.mark.parametrize("cplx", [False, True])
def test_power_of_two_invariance(cplx):
    """Section 2.1: scaling by 2^s is exact, so A 2^k gives the same A^ and
    therefore bitwise the same U, V, sigma', with s shifted by -k."""
    # no special lanes: every entry keeps its exponent in [-700, 650] after scaling
    A = scaled_law(4000, 5, cplx, emin=-400, emax=400, special_frac=0.0)
    A[:, ::50] = 0  # zero matrices stay zero (s = BIG) and are skipped below
    base = O.svd2(A)
    for k in (-300, -17, 1, 250):
        r = O.svd2(A * 2.0 ** k)
        nz = base["s"] != np.finfo(np.float64).max
        assert np.array_equal(r["s"][nz], base["s"][nz] - k)
        for i in range(len(base["trains"]) - 1):
            assert _same_bits(r["trains"][i], base["trains"][i]), i


def test_real_equals_complex_with_zero_imag():
    """The real path (sign-bit D*, D~, D^ of eq. (10)) must agree with the
    complex path (eqs. (1), (4), (8), (9)) on real data.  Where an entry is an
    exact zero the two paths may see a zero pivot with opposite signs (sign
    bits versus fma results) and legitimately pick the other sign for a
    column of U and V; there sigma must still agree bitwise and both results
    must be valid SVDs."""
    A = np.concatenate([uniform_real(3000, 7), scaled_law(3000, 8, False),
                        random_bits(3000, 9, False)], axis=1)
    rd = O.svd2(A)
    rz = O.svd2(A.astype(np.complex128))
    for key in ("smax", "smin", "s"):
        assert _same_bits(rd[key], rz[key]), key
    generic = np.all(A != 0, axis=0)
    assert generic.mean() > 0.98
    for X in ("U", "V"):
        assert _same_bits(rd[X][:, generic].ravel(), rz[X][:, generic].real.ravel().copy())
        assert np.all(rz[X].imag == 0)
    for r, cplx in ((rd, False), (rz, True)):
        met = O.metrics(r["inputs"], r["trains"], cplx)
        for key in ("rho", "delta", "eta"):
            assert met[key].max() <= 16 * EPS64


def test_exact_sigma_on_diagonal():
    rng = np.random.default_rng(12)
    a = scaled_law(2000, 13, False, special_frac=0)[0]
    b = scaled_law(2000, 14, False, special_frac=0)[0]
    A = np.stack([a, np.zeros_like(a), np.zeros_like(a), b])
    r = O.svd2(A, backscale="safe")
    ok = r["s"] == 0  # backscaled lanes
    big = np.maximum(np.abs(a), np.abs(b))
    small = np.minimum(np.abs(a), np.abs(b))
    assert ok.mean() > 0.5
    assert np.array_equal(r["smax"][ok], big[ok])
    assert np.array_equal(r["smin"][ok], small[ok])
    del rng


def test_zero_matrix():
    for cplx in (False, True):
        A = np.zeros((4, 3), dtype=np.complex128 if cplx else np.float64)
        r = O.svd2(A)
        assert np.all(r["s"] == np.finfo(np.float64).max)
        assert np.all(r["smax"] == 0) and np.all(r["smin"] == 0)
        eye = np.array([1, 0, 0, 1.0])[:, None]
        assert np.array_equal(np.abs(r["U"]), np.broadcast_to(eye, (4, 3)))
        assert np.array_equal(np.abs(r["V"]), np.broadcast_to(eye, (4, 3)))


def test_rank_one_and_triangular_and_extremes():
    rng = np.random.default_rng(15)
    u = rng.standard_normal((2, 500))
    v = rng.standard_normal((2, 500))
    A = np.stack([u[0] * v[0], u[1] * v[0], u[0] * v[1], u[1] * v[1]])
    r = O.svd2(A)
    assert np.all(r["smin"] <= 4 * EPS64 * r["smax"])
    # entries near DBL_MAX: s in {-1, -2}, sigma' finite
    big = np.finfo(np.float64).max * (1 - rng.random((4, 500)) / 16)
    r = O.svd2(big * np.sign(rng.standard_normal((4, 500))))
    assert np.all(np.isin(r["s"], [-1.0, -2.0]))
    assert np.all(np.isfinite(r["smax"]))
    met = O.metrics(r["inputs"], r["trains"], False)
    assert met["rho"].max() <= 16 * EPS64
    # all-subnormal entries: large s, exact after backscale
    k = rng.integers(1, 2 ** 52, size=(4, 500)).astype(np.float64)
    sub = np.ldexp(k, -1074) * np.sign(rng.standard_normal((4, 500)))
    r = O.svd2(sub)
    assert np.all(r["s"] >= 1021 + 1022) and np.all(r["s"] <= 1021 + 1074)
    met = O.metrics(r["inputs"], r["trains"], False)
    assert met["rho"].max() <= 16 * EPS64
    # upper triangular complex
    A = scaled_law(2000, 16, True, special_frac=0)
    A[1] = 0
    r = O.svd2(A)
    met = O.metrics(r["inputs"], r["trains"], True)
    assert met["rho"].max() <= 16 * EPS64


# ---------------------------------------------------------------------------
# Theorem 1 and the bounds of its proof, on traced intermediates
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("cplx", [False, True])
def test_theorem1_invariants(cplx):
    A = np.concatenate([scaled_law(300, 17, cplx), random_bits(300, 18, cplx),
                        scaled_law(300, 19, cplx, special_frac=1.0)], axis=1)
    comps = O.split(A, np.float64)
    for k in range(A.shape[1]):
        a = np.array([c[k] for c in comps])
        t = O.trace(a, cplx)
        if t["s"] == np.finfo(np.float64).max:
            assert t["smax"] == 0 and t["smin"] == 0
            continue
        assert -2 <= t["s"] <= 1021 + 1074
        assert np.isfinite(t["smax"]) and t["smax"] >= t["smin"] >= 0
        assert np.sqrt(2) * (1 + 4 * EPS64) >= abs(t["tpsi"]) >= abs(t["tphi"]) >= 0
        assert 1 / np.sqrt(2) < t["cphi"] <= 1
        assert t["cpsi"] >= (1 / np.sqrt(3)) * (1 - 4 * EPS64)
        assert t["smax"] <= np.sqrt(3) * t["r11"] * (1 + 8 * EPS64)
        assert t["r11"] * (1 + 8 * EPS64) >= max(t["r12"], t["r22"])
        assert t["x"] ** 2 + t["y"] ** 2 <= 1 + 16 * EPS64
        assert t["r11"] < 2.0 ** (1021 + 2)
        assert t["t2"] <= 0 and np.signbit(t["t2"])
        assert t["n1"] >= t["n2"]


# ---------------------------------------------------------------------------
# REF and MIRROR readings agree (sigma_max to 4 ulp, sigma_min normwise)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("cplx", [False, True])
def test_ref_vs_mirror(cplx):
    A = np.concatenate([scaled_law(20000, 21, cplx), random_bits(20000, 22, cplx)], axis=1)
    a = O.svd2(A, policy="ref")
    b = O.svd2(A, policy="mirror")
    assert np.array_equal(a["s"], b["s"])
    nz = a["smax"] > 0
    rel = np.abs(a["smax"][nz] - b["smax"][nz]) / a["smax"][nz]
    assert rel.max() <= 4 * EPS64
    assert np.all(np.abs(a["smin"][nz] - b["smin"][nz]) <= 4 * EPS64 * a["smax"][nz])


# ---------------------------------------------------------------------------
# FP32 form and its FP64 rescue
# ---------------------------------------------------------------------------

def test_fp32_closed_form_exhaustive_real():
    M = int_matrices_real()
    r = O.svd2(M.astype(np.float32), dtype=np.float32)
    for j in range(M.shape[1]):
        if not M[:, j].any():
            continue
        xs, ns = exact_sigma(M[:, j])
        smax, smin = backscaled(r, j)
        assert abs(smax - xs) / xs <= 4 * EPS32
        assert abs(smin - ns) / xs <= 4 * EPS32


@pytest.mark.parametrize("mode", [1, 2, 3])
@pytest.mark.parametrize("cplx", [False, True])
def test_fp32_rescue_restores_relative_sigma_min(cplx, mode):
    """On near-singular FP32 inputs the plain FP32 sigma_min is only accurate
    normwise; with the FP64 rescue it must be accurate relatively, checked
    against the closed form in 60-digit arithmetic on the exact inputs."""
    rng = np.random.default_rng(23)
    n = 400
    # nearly rank-one: u v^T + tiny perturbation, formed in FP32
    dt = np.complex64 if cplx else np.float32
    u = rng.standard_normal((2, n)) + (1j * rng.standard_normal((2, n)) if cplx else 0)
    v = rng.standard_normal((2, n)) + (1j * rng.standard_normal((2, n)) if cplx else 0)
    A = np.stack([u[0] * np.conj(v[0]), u[1] * np.conj(v[0]), u[0] * np.conj(v[1]),
                  u[1] * np.conj(v[1])])
    A = (A + 3e-8 * rng.standard_normal((4, n))).astype(dt)
    plain = O.svd2(A, dtype=np.float32, rescue=False)
    resc = O.svd2(A, dtype=np.float32, rescue=mode)
    assert resc["flagged"].sum() > 0.5 * n
    worst_plain = worst_resc = 0.0
    for j in range(n):
        xs, ns = exact_sigma(A[:, j].astype(np.complex128) if cplx else A[:, j].astype(np.float64))
        if ns == 0 or not resc["flagged"][j]:
            continue
        worst_plain = max(worst_plain, float(abs(backscaled(plain, j)[1] - ns) / ns))
        worst_resc = max(worst_resc, float(abs(backscaled(resc, j)[1] - ns) / ns))
        assert float(abs(backscaled(resc, j)[0] - xs) / xs) <= 4 * EPS32
    assert worst_resc <= 8 * EPS32, worst_resc / EPS32
    assert worst_plain > 100 * EPS32  # the rescue is needed on these inputs
    met = O.metrics(resc["inputs"], resc["trains"], cplx)
    for key in ("rho", "delta", "eta"):
        assert met[key].max() <= 16 * EPS32, (key, met[key].max() / EPS32)


@pytest.mark.parametrize("mode", [1, 2, 3])
@pytest.mark.parametrize("cplx", [False, True])
def test_fp32_scaled_law_bounds(cplx, mode):
    A = scaled_law(20000, 24, cplx, dtype=np.float32)
    r = O.svd2(A, dtype=np.float32, rescue=mode)
    met = O.metrics(r["inputs"], r["trains"], cplx)
    for key in ("rho", "delta", "eta"):
        assert met[key].max() <= 16 * EPS32, (key, met[key].max() / EPS32)
    # against the FP64 oracle on the exact upcast: sigma_max relatively
    r64 = O.svd2(A.astype(np.complex128 if cplx else np.float64))
    s64 = np.array([float(backscaled(r64, j)[0]) for j in range(0, 20000, 10)])
    s32 = np.array([float(backscaled(r, j)[0]) for j in range(0, 20000, 10)])
    nz = s64 > 0
    assert np.all(np.abs(s32[nz] - s64[nz]) <= 4 * EPS32 * s64[nz])


@pytest.mark.parametrize("form", ["tangent", "sine"])
@pytest.mark.parametrize("cplx", [False, True])
def test_fp32_middle_rescue_against_fp64_tail(cplx, form):
    """The middle rescue (mode 3) runs the same FP64 triangular SVD as the
    FP64 tail (mode 1) and only assembles U, V in FP32 from its rounded
    angles: sigma' and s must be bitwise mode 1's, U and V within 4 eps32 of
    mode 1's (assembled in FP64, rounded once), and every unflagged lane
    bitwise the plain FP32 result.  Swapped or unrounded angles, a dropped
    phase or the FP32 r'_22 in place of the FP64 one break one of these."""
    from workloads import to_trains
    rng = np.random.default_rng(29)
    n = 4000
    u = rng.standard_normal((2, n)) + (1j * rng.standard_normal((2, n)) if cplx else 0)
    v = rng.standard_normal((2, n)) + (1j * rng.standard_normal((2, n)) if cplx else 0)
    near = np.stack([u[0] * np.conj(v[0]), u[1] * np.conj(v[0]), u[0] * np.conj(v[1]),
                     u[1] * np.conj(v[1])]) + 3e-8 * rng.standard_normal((4, n))
    dt = np.complex64 if cplx else np.float32
    A = np.concatenate([near.astype(dt), scaled_law(n, 30, cplx, dtype=np.float32)], axis=1)
    tr = to_trains(A, np.float32)
    o0, f0 = O.run_trains(tr, cplx, np.float32, rescue=0, form=form)
    o1, f1 = O.run_trains(tr, cplx, np.float32, rescue=1, form=form)
    o3, f3 = O.run_trains(tr, cplx, np.float32, rescue=3, form=form)
    assert np.array_equal(f1, f3) and f3.sum() > n // 2
    k = 16 if cplx else 8
    for i in range(k, k + 3):
        assert np.array_equal(o1[i], o3[i], equal_nan=True), i
    fl = f3.astype(bool)
    for i in range(k):
        d = np.abs(o3[i][fl].astype(np.float64) - o1[i][fl].astype(np.float64))
        assert d.max() <= 4 * EPS32, (i, d.max() / EPS32)
        assert np.array_equal(o3[i][~fl], o0[i][~fl]), i
    assert any(not np.array_equal(o3[i][fl], o1[i][fl]) for i in range(k))  # a different assembly


# ---------------------------------------------------------------------------
# The sine form of the assembly, eq. (31), against the tangent form, eq. (29)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("kind", ["d", "z", "s", "c"])
@pytest.mark.parametrize("law", ["scaled", "bits"])
def test_sine_form_is_the_tangent_form(kind, law):
    """Eqs. (29) and (31) are two formulas for the same U, written separately
    (the sines from sin = cos * tan, section 7): on the same lanes they agree
    within 4 eps entrywise (U's entries are at most 1 in magnitude); V, the
    scaled singular values and s are bitwise the same; and the sine form's
    rho, delta, eta (eqs. (33)-(35), binary128) stay within 16 eps.  A wrong
    sign, a swapped product or a dropped phase in either formula breaks the
    first check by orders of magnitude."""
    from workloads import to_trains
    cplx, dt = kind in "zc", (np.float64 if kind in "dz" else np.float32)
    n = 1 << 15
    if law == "bits":
        if dt == np.float32:
            pytest.skip("the random-bit law is the FP64 workload")
        A = random_bits(n, 811, cplx)
    else:
        A = scaled_law(n, 812, cplx, dtype=dt)
    tr = to_trains(A, dt)
    resc = dt == np.float32
    ot, ft = O.run_trains(tr, cplx, dt, rescue=resc)
    os_, fs = O.run_trains(tr, cplx, dt, rescue=resc, form="sine")
    assert np.array_equal(ft, fs)
    k = 16 if cplx else 8
    eps = float(np.finfo(dt).eps)
    for i in range(k // 2):
        d = np.abs(ot[i].astype(np.float64) - os_[i].astype(np.float64))
        assert np.nanmax(d) <= 4 * eps, (i, np.nanmax(d) / eps)
    for i in range(k // 2, k + 3):
        assert np.array_equal(ot[i], os_[i], equal_nan=True), i
    met = O.metrics(tr, os_, cplx)
    for key in ("rho", "delta", "eta"):
        assert np.nanmax(met[key]) <= 16 * eps, (key, np.nanmax(met[key]) / eps)


@pytest.mark.parametrize("dt", [np.float64, np.float32])
def test_subnormal_phase_keeps_u_unitary(dt):
    """A complex pivot whose modulus is subnormal after the scaling of eq. (2)
    (here a_21 = (-4 + i) 2^-1074 beside a_11 = 2^1021, which the scaling
    leaves unchanged): eq. (1) taken literally gives the "phase" (-1, 1/4) of
    modulus 1.03 and a U that is 2^-4 away from unitary; the phase is taken of
    an exactly rescaled z, so U is unitary to rounding (delta <= 16 eps) and
    the residual stays small.  The second lane is one found that way in the
    seeded +-m 2^e workload (r'_22 subnormal after the QR step)."""
    from workloads import to_trains
    tiny = np.ldexp(1.0, -1074 if dt == np.float64 else -149)
    big = np.ldexp(1.0, 1021 if dt == np.float64 else 125)
    lanes = [[big, (-4 + 1j) * tiny, 0.0, 0.0]]
    if dt == np.float64:
        h = [float.fromhex(x) for x in ("-0x1.8f3ff0bbc6878p-114", "0x1.b7b4128a87457p-115", "0x0.0p+0",
                                        "0x0.0p+0", "0x1.da9c4603b1d54p-561", "0x1.44b5677d98d6fp+972",
                                        "0x1.3f8a762830dd4p-36", "-0x1.cc6cffd77a71fp-496")]
        lanes.append([h[0] + 1j * h[1], h[2] + 1j * h[3], h[4] + 1j * h[5], h[6] + 1j * h[7]])
    A = np.array(lanes, dtype=np.complex128).T.astype(np.complex128 if dt == np.float64 else np.complex64)
    tr = to_trains(A, dt)
    eps = float(np.finfo(dt).eps)
    for form in ("tangent", "sine"):
        out, _ = O.run_trains(tr, True, dt, form=form)
        met = O.metrics(tr, out, True)
        assert np.max(met["delta"]) <= 16 * eps, (form, met["delta"] / eps)
        assert np.max(met["rho"]) <= 16 * eps, (form, met["rho"] / eps)


# ---------------------------------------------------------------------------
# FP32 rescue: which lanes are near-degenerate
# ---------------------------------------------------------------------------

def _flag_rule_cases(cplx):
    """Matrices whose singular values are exact in FP32 (diagonal and
    anti-diagonal, entries times 1, i, -1 or -i, magnitudes 2^e and 2^e b) with
    b = sigma_min / sigma_max placed on both sides of 2^-20 down to one FP32
    ulp, plus the zero matrix, exactly rank-one ones and well-conditioned ones.
    Returns the (4, n) matrices and the exact ratio b (Fraction) per lane."""
    two20 = Fraction(1, 1 << 20)
    ratios = [two20, Fraction(1), Fraction(1, 2), two20 * 2, Fraction(0)]
    for k in range(1, 24):
        ratios += [two20 * (1 - Fraction(1, 1 << k)), two20 * (1 + Fraction(1, 1 << k))]
    ratios.append(two20 * (1 - Fraction(1, 1 << 24)))  # 1 - 2^-24 is representable too
    phases = [1, 1j, -1, -1j] if cplx else [1, -1]
    cols, bs = [], []
    for e in (-100, -40, 0, 37, 120):  # both singular values stay in the normal range
        big = 2.0 ** e
        for b in ratios:
            small = float(b) * big
            assert Fraction(np.float32(small).item()) == b * Fraction(big)  # exact in FP32
            for i, (p1, p2) in enumerate(itertools.product(phases, repeat=2)):
                x, y = p1 * big, p2 * small
                shape = i % 4
                if shape == 0:
                    m = (x, 0, 0, y)      # diag(x, y)
                elif shape == 1:
                    m = (y, 0, 0, x)      # diag(y, x): the column pivot swaps
                elif shape == 2:
                    m = (0, x, y, 0)      # [[0, y], [x, 0]]
                else:
                    m = (0, y, x, 0)
                cols.append(m)
                bs.append(b)
    zero = (0, 0, 0, 0)
    cols.append(zero)
    bs.append(None)
    A = np.array(cols, dtype=np.complex64 if cplx else np.float32).T
    if not cplx:
        A = A.real.astype(np.float32)
    return A, bs


@pytest.mark.parametrize("mode", [1, 2, 3])
@pytest.mark.parametrize("cplx", [False, True])
def test_fp32_rescue_flags_exactly_below_2_to_minus_20(cplx, mode):
    """The precision form rescues a lane iff sigma_min / sigma_max < 2^-20
    (the near-degenerate rule of the FP32 form).  On matrices whose singular
    values are exact in FP32 the ratio is known exactly, so the flag must be
    set on every lane with ratio below 2^-20 (down to one ulp below) and on
    exactly rank-one lanes, and on no other lane: not at 2^-20 itself, not one
    ulp above, not on well-conditioned lanes and not on the zero matrix.  A
    wrong exponent, a <= for <, or a rule that flags every lane fails here.
    The same marks come back from the per-matrix trace."""
    from workloads import to_trains
    A, bs = _flag_rule_cases(cplx)
    tr = to_trains(A, np.float32)
    outs, flagged = O.run_trains(tr, cplx, np.float32, policy="mirror", rescue=mode)
    k = 16 if cplx else 8
    want = np.array([b is not None and b < Fraction(1, 1 << 20) for b in bs])
    got = flagged.astype(bool)
    assert np.array_equal(got, want), (np.nonzero(got != want)[0][:10], [bs[i] for i in np.nonzero(got != want)[0][:10]])
    # the singular values of these lanes are exact in FP32, rescued or not
    s = outs[k + 2].astype(np.int64)
    nz = np.array([b is not None for b in bs])
    smax = np.ldexp(outs[k].astype(np.float64), -s)
    smin = np.ldexp(outs[k + 1].astype(np.float64), -s)
    for i in np.nonzero(nz)[0]:
        assert Fraction(smin[i]) == bs[i] * Fraction(smax[i]), i
    # the per-matrix trace takes the same decision
    for i in list(range(0, len(bs), 37)) + [len(bs) - 1]:
        a = np.stack([t[i] for t in tr])
        assert bool(O.trace(a, cplx, np.float32, rescue=mode)["rescued"]) == want[i], i
