"""Pins of the oracle's phase outputs (R and the unitary factors U_+, V_+ of
the URV factorization, section 2.2, eqs. (9) and (11)) against what the
mathematics fixes (no GPU):

* A^ = 2^s A = U_+ R V_+^* in exact rational arithmetic, within a few eps;
* U_+ and V_+ unitary, R upper triangular, real, with r11 >= max(r12, r22) >= 0;
* the singular values of R, in 60-digit arithmetic, are those of A^ (so the
  oracle's sigma' of the full pipeline within its bounds);
* hand cases whose factors follow from the definitions by inspection
  (diagonal with signs, the column swap P_c, the row swap P_r, a phase).
"""
from fractions import Fraction

import mpmath as mp
import numpy as np
import pytest

import oracle.oracle as O
from workloads import SEED_BASE, random_bits, scaled_law, uniform_real

EPS = {np.float64: 2.0 ** -53, np.float32: 2.0 ** -24}
mp.mp.dps = 60


def _cx(z):
    z = complex(z)
    return (Fraction(z.real), Fraction(z.imag))


def _mul(a, b):
    return (a[0] * b[0] - a[1] * b[1], a[0] * b[1] + a[1] * b[0])


def _add(a, b):
    return (a[0] + b[0], a[1] + b[1])


def _conj(a):
    return (a[0], -a[1])


def _abs2(a):
    return a[0] * a[0] + a[1] * a[1]


def _mat(X, k):
    """(4, n) element order 11, 21, 12, 22 -> 2x2 of exact complex pairs"""
    return [[_cx(X[0, k]), _cx(X[2, k])], [_cx(X[1, k]), _cx(X[3, k])]]


def _prod(X, Y):
    return [[_add(_mul(X[i][0], Y[0][j]), _mul(X[i][1], Y[1][j])) for j in range(2)] for i in range(2)]


def _adj(X):
    return [[_conj(X[j][i]) for j in range(2)] for i in range(2)]


def _fro2(X):
    return sum(_abs2(X[i][j]) for i in range(2) for j in range(2))


def _diff(X, Y):
    return [[(X[i][j][0] - Y[i][j][0], X[i][j][1] - Y[i][j][1]) for j in range(2)] for i in range(2)]


def _eye():
    one, zero = (Fraction(1), Fraction(0)), (Fraction(0), Fraction(0))
    return [[one, zero], [zero, one]]


def _inputs(kind, n, seed):
    cplx = kind in ("z", "c")
    dt = np.float64 if kind in ("d", "z") else np.float32
    emax = 40 if dt == np.float64 else 20
    A = scaled_law(n, seed, cplx, dtype=dt, emin=-emax, emax=emax)
    B = uniform_real(n, seed + 1, dtype=dt)
    if cplx:
        B = (B + 1j * uniform_real(n, seed + 2, dtype=dt)).astype(np.complex128 if dt == np.float64 else np.complex64)
    C = random_bits(n // 4, seed + 3, cplx, dtype=dt)
    return np.concatenate([A, B, C], axis=1), dt, cplx


@pytest.mark.parametrize("kind", ["d", "z", "s", "c"])
def test_urv_reconstructs_the_scaled_input(kind):
    """A^ = U_+ R V_+^* (eq. (11)) with A^ = 2^s A formed exactly, U_+ and V_+
    unitary, R real upper triangular with r11 >= max(r12, r22) >= 0."""
    A, dt, cplx = _inputs(kind, 160, SEED_BASE + 700 + ord(kind))
    f = O.urv(A, dtype=dt)
    r = O.svd2(A, dtype=dt)
    eps = EPS[dt]
    worst_res = worst_u = 0.0
    for k in range(A.shape[1]):
        s = r["s"][k]
        if s == np.finfo(dt).max:  # zero matrix
            continue
        Ah = [[(x[0] * Fraction(2) ** int(s), x[1] * Fraction(2) ** int(s)) for x in row] for row in _mat(A, k)]
        r11, r12, r22 = (Fraction(float(f[x][k])) for x in ("r11", "r12", "r22"))
        assert r11 >= r12 >= 0 and r11 >= r22 >= 0, (kind, k)
        zero = (Fraction(0), Fraction(0))
        R = [[(r11, Fraction(0)), (r12, Fraction(0))], [zero, (r22, Fraction(0))]]
        Up, Vp = _mat(f["Up"], k), _mat(f["Vp"], k)
        res = _fro2(_diff(Ah, _prod(_prod(Up, R), _adj(Vp)))) / _fro2(Ah)
        uu = max(_fro2(_diff(_prod(_adj(Up), Up), _eye())), _fro2(_diff(_prod(_adj(Vp), Vp), _eye())))
        worst_res = max(worst_res, float(res) ** 0.5 / eps)
        worst_u = max(worst_u, float(uu) ** 0.5 / eps)
    assert worst_res <= 8, (kind, worst_res)
    assert worst_u <= 16, (kind, worst_u)


@pytest.mark.parametrize("kind", ["d", "z", "s", "c"])
def test_sigma_of_r_is_sigma_prime(kind):
    """The exact singular values of R (60 digits) agree with the full
    pipeline's sigma' (the triangular SVD of section 2.3 of the same R):
    sigma'_max within 4 eps, sigma'_min within 8 eps relative to itself."""
    A, dt, cplx = _inputs(kind, 120, SEED_BASE + 760 + ord(kind))
    f = O.urv(A, dtype=dt)
    r = O.svd2(A, dtype=dt)
    eps = EPS[dt]
    for k in range(A.shape[1]):
        r11, r12, r22 = (mp.mpf(float(f[x][k])) for x in ("r11", "r12", "r22"))
        F, D = r11 ** 2 + r12 ** 2 + r22 ** 2, r11 * r22
        p, q = mp.sqrt(F + 2 * D), mp.sqrt(max(F - 2 * D, mp.mpf(0)))
        smax = (p + q) / 2
        smin = 2 * D / (p + q) if D != 0 else mp.mpf(0)
        gmax, gmin = mp.mpf(float(r["smax"][k])), mp.mpf(float(r["smin"][k]))
        if smax == 0:
            assert gmax == 0 and gmin == 0
            continue
        assert abs(gmax - smax) <= 4 * eps * smax, (kind, k)
        assert abs(gmin - smin) <= 8 * eps * smin + 1e-300, (kind, k)


def _one(A, dt):
    f = O.urv(A, dtype=dt)
    s = int(O.svd2(A, dtype=dt)["s"][0])
    r11, r12, r22 = (float(np.ldexp(np.float64(f[x][0]), -s)) for x in ("r11", "r12", "r22"))
    return r11, r12, r22, [complex(x) for x in f["Up"][:, 0]], [complex(x) for x in f["Vp"][:, 0]]


@pytest.mark.parametrize("dt", [np.float64, np.float32])
def test_hand_cases(dt):
    """Factors that follow from the definitions by inspection (element order
    11, 21, 12, 22); R is compared with the scaling 2^s of eq. (2) divided
    out."""
    # diag(3, -2): no swap, D = I, Q_alpha = I, D~ = I, D^ = diag(1, -1)
    assert _one(np.array([[3.0], [0.0], [0.0], [-2.0]]), dt) == (3.0, 0.0, 2.0, [1, 0, 0, -1], [1, 0, 0, 1])
    # diag(-1, 4): P_c swaps the columns (column 2 is longer), then P_r the
    # rows (|a'_11| = 0 < |a'_21| = 4): A'' = [[4, 0], [0, -1]], D = I,
    # D^ = diag(1, -1), so U_+ = P_r D^ = [[0, -1], [1, 0]] and V_+ = P_c
    assert _one(np.array([[-1.0], [0.0], [0.0], [4.0]]), dt) == (4.0, 0.0, 1.0, [0, 1, -1, 0], [0, 1, 1, 0])
    # [[0, 0], [-2, 0]]: the row swap only, D = diag(-1, 1): U_+ = P_r D
    assert _one(np.array([[0.0], [-2.0], [0.0], [0.0]]), dt) == (2.0, 0.0, 0.0, [0, -1, 1, 0], [1, 0, 0, 1])
    # [[2, 1], [0, 1]] (already R): U_+ = V_+ = I
    assert _one(np.array([[2.0], [0.0], [1.0], [1.0]]), dt) == (2.0, 1.0, 1.0, [1, 0, 0, 1], [1, 0, 0, 1])
    cdt = np.complex128 if dt == np.float64 else np.complex64
    # [[i, 0], [0, 1]]: D = diag(i, 1), everything else the identity
    assert _one(np.array([[1j], [0], [0], [1]], dtype=cdt), dt) == (1.0, 0.0, 1.0, [1j, 0, 0, 1], [1, 0, 0, 1])
    # [[2, i], [0, 1]]: r'_12 = i, so D~ = diag(1, -i); r'_22 = 1 conj(i) =
    # -i, so D^ = diag(1, -i); R = [[2, 1], [0, 1]]
    assert _one(np.array([[2], [0], [1j], [1]], dtype=cdt), dt) == (2.0, 1.0, 1.0, [1, 0, 0, -1j], [1, 0, 0, -1j])
