"""Pins of oracle/stability.py (Sec. 4): the stability functions against the
schemes and iterations they describe, run step by step on the scalar test
equation or on a Fourier mode."""

import cmath

import numpy as np
import pytest

from oracle import pint
from oracle.stability import imex_amp, mgrit_stability, settls_roots, stability_map


@pytest.mark.parametrize("xl,xn", [(0.3j, -0.05 + 0.4j), (2.5j, 0.1 - 0.2j), (0.0, 0.7j)])
def test_imex_amp_is_the_scheme(xl, xn):
    """CN half step, Heun step (keeping U*), CN half step on u' = (L + N) u."""
    def cn_half(u):
        return (1 + xl / 4) * u / (1 - xl / 4)
    u = cn_half(1.0 + 0j)
    ub = xn * u
    ubb = xn * (u + ub)
    u = cn_half(u + 0.5 * (ub + ubb))
    assert abs(u - imex_amp(xl, xn)) < 1e-15 * abs(u)


@pytest.mark.parametrize("xl,xn,ks", [(0.5j, -0.1 + 0.3j, 0.7), (3.0j, 0.05 + 0.2j, 2.0),
                                      (0.2j, -0.3 - 0.1j, 4.5)])
def test_settls_roots_are_the_scheme(xl, xn, ks):
    """Run SL-SI-SETTLS (eq. SL_SI_SETTLS) on u_j = a_n exp(i kappa x_j) with
    exact interpolation (a value at the departure point is the grid value
    times exp(-i ks)): the two-step recurrence for a_n, started from two
    seeds, is a combination of both roots, which a 2x2 fit recovers."""
    e = cmath.exp(-1j * ks)
    A1, A2 = settls_roots(xl, xn, ks)
    a = [1.0 + 0j, 0.3 - 0.8j]
    for n in range(1, 12):
        rhs = e * a[n] * (1 + xl / 2) + xn / 2 * ((2 * a[n] - a[n - 1]) * e + a[n])
        a.append(rhs / (1 - xl / 2))
    # a_n = c1 A1^n + c2 A2^n for every n
    c1, c2 = np.linalg.solve(np.array([[1, 1], [A1, A2]]), np.array(a[:2]))
    for n in range(len(a)):
        want = c1 * A1 ** n + c2 * A2 ** n
        assert abs(a[n] - want) <= 1e-12 * max(1.0, abs(want))


def test_settls_crank_nicolson_limit():
    """xi_N = 0, no shift: one root is 0, the other the CN factor."""
    xl = 0.8j
    A = sorted(settls_roots(xl, 0.0, 0.0), key=abs)
    assert abs(A[0]) < 1e-16
    assert abs(A[1] - (1 + xl / 2) / (1 - xl / 2)) < 1e-15


@pytest.mark.parametrize("nu", [0, 1, 2, 3])
def test_mgrit_stability_solves_recurrence(nu):
    """Brute-force iteration of u^k_n = R u^k_{n-1} + S u^{k-1}_{n-nu-1}."""
    F, R = (0.995 + 0.02j) ** 4, 0.98 + 0.06j
    S = F ** nu * (F - R)
    N = 14
    prev = [R ** n for n in range(N + 1)]
    for k in range(0, 8):
        if k > 0:
            cur = [1.0 + 0j]
            for n in range(1, N + 1):
                j = n - nu - 1
                cur.append(R * cur[n - 1] + (S * prev[j] if j >= 0 else 0.0))
            prev = cur
        for n in range(N + 1):
            assert abs(prev[n] - mgrit_stability(n, k, F, R, nu)) < 1e-14


def test_mgrit_stability_parareal_cases():
    """nu = 0 is the Parareal function (itself pinned against the Parareal
    iteration); k = 0 is the coarse propagator alone; k = n is the fine one
    (exact termination)."""
    F, R = 0.97 + 0.2j, 0.9 + 0.35j
    for n in range(0, 9):
        for k in range(0, n + 1):
            assert abs(mgrit_stability(n, k, F, R, 0) - pint.parareal_stability(n, k, R, F)) < 1e-14
        assert abs(mgrit_stability(n, 0, F, R, 0) - R ** n) < 1e-15
        assert abs(mgrit_stability(n, n, F, R, 0) - F ** n) < 1e-13


def test_stability_map_scheme_imex_on_imaginary_axis():
    """For imaginary xi_L the CN factor has modulus 1, so |A_IMEX| is the
    Heun factor |1 + xi_N + xi_N^2/2| (1 at xi_N = 0, above 1 on the
    imaginary axis)."""
    m = stability_map("scheme", "imex", 5.0j, [0.0], [0.0, 0.5])
    assert abs(m[0][0] - 1.0) < 1e-15
    assert abs(m[1][0] - abs(1 + 0.5j + (0.5j) ** 2 / 2)) < 1e-15
