"""Pins of the oracle's Parareal and MGRIT drivers (paper Sec. 3 and 4.2)."""

import numpy as np
import pytest

from oracle import pint
from oracle.norms import rel_err
from oracle.swe import Model
from paper_2306_09497_amd import workloads


def imex_amp(xl, xn):
    """Scalar IMEX amplification: CN half steps around a Heun step."""
    ai = (4 + xl) / (4 - xl)
    return ai * (1 + xn + 0.5 * xn * xn) * ai


@pytest.mark.parametrize("k", [0, 1, 3, 7])
def test_parareal_stability_function(k):
    """P13: on u' = (lam_L + lam_N) u, the Parareal iterate equals
    sum_{i<=k} C(n,i) (F-R)^i R^(n-i) u0 (Sec. 4.2, eq. recurrence_parareal)."""
    lamL, lamN = 2.5e-3j, -1e-5 + 4e-5j
    dtf, nf, m = 60.0, 30, 10
    dtc, nc = dtf * m, 3
    F = imex_amp(lamL * dtf, lamN * dtf) ** nf
    R = imex_amp(lamL * dtc, lamN * dtc) ** nc
    N = 12
    u0 = 1.0 + 0.5j
    U, _ = pint.parareal(u0, N, lambda u: F * u, lambda u: R * u, k)
    for n in range(N + 1):
        want = pint.parareal_stability(n, k, R, F) * u0
        assert abs(U[n] - want) <= 1e-13 * abs(want) + 1e-15


def test_parareal_finite_termination_scalar():
    """P14: after N iterations Parareal reproduces the serial fine solution."""
    F, R = 0.99 + 0.05j, 0.97 + 0.1j
    U, _ = pint.parareal(1.0 + 0j, 9, lambda u: F * u, lambda u: R * u, 9)
    ser = pint.serial(1.0 + 0j, 9, lambda u: F * u)
    for a, b in zip(U, ser):
        assert abs(a - b) < 1e-15


def test_mgrit_recurrence_scalar():
    """Two-level MGRIT F(CF)^nu on the scalar equation follows the paper's
    overlapping-Parareal relation (eq. parareal_FCF_nrelax):
    u^k_n = G u^k_{n-1} + F^(nu+1) u^{k-1}_{n-nu-1} - G F^nu u^{k-1}_{n-nu-1},
    where the C-relaxation at the first nu C-points starts from u_0."""
    f, g, m = 0.995 + 0.02j, 0.98 + 0.06j, 4
    F = f ** m
    N1 = 10
    for nu in (0, 1, 2):
        prev = [g ** n for n in range(N1 + 1)]          # iteration 0
        for k in range(1, 5):
            C, _ = pint.mgrit2(1.0 + 0j, N1, m, lambda u: f * u, lambda u: g * u, nu, k)
            cur = [1.0 + 0j]
            for n in range(1, N1 + 1):
                j = n - nu - 1
                if j >= 0:
                    src, p = prev[j], nu
                else:                       # relaxation chain starts at u_0
                    src, p = 1.0 + 0j, n - 1
                cur.append(g * cur[n - 1] + F ** (p + 1) * src - g * F ** p * src)
            for a, b in zip(C, cur):
                assert abs(a - b) < 1e-14
            prev = cur


def test_mgrit_nu0_is_parareal_scalar():
    """P15 (scalar): MGRIT with (levels, nu) = (2, 0) is Parareal with
    F = Phi_0^m and G = Phi_1, bitwise."""
    f, g, m = 0.999 + 0.01j, 0.99 + 0.04j, 5
    for k in range(0, 6):
        C, _ = pint.mgrit2(1.0 + 0j, 8, m, lambda u: f * u, lambda u: g * u, 0, k)
        P, _ = pint.parareal(1.0 + 0j, 8, lambda u: (((( f * u) * f) * f) * f) * f,
                             lambda u: g * u, k)
        assert all(a == b for a, b in zip(C, P))


@pytest.fixture(scope="module")
def c1_small():
    """A shortened C1 problem: T21, 4 slices of 20 min, fine 60 s, coarse 600 s."""
    md = Model(21, 64, 32, phibar=2.94e4)
    U0 = workloads.solid_body(21, noise=1e-6, seed=0)
    fine = lambda u: md.propagate(u, 60.0, 20)
    coarse = lambda u: md.propagate(u, 600.0, 2)
    return md, U0, fine, coarse


def test_parareal_exact_swe(c1_small):
    """P14: Parareal with k = N reproduces the serial fine states (bitwise in
    this deterministic oracle)."""
    md, U0, fine, coarse = c1_small
    N = 4
    U, _ = pint.parareal(U0, N, fine, coarse, N)
    ser = pint.serial(U0, N, fine)
    for a, b in zip(U, ser):
        assert np.array_equal(a, b)


def test_mgrit_swe(c1_small):
    """P15/P16 on the SWE: MGRIT(2,0) equals Parareal bitwise (fine = 20 steps
    of Phi_0), and MGRIT FCF is exact after ceil(N_1/2) iterations."""
    md, U0, fine, coarse = c1_small
    phi0 = lambda u: md.propagate(u, 60.0, 1)
    for k in (1, 2):
        C, _ = pint.mgrit2(U0, 4, 20, phi0, coarse, 0, k)
        P, _ = pint.parareal(U0, 4, fine, coarse, k)
        for a, b in zip(C, P):
            assert np.array_equal(a, b)
    C, _ = pint.mgrit2(U0, 4, 20, phi0, coarse, 1, 2)
    ser = pint.serial(U0, 4, fine)
    for a, b in zip(C, ser):
        assert np.max(rel_err(a, b, 21)) < 1e-13
    # and not yet exact after one FCF iteration
    C1, _ = pint.mgrit2(U0, 4, 20, phi0, coarse, 1, 1)
    assert np.max(rel_err(C1[4], ser[4], 21)) > 1e-9


def _logistic(h):
    """One explicit Euler step of u' = u (1 - u): a nonlinear scalar stand-in
    for a propagator (the coarse levels take longer steps)."""
    return lambda u: u + h * (u * (1.0 - u))


@pytest.mark.parametrize("nu", [0, 1])
def test_mgrit3_single_level2_interval_is_two_level(nu):
    """Three-level MGRIT whose level 1 holds a single level-2 interval solves
    the level-1 problem exactly by relaxation: bitwise the two-level iterate."""
    h, m, N1 = 0.05, 3, 4
    phi0, phi1, phi2 = _logistic(h), _logistic(m * h), _logistic(m * N1 * h)
    for k in (1, 2, 3):
        C3, _ = pint.mgrit3(0.1, N1, m, phi0, phi1, phi2, nu, k, m1=N1)
        C2, _ = pint.mgrit2(0.1, N1, m, phi0, phi1, nu, k)
        assert all(a == b for a, b in zip(C3, C2)), (k, C3, C2)


@pytest.mark.parametrize("nu", [0, 1])
def test_mgrit3_exact_level2_linear_is_two_level(nu):
    """On a linear problem with Phi_2 = Phi_1^m1 the level-2 correction of the
    FAS level-1 problem is exact, so one cycle on levels (1, 2) reproduces the
    two-level iterate (up to rounding): pins the signs and indices of the
    level-1 and level-2 right-hand sides."""
    f, g, m, m1, N1 = 0.995 + 0.02j, 0.98 + 0.06j, 3, 2, 8
    phi0 = lambda u: f * u
    phi1 = lambda u: g * u
    phi2 = lambda u: g * (g * u)
    for k in (1, 2, 3):
        C3, _ = pint.mgrit3(1.0 + 0j, N1, m, phi0, phi1, phi2, nu, k, m1=m1)
        C2, _ = pint.mgrit2(1.0 + 0j, N1, m, phi0, phi1, nu, k)
        for a, b in zip(C3, C2):
            assert abs(a - b) < 1e-14, (k, a, b)
    # an inexact Phi_2 gives a different iterate (the level-2 solve matters)
    C3x, _ = pint.mgrit3(1.0 + 0j, N1, m, phi0, phi1, lambda u: 0.96 * u, nu, 1, m1=m1)
    C2x, _ = pint.mgrit2(1.0 + 0j, N1, m, phi0, phi1, nu, 1)
    assert max(abs(a - b) for a, b in zip(C3x, C2x)) > 1e-6


@pytest.mark.parametrize("nu,cycles", [(0, 1), (1, 1), (1, 2)])
def test_mgrit3_finite_termination(nu, cycles):
    """An exact prefix stays bitwise exact through both levels' corrections,
    so three-level MGRIT reproduces the serial fine C-points after
    ceil(N_1/(nu+1)) iterations, and not one iteration earlier."""
    h, m, m1, N1 = 0.05, 2, 2, 8
    phi0, phi1, phi2 = _logistic(h), _logistic(0.9 * m * h), _logistic(0.8 * m * m1 * h)
    ser = pint.serial(0.1, N1, lambda u: phi0(phi0(u)))
    kmax = -(-N1 // (nu + 1))
    C, _ = pint.mgrit3(0.1, N1, m, phi0, phi1, phi2, nu, kmax, m1=m1, cycles=cycles)
    assert all(a == b for a, b in zip(C, ser))
    Cm, _ = pint.mgrit3(0.1, N1, m, phi0, phi1, phi2, nu, kmax - 1, m1=m1, cycles=cycles)
    assert abs(Cm[N1] - ser[N1]) > 0


def test_mgrit3_swe_single_level2_interval(c1_small):
    """The same identity on the SWE: one level-2 interval reproduces the
    two-level MGRIT iterate bitwise."""
    md, U0, fine, coarse = c1_small
    phi0 = lambda u: md.propagate(u, 60.0, 1)
    phi2 = lambda u: md.propagate(u, 2400.0, 1)
    C3, _ = pint.mgrit3(U0, 4, 20, phi0, coarse, phi2, 1, 1, m1=4)
    C2, _ = pint.mgrit2(U0, 4, 20, phi0, coarse, 1, 1)
    for a, b in zip(C3, C2):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("nu,cycles", [(0, 1), (1, 1), (2, 1), (1, 2)])
def test_mgrit3_level1_cycle_matches_matrix_form(nu, cycles):
    """One two-level cycle on levels (1, 2) of a linear level-1 problem
    w_i = g w_{i-1} + c_i, written independently as block relaxation and
    coarse-grid correction on the bidiagonal system A w = b: F-relaxation
    solves the F rows given the C values, C-relaxation the C rows given the F
    values, and the level-2 correction adds e = A_2^{-1} r on the C points
    (A_2 bidiagonal with the inexact level-2 factor g2), with FAS and
    injection; then F-relaxation."""
    rng = np.random.default_rng(5)
    N1, m1 = 12, 3
    N2 = N1 // m1
    g, g2 = 0.97 + 0.05j, 0.90 + 0.12j
    c = rng.standard_normal(N1 + 1) + 1j * rng.standard_normal(N1 + 1)
    W0 = rng.standard_normal(N1 + 1) + 1j * rng.standard_normal(N1 + 1)

    got = pint._two_level_on_level1(list(W0), lambda i, w: g * w + c[i],
                                    lambda u: g2 * u, m1, nu, cycles)

    # matrix form: unknowns w_1..w_N1, A w = b
    A = np.eye(N1, dtype=complex) - g * np.eye(N1, k=-1)
    b = c[1:].copy()
    b[0] += g * W0[0]
    Cset = [m1 * j - 1 for j in range(1, N2 + 1)]          # rows of w_{m1 j}
    Fset = [r for r in range(N1) if r not in Cset]
    w = W0[1:].copy()

    def relax(w, rows):
        w = w.copy()
        other = [r for r in range(N1) if r not in rows]
        rhs = b[rows] - A[np.ix_(rows, other)] @ w[other]
        w[rows] = np.linalg.solve(A[np.ix_(rows, rows)], rhs)
        return w

    A2 = np.eye(N2, dtype=complex) - g2 * np.eye(N2, k=-1)
    for _ in range(cycles):
        w = relax(w, Fset)
        for _ in range(nu):
            w = relax(w, Cset)
            w = relax(w, Fset)
        r = b - A @ w
        w[Cset] += np.linalg.solve(A2, r[Cset])
        w = relax(w, Fset)
    assert np.allclose(np.array(got[1:]), w, rtol=0, atol=1e-12)
    assert got[0] == W0[0]


def test_spatial_coarsening_parareal(c1_small):
    """Coarse level at truncation Mc < M (reading: coarse propagator =
    pad(coarse model step(truncate(u)))): the difference-first update leaves
    every coefficient above Mc equal to the fine propagator's bitwise, and
    k = N still reproduces serial fine."""
    from oracle import sht
    md, U0, fine, _ = c1_small
    Mc = 10
    mdc = Model(Mc, 32, 16, phibar=2.94e4)
    coarse = lambda u: sht.pad(mdc.propagate(sht.truncate(u, 21, Mc), 600.0, 2), Mc, 21)
    U1, _ = pint.parareal(U0, 4, fine, coarse, 1)
    hi = np.array([n > Mc for m in range(22) for n in range(m, 22)])
    for n in range(4):
        assert np.array_equal(U1[n + 1][:, hi], fine(U0 if n == 0 else pint.serial(
            U0, 4, coarse)[n])[:, hi])
    U, _ = pint.parareal(U0, 4, fine, coarse, 4)
    ser = pint.serial(U0, 4, fine)
    for a, b in zip(U, ser):
        assert np.array_equal(a, b)


def _ab2_coarse(lam, h, steps):
    """A two-step coarse scheme on u' = lam u (second-order Adams-Bashforth;
    without a previous state the first step takes u_{n-1} = u_n, i.e. Euler):
    (u, p) -> (u after `steps` steps, the state one step before it)."""
    def G(u, p):
        prev = u if p is None else p
        for _ in range(steps):
            u, prev = u + h * lam * (1.5 * u - 0.5 * prev), u
        return u, prev
    return G


def test_parareal_carry_first_sweep_is_the_serial_two_step_run():
    """Iterate 0 of the carried sweep equals the uninterrupted two-step run
    over the whole horizon, bitwise (one-step only at its very first step)."""
    lam, h, c, N = -0.3 + 1.1j, 0.05, 3, 6
    G = _ab2_coarse(lam, h, c)
    U, _ = pint.parareal_carry(1.0 + 0.5j, N, lambda u: u, G, 0)
    u, prev = 1.0 + 0.5j, None
    for n in range(N):
        u, prev = G(u, prev)
        assert U[n + 1] == u
    # the same run restarted one-step at every slice differs
    R, _ = pint.parareal(1.0 + 0.5j, N, lambda u: u, lambda u: G(u, None)[0], 0)
    assert R[2] != U[2]


def test_parareal_carry_without_history_is_parareal():
    """A coarse scheme that ignores its carried state gives Parareal's
    iterates bitwise; with k = N the carried sweep ends at the serial fine
    solution bitwise (finite termination, Sec. 3.1)."""
    lam, N = 0.2 - 0.9j, 5
    F = np.exp(lam * 0.5)
    R = 1.0 + lam * 0.5

    def fine(u):
        return F * u

    for k in range(N + 1):
        A, _ = pint.parareal_carry(1.0 + 0j, N, fine, lambda u, p: (R * u, u), k)
        B, _ = pint.parareal(1.0 + 0j, N, fine, lambda u: R * u, k)
        assert A == B
    G = _ab2_coarse(lam, 0.1, 5)
    U, _ = pint.parareal_carry(1.0 + 0j, N, fine, G, N)
    assert U == pint.serial(1.0 + 0j, N, fine)


def _ab2_step(lam, h):
    """One step of the two-step scheme of _ab2_coarse: (u, p) -> u'."""
    def g(u, p):
        prev = u if p is None else p
        return u + h * lam * (1.5 * u - 0.5 * prev)
    return g


def test_mgrit2_sl_without_history_is_mgrit2():
    """A coarse step that ignores its history gives the two-level MGRIT
    iterates bitwise (nu = 0, 1)."""
    lam, N, m = -0.4 + 0.8j, 6, 3
    phi0 = lambda u: u * np.exp(lam * 0.1)
    g1 = lambda u: u * (1.0 + lam * 0.3)
    for nu in (0, 1):
        a, _ = pint.mgrit2(1.0 + 0.2j, N, m, phi0, g1, nu, 3)
        b, _ = pint.mgrit2_sl(1.0 + 0.2j, N, m, phi0, lambda u, p: g1(u), nu, 3)
        assert a == b


def test_mgrit2_sl_initial_sweep_and_nu0_carried_parareal():
    """Iterate 0 is the uninterrupted two-step run; with nu = 0 the
    iteration is Parareal whose coarse runs carry the previous slice state
    (one step per slice), bitwise."""
    lam, N, m, h = 0.3 - 1.2j, 6, 4, 0.05
    g = _ab2_step(lam, h)
    phi0 = lambda u: u * np.exp(lam * h / m)
    C, _ = pint.mgrit2_sl(1.0 + 0.5j, N, m, phi0, g, 0, 0)
    u, prev = 1.0 + 0.5j, None
    for n in range(N):
        u, prev = g(u, prev), u
        assert C[n + 1] == u
    G = lambda u, p: (g(u, p), u)
    for k in range(1, 4):
        a, _ = pint.mgrit2_sl(1.0 + 0.5j, N, m, phi0, g, 0, k)
        b, _ = pint.parareal_carry(1.0 + 0.5j, N, lambda u: pint.serial(u, m, phi0)[-1], G, k)
        assert a == b


@pytest.mark.parametrize("nu", [0, 1, 2])
def test_mgrit2_sl_finite_termination(nu):
    """With the history taken from the same coarse sequence, a converged
    prefix stays bitwise exact: after ceil(N/(nu+1)) iterations every
    C-point is the serial fine solution bitwise (Sec. 3.2.3)."""
    lam, N, m, h = -0.2 + 0.9j, 7, 3, 0.2
    g = _ab2_step(lam, h)
    phi0 = lambda u: u * np.exp(lam * h / m)
    ref = pint.serial(1.0 - 0.3j, N * m, phi0)
    k = -(-N // (nu + 1))
    C, _ = pint.mgrit2_sl(1.0 - 0.3j, N, m, phi0, g, nu, k)
    assert C == [ref[i * m] for i in range(N + 1)]
    C1, _ = pint.mgrit2_sl(1.0 - 0.3j, N, m, phi0, g, nu, 1)
    assert C1[N] != ref[N * m]                  # not converged after one iteration
