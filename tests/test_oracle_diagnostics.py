"""Pins of oracle/diagnostics.py (kinetic-energy spectrum, spectral max-norm
errors, physical-space L2 errors) against closed forms, Gauss quadrature of
the synthesised wind and hand-worked small cases."""

import numpy as np
import pytest

from oracle.diagnostics import grid_l2_errors, ke_spectrum, spectral_errors
from oracle.sht import Grid, idx, ncoef

A = 6.37122e6


def test_ke_spectrum_solid_body_closed_form():
    """Solid-body rotation u = u0 cos(lat), v = 0: xi = 2 u0 mu / a is
    (2 u0 / (a sqrt 3)) Y_{0,1}, and the area mean of u^2 is 2/3 u0^2, so the
    whole spectrum is E(1) = u0^2 / 6."""
    M, u0 = 12, 38.6
    U = np.zeros((3, ncoef(M)), dtype=complex)
    U[0, 0] = 2.94e4
    U[1, idx(M, 0, 1)] = 2.0 * u0 / (A * np.sqrt(3.0))
    E = ke_spectrum(U, M, A)
    assert E[1] == pytest.approx(u0 * u0 / 6.0, rel=1e-14)
    assert np.all(E[2:] == 0.0) and E[0] == 0.0


@pytest.mark.parametrize("m,n", [(0, 3), (2, 3), (5, 7)])
def test_ke_spectrum_single_harmonic(m, n):
    """One vorticity and one divergence harmonic at (m, n): the conjugate
    partner at -m doubles the energy of m > 0."""
    M = 9
    U = np.zeros((3, ncoef(M)), dtype=complex)
    c, d = 1e-5 * (0.3 + (0.4j if m else 0.0)), 2e-6 * (1.0 - (0.7j if m else 0.0))
    U[1, idx(M, m, n)] = c
    U[2, idx(M, m, n)] = d
    E = ke_spectrum(U, M, A)
    mult = 1.0 if m == 0 else 2.0
    want = 0.25 * A * A / (n * (n + 1.0)) * mult * (abs(c) ** 2 + abs(d) ** 2)
    assert E[n] == pytest.approx(want, rel=1e-14)
    assert np.count_nonzero(E) == 1


def test_ke_spectrum_sum_is_quarter_mean_square_wind():
    """Sum over n of E(n) = 1/4 of the area mean of u^2 + v^2, the mean taken
    by Gauss quadrature of the wind synthesised on the grid (exact for this
    band-limited field)."""
    M, nlon, nlat = 10, 32, 16
    g = Grid(M, nlon, nlat, A)
    rng = np.random.default_rng(11)
    U = np.zeros((3, ncoef(M)), dtype=complex)
    for f in (1, 2):
        U[f] = 1e-5 * (rng.standard_normal(ncoef(M)) + 1j * rng.standard_normal(ncoef(M)))
        for n in range(M + 1):                 # m = 0 coefficients of a real field
            U[f, idx(M, 0, n)] = U[f, idx(M, 0, n)].real
        U[f, 0] = 0.0                          # no mean vorticity / divergence
    Uf, Vf = g.uv_fourier_from_psichi(U[1] * g.invlap, U[2] * g.invlap)
    c2 = g.coslat2[:, None]
    ug = g.fourier_to_grid(Uf) ** 2 / c2
    vg = g.fourier_to_grid(Vf) ** 2 / c2
    mean = 0.5 * np.sum(g.w * np.mean(ug + vg, axis=1))
    assert np.sum(ke_spectrum(U, M, A)) == pytest.approx(0.25 * mean, rel=1e-12)


def test_spectral_errors_hand_worked():
    """M = 2, packed order (0,0) (0,1) (0,2) (1,1) (1,2) (2,2)."""
    M, phibar = 2, 3.0e5
    ref = np.zeros((3, 6), dtype=complex)
    ref[0] = [phibar + 2.0, 1.0, -6.0, 3.0j, 0.0, 1.0]
    ref[1] = [0.0, 1.0, 2.0, 3.0j, 0.0, 4.0]
    ref[2] = [0.0, 0.0, 0.0, 0.0, 0.0, 0.0]
    x = ref.copy()
    x[0, 0] += 0.5                 # Phi' mean 2 -> 2.5
    x[0, 4] += 1.0                 # (1, 2)
    x[1, 1] += 0.25                # (0, 1)
    x[1, 4] += 0.5                 # (1, 2)
    E = spectral_errors(x, ref, M, phibar)
    # Phi': R=0 {(0,0)}: 0.5/2; R=1 adds (0,1),(1,1): 0.5/3; R=2: 1/6
    assert np.allclose(E[0], [0.25, 0.5 / 3.0, 1.0 / 6.0], rtol=1e-15, atol=0)
    # xi: R=0 reference and difference both 0; R=1: 0.25/3; R=2: 0.5/4
    assert np.allclose(E[1], [0.0, 0.25 / 3.0, 0.125], rtol=1e-15, atol=0)
    assert np.all(E[2] == 0.0)
    x[2, 3] = 1e-9                 # difference on a zero reference
    E = spectral_errors(x, ref, M, phibar)
    assert E[2, 0] == 0.0 and np.isinf(E[2, 1]) and np.isinf(E[2, 2])


def test_grid_l2_errors_closed_form():
    """Reference Phi' = b Y_{0,1} = b sqrt(3) mu, difference c Y_{1,1} with
    Y_{1,1} + conj = 2 Re(c e^{i lambda}) sqrt(3/2) sqrt(1 - mu^2), evaluated
    directly on the Gauss nodes; xi the same with the roles of (0,1) and
    (1,1) swapped."""
    M, nlon, nlat, phibar = 4, 16, 8, 2.9e5
    g = Grid(M, nlon, nlat, A)
    mu = np.polynomial.legendre.leggauss(nlat)[0][::-1]
    lam = 2.0 * np.pi * np.arange(nlon) / nlon
    b, c = 3.0, 0.2 - 0.1j
    ref = np.zeros((3, ncoef(M)), dtype=complex)
    ref[0, 0] = phibar
    ref[0, idx(M, 0, 1)] = b
    ref[1, idx(M, 1, 1)] = c
    ref[2, idx(M, 0, 2)] = 1.0
    x = ref.copy()
    x[0, idx(M, 1, 1)] += c
    x[1, idx(M, 0, 1)] += b
    y01 = np.sqrt(3.0) * mu[:, None] * np.ones(nlon)
    y11 = 2.0 * np.real(c * np.exp(1j * lam))[None, :] * np.sqrt(1.5) * np.sqrt(1 - mu ** 2)[:, None]
    e_phi = np.sqrt(np.sum(y11 ** 2) / np.sum((b * y01) ** 2))
    E = grid_l2_errors(x, ref, g, phibar)
    assert E[0] == pytest.approx(e_phi, rel=1e-13)
    assert E[1] == pytest.approx(1.0 / e_phi, rel=1e-13)
    assert E[2] == 0.0
