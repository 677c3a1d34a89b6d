"""Pins of the oracle's spherical-harmonic transform against closed forms,
library routines and exact identities (paper Sec. 2.2)."""

import math

import numpy as np
import pytest
from scipy.special import lpmv

from oracle import sht
from oracle.norms import spectral_norm

A = 6.37122e6


def rand_spec(M, rng, scale=1.0):
    c = rng.standard_normal(sht.ncoef(M)) + 1j * rng.standard_normal(sht.ncoef(M))
    c[:M + 1] = c[:M + 1].real            # m = 0 coefficients of a real field
    return scale * c


@pytest.mark.parametrize("nlat", [8, 32, 96, 384])
def test_gauss_moments(nlat):
    """P1: sum w = 2 and exact integration of mu^k for k <= 2 nlat - 1."""
    mu, w = sht.gauss_nodes(nlat)
    assert np.all(np.diff(mu) < 0)        # north to south
    x, wl = np.polynomial.legendre.leggauss(nlat)   # library routine
    assert np.max(np.abs(mu[::-1] - x)) < 1e-15
    assert np.max(np.abs(w[::-1] - wl) / wl) < 1e-9      # numpy loses digits here
    for k in range(2 * nlat):
        exact = 2.0 / (k + 1) if k % 2 == 0 else 0.0
        assert abs(np.sum(w * mu ** k) - exact) < 2e-15 * (1 + nlat / 32)


def test_pbar_closed_forms():
    """P2: Pbar_1^0 = sqrt3 mu, Pbar_1^1 = sqrt(3/2) sqrt(1-mu^2), and scipy's
    associated Legendre functions with the normalisation and the
    Condon-Shortley phase removed."""
    mu = np.linspace(-0.99, 0.99, 41)
    P = sht.pbar_table(20, mu)
    assert np.allclose(P[0][1], math.sqrt(3.0) * mu, rtol=0, atol=1e-15)
    assert np.allclose(P[1][0], math.sqrt(1.5) * np.sqrt(1 - mu ** 2), rtol=0, atol=1e-15)
    for m in range(0, 21):
        for n in range(m, 21):
            norm = math.sqrt((2 * n + 1) * math.factorial(n - m) / math.factorial(n + m))
            ref = (-1) ** m * norm * lpmv(m, n, mu)
            assert np.max(np.abs(P[m][n - m] - ref)) < 1e-12 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("M,nlat", [(21, 32), (63, 96), (255, 384)])
def test_pbar_orthonormal(M, nlat):
    """P2: discrete orthonormality 1/2 sum_j w_j Pbar_n Pbar_n' = delta."""
    mu, w = sht.gauss_nodes(nlat)
    P = sht.pbar_table(M, mu)
    for m in range(0, M + 1, max(1, M // 16)):
        G = 0.5 * (P[m] * w) @ P[m].T
        assert np.max(np.abs(G - np.eye(M - m + 1))) < 1e-13


def test_hbar_derivative():
    """Hbar_n^m = (1-mu^2) dPbar/dmu: closed forms for low degrees and a
    4th-order central difference of the Pbar recurrence elsewhere."""
    mu = np.linspace(-0.95, 0.95, 39)
    P = sht.pbar_table(13, mu)
    H = sht.hbar_table(P, mu, 13)
    s = np.sqrt(1 - mu ** 2)
    assert np.allclose(H[0][1], math.sqrt(3) * (1 - mu ** 2), atol=1e-14)
    assert np.allclose(H[0][2], (1 - mu ** 2) * 3 * math.sqrt(5) * mu, atol=1e-14)
    assert np.allclose(H[1][0], -math.sqrt(1.5) * mu * s, atol=1e-14)
    h = 1e-3
    Pp = [sht.pbar_table(13, mu + k * h) for k in (-2, -1, 1, 2)]
    for m in range(13):
        for n in range(m, 13):
            d = (Pp[0][m][n - m] - 8 * Pp[1][m][n - m] + 8 * Pp[2][m][n - m]
                 - Pp[3][m][n - m]) / (12 * h)
            assert np.max(np.abs(H[m][n - m] - (1 - mu ** 2) * d)) < 2e-6 * (n + 1) ** 4


def test_fourier_vs_direct_dft():
    """P3: longitude transform equals the direct sum
    s(lambda_k) = sum_{|m|<=M} s_m exp(i m lambda_k) and its inverse."""
    rng = np.random.default_rng(1)
    M, nlon, nlat = 21, 64, 4
    g = sht.Grid(M, nlon, 32)
    f = rng.standard_normal((nlat, M + 1)) + 1j * rng.standard_normal((nlat, M + 1))
    f[:, 0] = f[:, 0].real
    direct = np.zeros((nlat, nlon))
    for k in range(nlon):
        lam = 2 * np.pi * k / nlon
        direct[:, k] = f[:, 0].real + 2 * np.real(
            np.sum(f[:, 1:] * np.exp(1j * np.arange(1, M + 1) * lam), axis=1))
    assert np.max(np.abs(g.fourier_to_grid(f) - direct)) < 1e-14 * np.sum(np.abs(f)) / nlat
    assert np.max(np.abs(g.grid_to_fourier(direct) - f)) < 1e-14


@pytest.mark.parametrize("M,nlon,nlat", [(21, 64, 32), (63, 192, 96), (127, 384, 192)])
def test_roundtrip(M, nlon, nlat):
    """P4: analysis(synthesis(c)) = c on the truncation (exact Gauss quadrature)."""
    rng = np.random.default_rng(M)
    g = sht.Grid(M, nlon, nlat, A)
    c = rand_spec(M, rng)
    back = g.anal(g.synth(c))
    assert np.max(np.abs(back - c)) < 2e-13 * np.max(np.abs(c))


def test_parseval_norm():
    """The spectral norm equals the area-weighted grid mean of x^2."""
    rng = np.random.default_rng(5)
    g = sht.Grid(21, 64, 32, A)
    c = rand_spec(21, rng)
    x = g.synth(c)
    grid_ms = 0.5 * np.sum(g.w[:, None] * x ** 2) / g.nlon
    assert abs(spectral_norm(c, 21) ** 2 - grid_ms) < 1e-12 * grid_ms


@pytest.mark.parametrize("M,nlon,nlat", [(21, 66, 34), (63, 192, 96)])
def test_div_curl_of_gradients(M, nlon, nlat):
    """P5: div(grad psi) = curl(k x grad psi) = lap psi = -n(n+1)/a^2 psi,
    and curl(grad psi) = div(k x grad psi) = 0 (Sec. 2.2 eigenrelation)."""
    rng = np.random.default_rng(7)
    g = sht.Grid(M, nlon, nlat, A)
    psi = rand_spec(M, rng)
    dl = g.legendre_synth(g.im() * psi) / A        # (1/a) d psi / d lambda
    dm = g.legendre_synth(psi, g.H) / A            # (1/a)(1-mu^2) d psi / d mu
    # grad psi: p = dl/cos, q = cos dmu psi / a  ->  A = dl, B = dm
    div, curl = g.div_curl_from_fourier(dl, dm)
    lap = g.lap * psi
    scale = np.max(np.abs(lap))
    assert np.max(np.abs(div - lap)) < 1e-12 * scale
    assert np.max(np.abs(curl)) < 1e-12 * scale
    # k x grad psi = (-q, p): A = -dm, B = dl
    div2, curl2 = g.div_curl_from_fourier(-dm, dl)
    assert np.max(np.abs(curl2 - lap)) < 1e-12 * scale
    assert np.max(np.abs(div2)) < 1e-12 * scale


def test_solid_body_velocity():
    """U = u cos(lat) of solid-body rotation xi = 2 u0 mu / a is u0 (1-mu^2)."""
    M = 21
    g = sht.Grid(M, 64, 32, A)
    u0 = 38.6
    xi = np.zeros(g.nc, dtype=complex)
    xi[sht.idx(M, 0, 1)] = 2 * u0 / (A * math.sqrt(3))
    psi = xi * g.invlap
    U, V = g.uv_fourier_from_psichi(psi, np.zeros_like(psi))
    assert np.max(np.abs(U[:, 0] - u0 * (1 - g.mu ** 2))) < 1e-13 * u0
    assert np.max(np.abs(U[:, 1:])) < 1e-13 * u0 and np.max(np.abs(V)) < 1e-13 * u0


def test_wind_norm_parseval():
    """wind_norm^2 equals the area-weighted grid mean of u^2 + v^2."""
    from oracle.norms import wind_norm
    M = 21
    g = sht.Grid(M, 64, 32, A)
    rng = np.random.default_rng(8)
    xi, de = rand_spec(M, rng, 1e-5), rand_spec(M, rng, 1e-6)
    xi[0] = de[0] = 0.0
    U, V = g.uv_fourier_from_psichi(xi * g.invlap, de * g.invlap)
    Ug, Vg = g.fourier_to_grid(U), g.fourier_to_grid(V)
    ms = 0.5 * np.sum(g.w[:, None] * (Ug ** 2 + Vg ** 2) / g.coslat2[:, None]) / g.nlon
    assert abs(wind_norm(xi, de, M, A) ** 2 - ms) < 1e-12 * ms


def test_truncate_pad_against_transforms():
    """Spectral restriction and prolongation between truncations M and Mc
    (spatial coarsening of coarse levels): on the fine grid's nodes, a
    truncation-Mc grid synthesises a coarse state exactly as the fine grid
    synthesises its zero-padded copy, and analyses any fine field to the
    truncation of its fine coefficients (exact Gauss quadrature)."""
    M, Mc, nlon, nlat = 21, 10, 64, 32
    Gf = sht.Grid(M, nlon, nlat)
    Gcf = sht.Grid(Mc, nlon, nlat)                 # truncation Mc on the fine nodes
    rng = np.random.default_rng(11)
    cc = rng.standard_normal(sht.ncoef(Mc)) + 1j * rng.standard_normal(sht.ncoef(Mc))
    cc[:Mc + 1] = cc[:Mc + 1].real                 # m = 0 coefficients real
    assert np.allclose(Gcf.synth(cc), Gf.synth(sht.pad(cc, Mc, M)), rtol=0, atol=1e-13)
    cf = rng.standard_normal(sht.ncoef(M)) + 1j * rng.standard_normal(sht.ncoef(M))
    cf[:M + 1] = cf[:M + 1].real
    g = Gf.synth(cf)
    assert np.allclose(Gcf.anal(g), sht.truncate(cf, M, Mc), rtol=0, atol=1e-13)
    # round trip and the zeros above Mc
    assert np.array_equal(sht.truncate(sht.pad(cc, Mc, M), M, Mc), cc)
    padded = sht.pad(cc, Mc, M)
    for m in range(M + 1):
        for n in range(m, M + 1):
            if n > Mc:
                assert padded[sht.idx(M, m, n)] == 0
