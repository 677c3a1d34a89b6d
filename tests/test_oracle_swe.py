"""Pins of the oracle's SWE operators and IMEX step against closed forms,
invariants and exact identities (paper Sec. 2 and App. A)."""

import math

import numpy as np
import pytest

from oracle import sht
from oracle.norms import rel_err, spectral_norm
from oracle.swe import Model, T_LG, T_LC, T_NL, T_VISC, T_ALL
from paper_2306_09497_amd import workloads

A = 6.37122e6
OM = 7.292e-5


def rand_state(M, rng, amp=(1e3, 1e-5, 1e-6), decay=1.0):
    nc = sht.ncoef(M)
    U = np.zeros((3, nc), dtype=np.complex128)
    n = np.concatenate([np.arange(m, M + 1) for m in range(M + 1)]).astype(float)
    shape = 1.0 / (1.0 + n) ** decay
    for f in range(3):
        c = rng.standard_normal(nc) + 1j * rng.standard_normal(nc)
        c[:M + 1] = c[:M + 1].real
        U[f] = amp[f] * c * shape
    U[1, 0] = U[2, 0] = 0.0
    return U


def test_solid_body_advection():
    """P6: Phi' advected by solid-body rotation (delta = 0):
    N_Phi_{m,n} = -(u0/a) i m Phi'_{m,n} exactly."""
    M = 21
    md = Model(M, 64, 32, phibar=3e4)
    rng = np.random.default_rng(3)
    u0 = 40.0
    U = np.zeros((3, md.grid.nc), dtype=complex)
    U[0] = rand_state(M, rng)[0]
    U[0, 0] = 3e4
    U[1, sht.idx(M, 0, 1)] = 2 * u0 / (A * math.sqrt(3))
    N = md.tendencies(U)
    want = -(u0 / A) * md.grid.im() * U[0]
    assert np.max(np.abs(N[0] - want)) < 1e-12 * np.max(np.abs(want))


@pytest.mark.parametrize("M,nlon,nlat", [(21, 64, 32), (63, 192, 96)])
def test_balanced_flow(M, nlon, nlat):
    """P7: steady solid-body rotation in gradient-wind balance:
    L(U) + N(U) = 0 to rounding."""
    md = Model(M, nlon, nlat, phibar=2.94e4)
    U = workloads.solid_body(M)
    N = md.tendencies(U)
    L = md.apply_linear(U)
    scale = np.max(np.abs(N), axis=1) + np.max(np.abs(L), axis=1)
    assert np.all(np.max(np.abs(N + L), axis=1) <= 2e-12 * scale + 1e-300)


def test_tilted_solid_body_no_rotation():
    """P7: with Omega = 0 solid-body rotation about a tilted axis is steady:
    u = u0 cos(lat'), Phi = Phi0 - u0^2 mu'^2 / 2, mu' = mu cos(al) +
    cos(lat) cos(lambda) sin(al).  L_G(U) + N(U) = 0 (nonzero m = 1, 2)."""
    M = 21
    md = Model(M, 64, 32, omega=0.0, phibar=2.5e4)
    g = md.grid
    al, u0 = 0.7, 30.0
    cl = np.sqrt(g.coslat2)[:, None]
    mup = g.mu[:, None] * math.cos(al) + cl * np.cos(g.lam)[None, :] * math.sin(al)
    xi = g.anal(2 * u0 * mup / A)
    Phi = g.anal(2.6e4 - 0.5 * u0 ** 2 * mup ** 2)
    U = np.stack([Phi, xi, np.zeros_like(xi)])
    assert np.abs(xi[sht.idx(M, 1, 1)]) > 1e-6       # really non-zonal
    R = md.tendencies(U) + md.apply_linear(U, terms=T_LG)
    assert np.max(np.abs(R[1])) < 1e-13 * np.max(np.abs(md.tendencies(U)[1]) + 1e-30) + 1e-24
    # rounding floor: the 2.6e4 mean of Phi enters every analysed coefficient
    assert np.max(np.abs(R[2])) < 1e-11 * np.max(np.abs(md.apply_linear(U, T_LG)[2]))
    assert np.max(np.abs(R[0])) < 1e-12 * np.max(np.abs(Phi[1:]) * 1e-5)


def test_potential_flow_closed_form():
    """Divergent flow chi = c mu, xi = 0, Phi = Phi0 + d mu, with Phibar != Phi0:
    N_Phi = (c d / a^2)(3 mu^2 - 1) + 2 c (Phi0 - Phibar) mu / a^2,
    N_xi = 0, N_delta = -lap(|V|^2/2) = -2 c^2 / (sqrt5 a^4) Y_{0,2}."""
    M = 21
    phibar, phi0, c, d = 2.0e4, 2.3e4, 3.0e7, 500.0
    md = Model(M, 64, 32, phibar=phibar)
    U = np.zeros((3, md.grid.nc), dtype=complex)
    U[0, sht.idx(M, 0, 0)] = phi0
    U[0, sht.idx(M, 0, 1)] = d / math.sqrt(3)
    U[2, sht.idx(M, 0, 1)] = -2 * c / A ** 2 / math.sqrt(3)    # lap(c mu)
    N = md.tendencies(U)
    want = np.zeros_like(N)
    want[0, sht.idx(M, 0, 2)] = (c * d / A ** 2) * 2 / math.sqrt(5)
    want[0, sht.idx(M, 0, 1)] = 2 * c * (phi0 - phibar) / (A ** 2 * math.sqrt(3))
    want[2, sht.idx(M, 0, 2)] = -2 * c ** 2 / (math.sqrt(5) * A ** 4)
    for f in range(3):
        scale = max(np.max(np.abs(want[f])), np.max(np.abs(want[0])) * 1e-6)
        assert np.max(np.abs(N[f] - want[f])) < 1e-12 * scale


@pytest.mark.parametrize("M,nlon,nlat", [(21, 66, 34), (42, 128, 64)])
def test_coriolis_galerkin_vs_grid(M, nlon, nlat):
    """The Galerkin Coriolis matrices equal the projection of the grid-point
    operator: L_C U = (0, -div(f V), curl(f V)), f = 2 Omega mu, computed
    with the (pinned) vector transforms on an alias-free grid."""
    md = Model(M, nlon, nlat)
    g = md.grid
    U = rand_state(M, np.random.default_rng(11))
    psi, chi = U[1] * g.invlap, U[2] * g.invlap
    Uf, Vf = g.uv_fourier_from_psichi(psi, chi)
    f = 2 * OM * g.mu[:, None]
    fU = g.grid_to_fourier(f * g.fourier_to_grid(Uf))
    fV = g.grid_to_fourier(f * g.fourier_to_grid(Vf))
    div, curl = g.div_curl_from_fourier(fU, fV)
    LC = md.apply_linear(U, terms=T_LC)
    assert np.max(np.abs(LC[0])) == 0.0
    assert np.max(np.abs(LC[1] + div)) < 1e-12 * np.max(np.abs(div))
    assert np.max(np.abs(LC[2] - curl)) < 1e-12 * np.max(np.abs(curl))


def energy(U, md):
    """Linear SWE energy: sum' |Phi'|^2 + Phibar a^2/(n(n+1)) (|xi|^2 + |delta|^2)."""
    g = md.grid
    w = np.where(g.m_of == 0, 1.0, 2.0)
    n = g.n_of.astype(float)
    k = np.where(n > 0, md.phibar * md.a ** 2 / np.where(n > 0, n * (n + 1), 1), 0.0)
    e = w * np.abs(U[0]) ** 2 + w * k * (np.abs(U[1]) ** 2 + np.abs(U[2]) ** 2)
    e[0] = 0.0
    return float(np.sum(e))


def test_cn_energy_conservation():
    """P8: CN (a Cayley transform of a skew-adjoint operator in the energy
    inner product) conserves the linear SWE energy with Coriolis."""
    M = 21
    md = Model(M, 64, 32, phibar=5e4)
    U = rand_state(M, np.random.default_rng(2), decay=0.5)
    e0 = energy(U, md)
    for _ in range(300):
        U = md.cn_half(U, 1800.0, terms=T_LG | T_LC)
    assert abs(energy(U, md) - e0) < 1e-12 * e0


def test_cn_amplification():
    """P9: Omega = 0, gravity only: each (Phi, delta) mode is a combination of
    eigenvectors (1, -lambda/Phibar), lambda = +-i sqrt(n(n+1) Phibar)/a, each
    multiplied per half step by (4 + lambda dt)/(4 - lambda dt) (Sec. 4.1.1)."""
    M = 21
    pb, dt = 1e5, 900.0
    md = Model(M, 64, 32, omega=0.0, phibar=pb)
    g = md.grid
    U = rand_state(M, np.random.default_rng(4))
    out = md.cn_half(U, 2 * dt, terms=T_LG)     # alpha = (2 dt)/4 = dt/2
    n = g.n_of.astype(float)
    lam = 1j * np.sqrt(n * (n + 1) * pb) / A
    for k in range(1, g.nc):
        l1, l2 = lam[k], -lam[k]
        # solve c1 v1 + c2 v2 = (Phi, delta)
        Mv = np.array([[1, 1], [-l1 / pb, -l2 / pb]])
        c = np.linalg.solve(Mv, [U[0, k], U[2, k]])
        amp = [(4 + l * 2 * dt) / (4 - l * 2 * dt) for l in (l1, l2)]
        want = Mv @ (c * np.array(amp))
        assert abs(out[0, k] - want[0]) < 1e-12 * abs(U[0]).max()
        assert abs(out[2, k] - want[1]) < 1e-12 * abs(U[2]).max()
    assert np.max(np.abs(out[1] - U[1])) == 0.0


def test_viscosity_factor():
    """P10: backward-Euler damping b = 1/(1 + dt nu (n(n+1)/a^2)^(q/2))
    per step on every field (App. A)."""
    M = 21
    md = Model(M, 64, 32)
    U = rand_state(M, np.random.default_rng(5))
    dt, nu, q = 120.0, 1e15, 4
    out = md.imex_step(U, dt, nu, q, terms=T_VISC)
    n = md.grid.n_of.astype(float)
    b = 1.0 / (1.0 + dt * nu * (n * (n + 1) / A ** 2) ** 2)
    assert np.allclose(out, U * b[None, :], rtol=1e-15, atol=0)
    assert out[0, 0] == U[0, 0]


def jet_state(M, nlon, nlat, phibar=9.80616e4, amp=120.0, lam_c=1.0):
    md = Model(M, nlon, nlat, phibar=phibar)
    G = workloads.jet_bump_grid(md.grid.mu, nlon, phibar=phibar, amp=amp, lam_c=lam_c)
    U = np.stack([md.grid.anal(G[0]), md.grid.anal(G[1]), md.grid.anal(G[2])])
    return md, U


def test_mass_conservation():
    """P11: the (0,0) coefficient of Phi (global mass) is invariant."""
    md, U = jet_state(21, 64, 32)
    m0 = U[0, 0]
    for _ in range(60):
        U = md.imex_step(U, 300.0, 1e16, 4, terms=T_ALL)
    assert abs(U[0, 0] - m0) < 1e-13 * abs(m0)
    assert abs(U[0, 0].imag) == 0.0


def test_alias_free_tendencies():
    """P12: on a 3/2-rule grid, N(U) equals N(U) on a twice finer grid."""
    M = 42
    md1, U = jet_state(M, 128, 64, amp=300.0)
    md2 = Model(M, 256, 128, phibar=md1.phibar)
    U = U + rand_state(M, np.random.default_rng(9), amp=(50.0, 2e-6, 5e-7))
    N1, N2 = md1.tendencies(U), md2.tendencies(U)
    for f in range(3):
        assert np.max(np.abs(N1[f] - N2[f])) < 1e-12 * np.max(np.abs(N2[f]))


def test_steady_state_second_order():
    """P18: the balanced state drifts only by the O(dt^2) splitting error."""
    M = 21
    md = Model(M, 64, 32, phibar=2.94e4)
    U0 = workloads.solid_body(M)
    T = 6 * 3600.0
    drift = []
    for dt in (1200.0, 600.0):
        U = md.propagate(U0, dt, int(T / dt))
        drift.append(np.max(rel_err(U, U0, M)))
    ratio = drift[0] / drift[1]
    assert drift[0] < 1e-3
    assert 3.5 < ratio < 4.5


def test_second_order_in_time():
    """P19: the IMEX step is second order (Heun reading of the explicit
    stage); a first-order variant would show ratio ~2."""
    md, U0 = jet_state(21, 64, 32)
    T = 4 * 3600.0
    ref = md.propagate(U0, 600.0 / 8, int(T / (600.0 / 8)))
    errs = []
    for dt in (600.0, 300.0):
        U = md.propagate(U0, dt, int(T / dt))
        errs.append(np.max(rel_err(U, ref, 21)))
    ratio = errs[0] / errs[1]
    assert 3.3 < ratio < 4.7, (errs, ratio)


def test_float64_rounding_floor_of_divergence_tendency():
    """The float64 oracle against itself in extended precision: the plain
    spectral L2 of N_delta carries a rounding floor far above the other fields
    (the Laplacian of the kinetic energy amplifies rounding by n(n+1)), while
    the wind norm and Phi' stay near machine precision.  This is why parity
    of vorticity/divergence is stated in the wind norm."""
    from oracle.norms import state_rel_err
    M = 63
    md, U = jet_state(M, 192, 96)
    U = workloads.white_noise(M, U, 1e-4, 2)
    mx = Model(M, 192, 96, phibar=md.phibar, extended=True)
    N0 = md.tendencies(U)
    Nx = mx.tendencies(U.astype(np.clongdouble)).astype(np.complex128)
    plain = rel_err(N0, Nx, M)
    energy = state_rel_err(N0, Nx, M)
    assert plain[2] > 5 * energy[1]          # delta is the ill-conditioned field
    assert np.all(energy < 1e-12) and plain[0] < 1e-13
