"""Pins of the SL-SI-SETTLS oracle (Sec. 2.3.2, Sec. 3.2.4) against closed
forms and against the dense Galerkin operator of the IMEX oracle."""

import math

import numpy as np
import pytest

from oracle import sl
from oracle.sht import gauss_nodes, m_slice
from oracle.swe import Model
from paper_2306_09497_amd import workloads

A = 6.37122e6


def _lat(nlat):
    return np.arcsin(gauss_nodes(nlat)[0])


def test_interp_exact_on_cubic_products():
    """Away from the seam and the poles the stencil is a plain tensor-product
    cubic: products of cubics in longitude and latitude come out exactly."""
    nlat, nlon = 32, 64
    lat = _lat(nlat)
    lam_g, th_g = np.meshgrid(2 * np.pi * np.arange(nlon) / nlon, lat)
    rng = np.random.default_rng(1)
    p = rng.standard_normal(4)
    q = rng.standard_normal(4)

    def f(lam, th):
        return np.polyval(p, lam) * np.polyval(q, th)

    dl = 2 * np.pi / nlon
    lam = rng.uniform(dl, 2 * np.pi - 3 * dl, 500)
    th = rng.uniform(lat[nlat - 3], lat[2], 500)
    got = sl.interp(lat, nlon, f(lam_g, th_g), lam, th)
    assert np.max(np.abs(got - f(lam, th))) <= 1e-11 * np.max(np.abs(f(lam, th)))


def test_interp_fourth_order_across_the_poles():
    """A smooth field on the sphere, sampled in the polar caps and beyond the
    outermost Gauss rows (where the mirrored rows are used): the error falls
    by about 2^4 per grid doubling."""
    k = np.array([0.3, -0.5, 0.8])
    k /= np.linalg.norm(k)
    rng = np.random.default_rng(2)
    lam = rng.uniform(0, 2 * np.pi, 400)
    th = np.concatenate([rng.uniform(1.35, np.pi / 2, 200), rng.uniform(-np.pi / 2, -1.35, 200)])
    exact = np.exp(np.tensordot(k, sl.cart(lam, th), axes=1))
    errs = []
    for nlat in (24, 48, 96):
        nlon = 2 * nlat
        lam_g, th_g = np.meshgrid(2 * np.pi * np.arange(nlon) / nlon, _lat(nlat))
        g = np.exp(np.tensordot(k, sl.cart(lam_g, th_g), axes=1))
        errs.append(np.max(np.abs(sl.interp(_lat(nlat), nlon, g, lam, th) - exact)))
    assert errs[0] < 1e-3
    assert errs[0] / errs[1] > 12 and errs[1] / errs[2] > 12


def test_vector_components_interpolate_without_sign_flips():
    """Cartesian components of a tangent field (solid-body rotation about a
    tilted axis) are linear in position: interpolated across a pole they stay
    tangent and of the right length."""
    nlat, nlon = 48, 96
    lat = _lat(nlat)
    lam_g, th_g = np.meshgrid(2 * np.pi * np.arange(nlon) / nlon, lat)
    ax = np.array([1.0, 0.0, 1.0]) / math.sqrt(2.0)
    V = np.cross(ax[:, None, None], sl.cart(lam_g, th_g), axis=0)
    lam = np.linspace(0.1, 6.2, 50)
    th = np.full(50, 1.55)
    x = sl.cart(lam, th)
    want = np.cross(ax[:, None], x, axis=0)
    got = sl.interp(lat, nlon, V, lam, th)
    assert np.max(np.abs(got - want)) < 1e-5


def test_rotation_takes_departure_to_arrival():
    rng = np.random.default_rng(3)
    xd = rng.standard_normal((3, 20))
    xd /= np.linalg.norm(xd, axis=0)
    xa = xd + 0.05 * rng.standard_normal((3, 20))
    xa /= np.linalg.norm(xa, axis=0)
    assert np.allclose(sl.rotate_to(xd, xd, xa), xa, atol=1e-14)
    # an orthogonal map: lengths and the tangent property are kept
    t = np.cross(xd, rng.standard_normal((3, 20)), axis=0)
    rt = sl.rotate_to(t, xd, xa)
    assert np.allclose(np.linalg.norm(rt, axis=0), np.linalg.norm(t, axis=0), rtol=1e-14)
    assert np.max(np.abs(np.sum(rt * xa, axis=0))) < 1e-14


def test_trajectory_fixed_point_for_solid_body_rotation():
    """For a steady solid-body rotation V = w a (k x x) the fixed point of eq.
    SETTLS_trajectories is the arrival point turned back about k by exactly
    2 atan(w dt / 2) (the implicit-midpoint rotation)."""
    nlat, nlon = 64, 128
    lat = _lat(nlat)
    lam_g, th_g = np.meshgrid(2 * np.pi * np.arange(nlon) / nlon, lat)
    k = np.array([0.4, 0.2, 0.9])
    k /= np.linalg.norm(k)
    w = 40.0 / A
    dt = 3600.0
    xa = sl.cart(lam_g, th_g)
    V = w * A * np.cross(k[:, None, None], xa, axis=0)
    xd = sl.departure_points(lat, nlon, V, V, dt, A, 40)
    al = -2.0 * math.atan(0.5 * w * dt)
    kx = np.tensordot(k, xa, axes=1)
    want = (xa * math.cos(al) + np.cross(k[:, None, None], xa, axis=0) * math.sin(al)
            + k[:, None, None] * kx * (1 - math.cos(al)))
    moved = np.max(np.linalg.norm(xa - want, axis=0))
    assert moved > 0.02
    assert np.max(np.linalg.norm(xd - want, axis=0)) < 1e-6 * moved


def _smooth_state(M, seed, phibar):
    return workloads.solid_body(M, phi0=phibar, noise=0.05, seed=seed)


def test_no_displacement_limit_is_crank_nicolson_on_L():
    """With no trajectory iterations (x_d = x_a) the scheme is Crank-Nicolson
    on L with the extrapolated N_R:
    (I - dt/2 L) U^{n+1} = (I + dt/2 L) U^n + dt/2 (3 N_R^n - N_R^{n-1}).
    The grid-point linear terms must equal the dense Galerkin L."""
    M, pb, dt = 21, 3.0e4, 1800.0
    md = Model(M, 64, 32, phibar=pb)
    U = _smooth_state(M, 4, pb)
    Up = _smooth_state(M, 5, pb)
    st = sl.SLStepper(md, dt, iters=0)
    got = st.step(U, Up)
    gr = md.grid

    def nr(X):
        ph, d = st.grid_fields(X)[:2]
        out = np.zeros_like(X)
        out[0] = gr.anal(-ph * d)
        return out

    rhs = U + 0.5 * dt * md.apply_linear(U) + 0.5 * dt * (3 * nr(U) - nr(Up))
    want = np.zeros_like(U)
    for m in range(M + 1):
        L = md.linear_matrix(m)
        s = m_slice(M, m)
        K = M - m + 1
        x = np.linalg.solve(np.eye(3 * K) - 0.5 * dt * L,
                            np.concatenate([rhs[0, s], rhs[1, s], rhs[2, s]]))
        want[0, s], want[1, s], want[2, s] = x[:K], x[K:2 * K], x[2 * K:]
    for f in range(3):
        ref = want[f].copy()
        if f == 0:
            ref[0] -= pb                                  # compare Phi'
        assert np.linalg.norm(got[f] - want[f]) <= 1e-11 * np.linalg.norm(ref), f


def _williamson2(md, u0, alpha):
    """Steady solid-body flow about an axis tilted by alpha (Williamson et
    al. 1992, test 2; with f = 2 Omega mu fixed to the polar axis the tilted
    flow is steady for Omega = 0 only): spectral state of an oracle Model."""
    gr, a, om = md.grid, md.a, md.omega
    lat = np.arcsin(gr.mu)
    lam, th = np.meshgrid(gr.lam, lat)
    s = -np.cos(lam) * np.cos(th) * np.sin(alpha) + np.sin(th) * np.cos(alpha)
    phi = md.phibar - (a * om * u0 + 0.5 * u0 * u0) * s * s
    u = u0 * (np.cos(th) * np.cos(alpha) + np.cos(lam) * np.sin(th) * np.sin(alpha))
    v = -u0 * np.sin(lam) * np.sin(alpha)
    cos = np.cos(th)
    div, curl = gr.div_curl_from_fourier(gr.grid_to_fourier(u * cos), gr.grid_to_fourier(v * cos))
    U = np.stack([gr.anal(phi), curl, div])
    U[1][0] = U[2][0] = 0.0
    return U


def test_steady_tilted_flow_is_kept():
    """Tilted steady flow: after 12 h the state has moved by less than 1e-4
    (5e-5 at dt = 3600 s); a wind projected on the arrival frame without
    being turned there loses about 1e-3 of its length."""
    M = 42
    md = Model(M, 128, 64, omega=0.0, phibar=2.94e4)
    U0 = _williamson2(md, 2 * math.pi * A / (12 * 86400.0), math.pi / 4)
    for dt in (3600.0, 1800.0):
        st = sl.SLStepper(md, dt)
        U, _ = st.propagate(U0, int(round(12 * 3600 / dt)))
        for f in (0, 1):
            ref = U0[f].copy()
            if f == 0:
                ref[0] -= md.phibar
            assert np.linalg.norm(U[f] - U0[f]) < 1e-4 * np.linalg.norm(ref), (dt, f)


def test_second_order_in_time():
    """A smooth large-scale perturbation of solid-body flow, 12 h, against a
    fine IMEX reference (dt = 60 s): the error of every field falls by about
    4 per halving of dt (dt = 3600, 1800, 900 s; the interpolation floor is
    below these errors at T21)."""
    M, pb = 21, 2.94e4
    md = Model(M, 64, 32, phibar=pb)
    U0 = workloads.solid_body(M, phi0=pb)
    U0[0, workloads._idx(M, 2, 4)] += 800.0 * (1 + 0.5j)
    U0[1, workloads._idx(M, 3, 5)] += 2e-6
    T = 12 * 3600.0
    ref = md.propagate(U0, 60.0, int(T / 60.0))
    errs = []
    for dt in (3600.0, 1800.0, 900.0):
        U, _ = sl.SLStepper(md, dt).propagate(U0, int(round(T / dt)))
        errs.append([np.linalg.norm(U[f] - ref[f]) / np.linalg.norm(ref[f] - U0[f] * (f == 0))
                     for f in range(3)])
    errs = np.array(errs)
    r = errs[:-1] / errs[1:]
    assert np.all(r > 2.8) and np.all(r < 5.0), errs
