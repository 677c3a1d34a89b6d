"""Seeded synthetic initial states shaped like the paper's test cases.

This module holds no part of the method's arithmetic: it defines test inputs
only (closed-form spectral coefficients, analytic grid-point profiles and seeded
random numbers).  Both the GPU path and the CPU oracle consume what it makes.

Spectral layout: packed m-major, idx(m, n) = m(2M+3-m)/2 + (n-m), complex128,
fields ordered (Phi, xi, delta); Phi in full (its (0,0) coefficient is the area
mean).  Normalisation: 1/2 int Pbar^2 dmu = 1, so Y_{0,1} = sqrt(3) mu and
Y_{0,2} = sqrt(5) (3 mu^2 - 1) / 2.

* ``solid_body``: steady zonal flow u = u0 cos(lat) in gradient-wind balance,
  d Phi / d lat = -a u (f + u tan(lat) / a), which gives
  Phi = Phi0 - (a Omega u0 + u0^2/2) mu^2 and xi = 2 u0 mu / a, delta = 0.
  All of it is band-limited (n <= 2) and written down in closed form here.
  Optional seeded white spectral noise (relative amplitude ``noise``).
* ``jet_bump_grid``: a midlatitude zonal jet (smooth compact bump profile in
  latitude) in gradient-wind balance, plus a localised Gaussian height bump;
  returns grid-point (Phi, xi, delta) at caller-given Gauss latitudes.  This is
  a synthetic stand-in with the shape of the unstable-jet test (Sec. 5.2), not
  its published profile.
* ``gaussian_bumps_grid``: the Gaussian-bumps test case (Sec. 5.1): a fluid at
  rest with mean depth hbar and three Gaussian height bumps of amplitude A at
  the printed centres and widths; geopotential Phi = g (hbar + A sum_i
  exp(-a_i d_i^2)), d_i the great-circle angle to centre i.  Grid-point
  (Phi, xi, delta) at caller-given Gauss latitudes.
"""

import math

import numpy as np

A_EARTH = 6.37122e6
OMEGA = 7.292e-5
G_EARTH = 9.80616


def ncoef(M):
    return (M + 1) * (M + 2) // 2


def _idx(M, m, n):
    return m * (2 * M + 3 - m) // 2 + (n - m)


def _norm(c, M, exclude_mean):
    w = np.full(ncoef(M), 2.0)
    w[:M + 1] = 1.0                      # m = 0 block
    if exclude_mean:
        w[0] = 0.0
    return math.sqrt(float(np.sum(w * np.abs(c) ** 2)))


def white_noise(M, base, amp, seed):
    """Seeded white spectral noise added to every (m, n) with n >= 1.

    For field f the per-mode amplitude is amp * sigma_f * (X + iY)/sqrt(2),
    X, Y ~ N(0,1) (Y = 0 at m = 0); sigma_f is the norm of the base field
    (Phi without its mean; xi's norm is used for delta whose base is 0).
    Draw order: field, m, n.
    """
    rng = np.random.default_rng(seed)
    out = base.copy()
    sig = [_norm(base[0], M, True), _norm(base[1], M, False), _norm(base[2], M, False)]
    if sig[2] == 0.0:
        sig[2] = sig[1]
    for f in range(3):
        for m in range(M + 1):
            for n in range(max(m, 1), M + 1):
                x = rng.standard_normal()
                y = rng.standard_normal() if m > 0 else 0.0
                out[f, _idx(M, m, n)] += amp * sig[f] * complex(x, y) / math.sqrt(2.0)
    return out


def solid_body(M, a=A_EARTH, omega=OMEGA, u0=None, phi0=2.94e4, noise=0.0,
               seed=0):
    """(Phi, xi, delta) spectral coefficients of steady solid-body rotation."""
    if M < 2:
        raise ValueError("solid_body needs M >= 2")
    if u0 is None:
        u0 = 2.0 * math.pi * a / (12.0 * 86400.0)
    C = a * omega * u0 + 0.5 * u0 * u0
    U = np.zeros((3, ncoef(M)), dtype=np.complex128)
    # mu^2 = 1/3 Y_00 + 2/(3 sqrt 5) Y_02
    U[0, _idx(M, 0, 0)] = phi0 - C / 3.0
    U[0, _idx(M, 0, 2)] = -C * 2.0 / (3.0 * math.sqrt(5.0))
    # xi = 2 u0 mu / a = (2 u0 / (a sqrt 3)) Y_01
    U[1, _idx(M, 0, 1)] = 2.0 * u0 / (a * math.sqrt(3.0))
    if noise > 0.0:
        U = white_noise(M, U, noise, seed)
    return U


# ----------------------------------------------------------------------------
# jet + bump on a caller-given Gauss grid
# ----------------------------------------------------------------------------
def _bump(x):
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    inside = np.abs(x) < 1.0
    xi = x[inside]
    out[inside] = np.exp(1.0 - 1.0 / (1.0 - xi * xi))
    return out


def _bump_deriv(x):
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    inside = np.abs(x) < 1.0
    xi = x[inside]
    out[inside] = np.exp(1.0 - 1.0 / (1.0 - xi * xi)) * (-2.0 * xi / (1.0 - xi * xi) ** 2)
    return out


def jet_profile(theta, umax=80.0, theta0=math.pi / 4, width=math.radians(20.0)):
    return umax * _bump((theta - theta0) / width)


def jet_bump_grid(mu, nlon, a=A_EARTH, omega=OMEGA, g=G_EARTH,
                  phibar=G_EARTH * 1.0e4, umax=80.0, theta0=math.pi / 4,
                  width=math.radians(20.0), amp=120.0, alpha=1.0 / 3.0,
                  beta=1.0 / 15.0, theta_c=math.pi / 4, lam_c=0.0):
    """Grid-point (Phi, xi, delta), shape (3, nlat, nlon), at latitudes
    asin(mu) and longitudes 2 pi k / nlon."""
    from scipy.integrate import quad

    mu = np.asarray(mu, dtype=np.float64)
    theta = np.arcsin(mu)
    lam = 2.0 * np.pi * np.arange(nlon) / nlon
    lo, hi = theta0 - width, theta0 + width

    def u_of(t):
        return umax * float(_bump(np.array([(t - theta0) / width]))[0])

    def dphi(t):       # d Phi / d theta from gradient-wind balance
        u = u_of(t)
        return -a * u * (2.0 * omega * math.sin(t) + u * math.tan(t) / a)

    opts = dict(epsabs=1e-9, epsrel=1e-13, limit=200)
    # area mean of (Phi - Phi_south) is 1/2 int dphi (1 - sin t) dt
    mean_off = 0.5 * quad(lambda t: dphi(t) * (1.0 - math.sin(t)), lo, hi, **opts)[0]
    phi_south = phibar - mean_off
    total = quad(dphi, lo, hi, **opts)[0]
    phi_lat = np.empty(theta.size)
    for j, t in enumerate(theta):
        if t <= lo:
            phi_lat[j] = phi_south
        elif t >= hi:
            phi_lat[j] = phi_south + total
        else:
            phi_lat[j] = phi_south + quad(dphi, lo, t, **opts)[0]
    u = jet_profile(theta, umax, theta0, width)
    dudt = umax * _bump_deriv((theta - theta0) / width) / width
    xi_lat = -(dudt - u * np.tan(theta)) / a          # -(1/(a cos)) d(u cos)/d theta
    dl = np.angle(np.exp(1j * (lam[None, :] - lam_c)))  # wrapped to (-pi, pi]
    hprime = amp * np.exp(-(dl / alpha) ** 2) * np.exp(-((theta[:, None] - theta_c) / beta) ** 2)
    Phi = phi_lat[:, None] + g * hprime
    xi = np.repeat(xi_lat[:, None], nlon, axis=1)
    de = np.zeros_like(Phi)
    return np.stack([Phi, xi, de])


def jet_bump_params(seed, amp=120.0):
    """Seeded bump longitude (and the given amplitude)."""
    rng = np.random.default_rng(seed)
    return dict(lam_c=float(rng.uniform(0.0, 2.0 * math.pi)), amp=float(amp))


# centres (longitude, latitude) and sharpness a_i of the three bumps (Sec. 5.1)
GAUSSIAN_BUMPS = ((math.pi / 5, math.pi / 3, 20.0),
                  (6 * math.pi / 5, math.pi / 5, 80.0),
                  (8 * math.pi / 5, -math.pi / 4, 360.0))


def gaussian_bumps_grid(mu, nlon, g=G_EARTH, hbar=29400.0, amp=6000.0, bumps=GAUSSIAN_BUMPS):
    """Grid-point (Phi, xi, delta), shape (3, nlat, nlon): Phi = g (hbar + amp
    sum_i exp(-a_i d_i^2)), zero wind.  The mean geopotential parameter of the
    model is g * hbar."""
    mu = np.asarray(mu, dtype=np.float64)
    theta = np.arcsin(mu)[:, None]
    lam = 2.0 * np.pi * np.arange(nlon)[None, :] / nlon
    h = np.zeros((mu.size, nlon))
    for lam_i, th_i, a_i in bumps:
        c = np.sin(theta) * math.sin(th_i) + np.cos(theta) * math.cos(th_i) * np.cos(lam - lam_i)
        d = np.arccos(np.clip(c, -1.0, 1.0))
        h += np.exp(-a_i * d * d)
    Phi = g * (hbar + amp * h)
    zero = np.zeros_like(Phi)
    return np.stack([Phi, zero, zero.copy()])
