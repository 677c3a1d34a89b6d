"""Oracle: the semi-Lagrangian semi-implicit SETTLS step (Sec. 2.3.2, eqs.
SETTLS_trajectories and SL_SI_SETTLS) and its one-step variant (Sec. 3.2.4).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper writes the scheme for the state U generically.  On the sphere it is
read in the advective form of the equations of Sec. 2.1 (readings R33-R36):

* Phi' is carried as a scalar and the wind V = (u, v) as a vector along the
  trajectories; the linear terms are -Phibar delta (continuity) and
  -grad Phi' - f k x V (momentum), whose curl and divergence are L_C and L_G
  of Sec. 2.1; the nonlinear rest term is N_R = -Phi' delta.
* At the grid points at t_n:
      R_Phi = Phi' + dt/2 (-Phibar delta) + dt/2 (2 N_R^n - N_R^{n-1})
      R_V   = V + dt/2 (-grad Phi' - f k x V)
  both are interpolated to the departure points, dt/2 N_R^n is added at the
  arrival points, and U^{n+1} solves (I - dt/2 L) U^{n+1} = (R_Phi*, curl R_V*,
  div R_V*) in spectral space (L = L_G + L_C as in the IMEX Crank-Nicolson
  solve), followed by the backward-Euler viscosity (Sec. 2.3).
* Vectors are handled by their three Cartesian components, which are smooth
  across the poles; the interpolated vector is turned by the rotation that
  takes the departure point to the arrival point (about the axis x_d x x_a),
  then written in the arrival point's local east/north frame.
* Departure points: x_d^0 = x_a, then ``iters`` fixed-point iterations of eq.
  SETTLS_trajectories in 3-D, x_d <- normalise(x_a - dt/(2a) [2 V^n(x_d) -
  V^{n-1}(x_d) + V^n(x_a)]).
* Interpolation: tensor-product cubic Lagrange in (longitude, latitude) on
  the Gauss grid; the two rows beyond a pole are the two rows next to it,
  mirrored across the pole, at longitude + pi.
* One-step variant (Sec. 3.2.4): U^{n-1} is replaced by U^n.

Pins: tests/test_oracle_sl.py (exactness of the interpolation on cubic
products, its fourth-order convergence across the poles, the closed-form
fixed point of the trajectory iteration for solid-body rotation, the
no-displacement limit against the dense Galerkin linear operator, and the
preservation of a steady geostrophic flow with second-order convergence in
time).
"""

import numpy as np
import scipy.linalg

from .sht import m_slice


def cart(lam, th):
    """Unit position vectors [3, ...] of longitude lam, latitude th."""
    c = np.cos(th)
    return np.stack([c * np.cos(lam), c * np.sin(lam), np.sin(th)])


def frames(lam, th):
    """Local unit east and north vectors [3, ...]."""
    z = np.zeros_like(lam + th)
    east = np.stack([-np.sin(lam) + z, np.cos(lam) + z, z])
    north = np.stack([-np.sin(th) * np.cos(lam), -np.sin(th) * np.sin(lam), np.cos(th) + z])
    return east, north


def lonlat(x):
    """Longitude in [0, 2 pi) and latitude of unit vectors x [3, ...]."""
    lam = np.mod(np.arctan2(x[1], x[0]), 2.0 * np.pi)
    th = np.arctan2(x[2], np.hypot(x[0], x[1]))
    return lam, th


def _lagrange4(nodes, x):
    """Cubic Lagrange weights [4, ...] for nodes [4, ...] at x [...]."""
    w = []
    for i in range(4):
        wi = np.ones_like(x)
        for k in range(4):
            if k != i:
                wi = wi * (x - nodes[k]) / (nodes[i] - nodes[k])
        w.append(wi)
    return np.stack(w)


def interp(lat, nlon, f, lam, th):
    """Bicubic interpolation of grid fields f [..., nlat, nlon] (latitudes
    ``lat`` north to south, longitudes 2 pi k / nlon) at points (lam, th) of
    any shape; returns [..., *points.shape]."""
    nlat = lat.size
    # extended latitudes: two mirrored rows beyond each pole
    thx = np.concatenate([np.pi - lat[1::-1], lat, -np.pi - lat[:-3:-1]])
    rows = np.concatenate([[1, 0], np.arange(nlat), [nlat - 1, nlat - 2]])
    shift = np.concatenate([[nlon // 2] * 2, np.zeros(nlat, int), [nlon // 2] * 2])
    # interval e of thx (descending) with thx[e] >= th > thx[e+1], e in [1, nlat+1]
    e = np.searchsorted(-thx, -th, side="left") - 1
    e = np.clip(e, 1, nlat + 1)
    lat_nodes = np.stack([thx[e - 1 + r] for r in range(4)])
    wl = _lagrange4(lat_nodes, th)
    dl = 2.0 * np.pi / nlon
    x = lam / dl
    i = np.floor(x).astype(np.int64)
    t = x - i
    wk = _lagrange4(np.stack([np.full_like(t, -1.0), 0.0 * t, 1.0 + 0 * t, 2.0 + 0 * t]), t)
    out = 0.0
    for r in range(4):
        er = e - 1 + r
        row = rows[er]
        for c in range(4):
            col = np.mod(i - 1 + c + shift[er], nlon)
            out = out + wl[r] * wk[c] * f[..., row, col]
    return out


def departure_points(lat, nlon, Vn, Vx, dt, a, iters):
    """Departure points [3, nlat, nlon] (unit vectors) of the arrival grid.

    Vn, Vx: Cartesian velocity grids [3, nlat, nlon] at t_n and the
    extrapolated 2 V^n - V^{n-1}; eq. SETTLS_trajectories, ``iters`` times."""
    lam_a, th_a = np.meshgrid(2.0 * np.pi * np.arange(nlon) / nlon, lat)
    xa = cart(lam_a, th_a)
    xd = xa.copy()
    for _ in range(iters):
        lam, th = lonlat(xd)
        vd = interp(lat, nlon, Vx, lam, th)
        y = xa - (0.5 * dt / a) * (vd + Vn)
        xd = y / np.sqrt(np.sum(y * y, axis=0))
    return xd


def rotate_to(v, xd, xa):
    """Apply to vectors v [3, ...] the rotation taking unit vector xd to xa:
    v + w x v + (w (w.v) - |w|^2 v) / (1 + c), w = xd x xa, c = xd . xa."""
    w = np.cross(xd, xa, axis=0)
    c = np.sum(xd * xa, axis=0)
    wv = np.sum(w * v, axis=0)
    ww = np.sum(w * w, axis=0)
    return v + np.cross(w, v, axis=0) + (w * wv - ww * v) / (1.0 + c)


class SLStepper:
    """SL-SI-SETTLS steps of size dt on an ``oracle.swe.Model``."""

    def __init__(self, model, dt, nu=0.0, q=2, iters=2):
        self.model, self.dt, self.nu, self.q, self.iters = model, dt, nu, q, iters
        self._lu = {}

    def grid_fields(self, U):
        """Phi', delta, u, v, (1/(a cos)) dPhi'/dlambda, (1/a) dPhi'/dtheta on
        the Gauss grid."""
        md = self.model
        gr, a = md.grid, md.a
        Phi, xi, de = U
        Php = Phi.copy()
        Php[0] -= md.phibar
        cos = np.sqrt(gr.coslat2)[:, None]
        U_f, V_f = gr.uv_fourier_from_psichi(xi * gr.invlap, de * gr.invlap)
        ph = gr.synth(Php)
        d = gr.synth(de)
        u = gr.fourier_to_grid(U_f) / cos
        v = gr.fourier_to_grid(V_f) / cos
        gl = gr.synth(gr.im() * Php) / (a * cos)
        gt = gr.fourier_to_grid(gr.legendre_synth(Php, gr.H)) / (a * cos)
        return ph, d, u, v, gl, gt

    def _solve(self, rhs):
        """(I - dt/2 L) x = rhs per zonal wavenumber (dense LU)."""
        md = self.model
        out = np.zeros_like(rhs)
        for m in range(md.M + 1):
            if m not in self._lu:
                L = md.linear_matrix(m)
                self._lu[m] = scipy.linalg.lu_factor(np.eye(L.shape[0]) - 0.5 * self.dt * L)
            sl = m_slice(md.M, m)
            K = md.M - m + 1
            x = scipy.linalg.lu_solve(self._lu[m], np.concatenate([rhs[0, sl], rhs[1, sl],
                                                                   rhs[2, sl]]))
            out[0, sl], out[1, sl], out[2, sl] = x[:K], x[K:2 * K], x[2 * K:]
        return out

    def step(self, U, Uprev=None):
        """U^{n+1} from U^n and U^{n-1} (one-step variant when Uprev is None)."""
        md = self.model
        gr, a, dt = md.grid, md.a, self.dt
        nlat, nlon = gr.nlat, gr.nlon
        lat = np.arcsin(gr.mu)
        lam_a, th_a = np.meshgrid(gr.lam, lat)
        east, north = frames(lam_a, th_a)
        ph, d, u, v, gl, gt = self.grid_fields(U)
        if Uprev is None:
            php, dp, up, vp = ph, d, u, v
        else:
            php, dp, up, vp, _, _ = self.grid_fields(Uprev)
        f = 2.0 * md.omega * gr.mu[:, None]
        nr, nrp = -ph * d, -php * dp
        r_phi = ph + 0.5 * dt * (-md.phibar * d) + 0.5 * dt * (2.0 * nr - nrp)
        # -grad Phi' - f k x V, with k x (u, v) = (-v, u)
        ru = u + 0.5 * dt * (-gl + f * v)
        rv = v + 0.5 * dt * (-gt - f * u)
        Vn = u * east + v * north
        Vx = 2.0 * Vn - (up * east + vp * north)
        RV = ru * east + rv * north
        xd = departure_points(lat, nlon, Vn, Vx, dt, a, self.iters)
        lam_d, th_d = lonlat(xd)
        xa = np.stack([np.cos(th_a) * np.cos(lam_a), np.cos(th_a) * np.sin(lam_a),
                       np.sin(th_a)])
        phs = interp(lat, nlon, r_phi, lam_d, th_d) + 0.5 * dt * nr
        RVs = rotate_to(interp(lat, nlon, RV, lam_d, th_d), xd, xa)
        us = np.sum(RVs * east, axis=0)
        vs = np.sum(RVs * north, axis=0)
        cos = np.sqrt(gr.coslat2)[:, None]
        rhs = np.zeros_like(U)
        rhs[0] = gr.anal(phs)
        rhs[0][0] += md.phibar
        div, curl = gr.div_curl_from_fourier(gr.grid_to_fourier(us * cos),
                                             gr.grid_to_fourier(vs * cos))
        rhs[1], rhs[2] = curl, div
        rhs[1][0] = rhs[2][0] = 0.0
        assert nlat == lat.size
        return md.viscosity(self._solve(rhs), dt, self.nu, self.q)

    def propagate(self, U, nsteps, Uprev=None):
        """nsteps steps; the first one uses Uprev (one-step variant if None),
        the later ones the two-step scheme.  Returns (U^{n+nsteps}, U^{n+nsteps-1})."""
        prev = Uprev
        for _ in range(nsteps):
            U, prev = self.step(U, prev), U
        return U, prev
