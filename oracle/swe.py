"""Oracle: rotating shallow-water operators and the IMEX step (paper Sec. 2).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

State U = (Phi, xi, delta) as three packed spectral arrays (complex128), Phi
stored in full (its (0,0) coefficient is the global mean); Phi' = Phi - Phibar
where Phibar is a fixed run parameter (Sec. 2.1, eq. swe_sphere).

* L = L_G + L_C (linear gravity and Coriolis, Sec. 2.1).  Implemented as the
  Galerkin projection onto the truncation: the operators "multiply by mu" and
  "(1-mu^2) d/dmu" are built, per zonal wavenumber m, as dense matrices by exact
  Gauss quadrature of Pbar_n * (mu Pbar_n') and Pbar_n * Hbar_n'.  Coriolis
  uses div(fV) = f delta + (2 Omega / a) V and k.curl(fV) = f xi - (2 Omega / a) U
  with f = 2 Omega mu, U = u cos(lat), V = v cos(lat).
* N = N_A + N_R (nonlinear advection and rest, Sec. 2.1), pseudospectral on the
  Gauss grid (Sec. 2.2): velocities and gradients synthesised with Pbar and
  Hbar tables, products formed pointwise, then
      N_Phi   = analysis( -(U dPhi'/dlambda + V (1-mu^2) dPhi'/dmu)/(a c^2) - Phi' delta )
      N_xi    = -div(xi u, xi v)
      N_delta = curl(xi u, xi v) + n(n+1)/a^2 * analysis((U^2+V^2)/(2 c^2))
  with c^2 = 1 - mu^2.  The (0,0) coefficients of N_xi and N_delta are set to
  their exact value 0 (global mean of a divergence / curl).
* CN half step (eq. IMEX_implicit): solve (I - dt/4 L) x = (I + dt/4 L) y with
  a dense LU per zonal wavenumber (scipy.linalg.lu_factor).
* Explicit step (eq. IMEX_explicit) read as Heun's RK2:
      U** = U* + 1/2 (dt N(U*) + dt N(U* + dt N(U*))).
  The printed form omits the U* term; the paper's own amplification factor
  analysis (Sec. 4.1.1) only makes sense with it (a zero nonlinear term must
  give the identity).  Pinned by second-order convergence in time.
* Viscosity (App. A): backward Euler at the end of every step, each mode
  divided by 1 + dt nu (n(n+1)/a^2)^(q/2); applied to Phi', xi, delta (the
  (0,0) mode has factor 1).
* IMEX step (eq. IMEX): U^{n+1} = D_nu F_I^{dt/2}(F_E^{dt}(F_I^{dt/2}(U^n))).

The ``terms`` bit mask (LG=1, LC=2, NL=4, VISC=8) switches operators off for
tests only.

Pins: tests/test_oracle_swe.py (Laplacian/velocity closed forms, advection by
solid-body rotation, steady balanced flow, CN energy conservation and
amplification factor, viscosity factor, mass, alias-free tendencies, 2nd order
in time).
"""

import numpy as np
import scipy.linalg

from .sht import Grid, m_slice, idx

T_LG, T_LC, T_NL, T_VISC = 1, 2, 4, 8
T_ALL = 15


class Model:
    """Planet constants, grid and operators for one truncation."""

    def __init__(self, M, nlon, nlat, a=6.37122e6, omega=7.292e-5, g=9.80616,
                 phibar=2.94e4, extended=False):
        """``extended`` evaluates the tendencies in x87 extended precision; it
        only serves to measure the rounding floor of the float64 path."""
        self.grid = Grid(M, nlon, nlat, a, extended=extended)
        rdt = self.grid.rdt
        self.M, self.a, self.omega, self.g = M, rdt(a), rdt(omega), rdt(g)
        self.phibar = rdt(phibar)
        self._galerkin = None
        self._lu_cache = {}

    # ------------------------------------------------------------------
    # nonlinear tendencies N(U)
    # ------------------------------------------------------------------
    def tendencies(self, U):
        gr, a = self.grid, self.a
        Phi, xi, de = U
        Php = Phi.copy()
        Php[0] -= self.phibar                      # Phi' = Phi - Phibar
        psi = xi * gr.invlap                       # xi = lap psi
        chi = de * gr.invlap                       # delta = lap chi
        imf = gr.im()
        # Fourier coefficients on the Gauss latitudes
        xi_f = gr.legendre_synth(xi)
        de_f = gr.legendre_synth(de)
        ph_f = gr.legendre_synth(Php)
        phl_f = gr.legendre_synth(imf * Php)       # dPhi'/dlambda
        phg_f = gr.legendre_synth(Php, gr.H)       # (1-mu^2) dPhi'/dmu
        U_f, V_f = gr.uv_fourier_from_psichi(psi, chi)
        # grid point values
        xi_g, de_g, ph_g, phl_g, phg_g, Ug, Vg = (
            gr.fourier_to_grid(f) for f in (xi_f, de_f, ph_f, phl_f, phg_f, U_f, V_f))
        c2 = gr.coslat2[:, None]
        nphi_g = -(Ug * phl_g + Vg * phg_g) / (a * c2) - ph_g * de_g
        A_g = xi_g * Ug                           # (xi u) cos(lat)
        B_g = xi_g * Vg                           # (xi v) cos(lat)
        K_g = (Ug * Ug + Vg * Vg) / (2.0 * c2)    # kinetic energy V.V/2
        n_phi = gr.anal(nphi_g)
        K = gr.anal(K_g)
        div, curl = gr.div_curl_from_fourier(gr.grid_to_fourier(A_g),
                                             gr.grid_to_fourier(B_g))
        n_xi = -div
        n_de = curl - gr.lap * K                   # -lap(K) = n(n+1)/a^2 K
        n_xi[0] = 0.0
        n_de[0] = 0.0
        return np.stack([n_phi, n_xi, n_de])

    # ------------------------------------------------------------------
    # linear operator L = L_G + L_C, Galerkin projection per m
    # ------------------------------------------------------------------
    def _galerkin_mats(self):
        """Per m: (Mmu, D) with Mmu[n,n'] = 1/2 sum_j w_j Pbar_n mu Pbar_n' and
        D[n,n'] = 1/2 sum_j w_j Pbar_n Hbar_n' for n, n' in [m, M]."""
        if self._galerkin is None:
            gr = self.grid
            mats = []
            for m in range(self.M + 1):
                K = self.M - m + 1
                P = gr.P[m][:K]
                H = gr.H[m][:K]
                Mmu = 0.5 * (P * (gr.w * gr.mu)) @ P.T
                D = 0.5 * (P * gr.w) @ H.T
                mats.append((Mmu, D))
            self._galerkin = mats
        return self._galerkin

    def linear_matrix(self, m, terms=T_ALL):
        """Dense matrix of L restricted to zonal wavenumber m, acting on the
        stacked vector (Phi_n, xi_n, delta_n), n = m..M."""
        gr, a = self.grid, self.a
        K = self.M - m + 1
        n = np.arange(m, self.M + 1, dtype=np.float64)
        lap = -n * (n + 1.0) / a ** 2
        inv = np.where(n > 0, 1.0 / np.where(n > 0, lap, 1.0), 0.0)
        Mmu, D = self._galerkin_mats()[m]
        Z = np.zeros((K, K), dtype=np.complex128)
        I = np.eye(K)
        L = np.zeros((3 * K, 3 * K), dtype=np.complex128)
        if terms & T_LG:
            L[0:K, 2 * K:3 * K] += -self.phibar * I            # -Phibar delta
            L[2 * K:3 * K, 0:K] += -np.diag(lap)                # -lap Phi
        if terms & T_LC:
            two_om = 2.0 * self.omega
            Ipsi = np.diag(inv).astype(np.complex128)           # psi = inv * xi
            im = 1j * m
            # V = (1/a)[ i m psi + D chi ],  U = (1/a)[ i m chi - D psi ]
            V_xi = (im * Ipsi) / a
            V_de = (D @ Ipsi) / a
            U_xi = -(D @ Ipsi) / a
            U_de = (im * Ipsi) / a
            # xi row: -div(f V) = -(f delta + 2 Omega/a V)
            L[K:2 * K, 2 * K:3 * K] += -two_om * Mmu - (two_om / a) * V_de
            L[K:2 * K, K:2 * K] += -(two_om / a) * V_xi
            # delta row: k.curl(f V) = f xi - 2 Omega/a U
            L[2 * K:3 * K, K:2 * K] += two_om * Mmu - (two_om / a) * U_xi
            L[2 * K:3 * K, 2 * K:3 * K] += -(two_om / a) * U_de
        del Z
        return L

    def apply_linear(self, U, terms=T_ALL):
        out = np.zeros_like(U)
        for m in range(self.M + 1):
            sl = m_slice(self.M, m)
            v = np.concatenate([U[0, sl], U[1, sl], U[2, sl]])
            r = self.linear_matrix(m, terms) @ v
            K = self.M - m + 1
            out[0, sl], out[1, sl], out[2, sl] = r[:K], r[K:2 * K], r[2 * K:]
        return out

    def cn_half(self, U, dt, terms=T_ALL, ms=None):
        """Crank-Nicolson half step: (I - dt/4 L) x = (I + dt/4 L) U.

        ``ms`` restricts the solve to the listed zonal wavenumbers (the
        others are left zero), for sampled checks at large M."""
        alpha = self.grid.rdt(dt) / 4
        key = (float(alpha), terms & (T_LG | T_LC))
        ms = range(self.M + 1) if ms is None else ms
        facs = self._lu_cache.setdefault(key, {})
        out = np.zeros_like(U)
        ext = self.grid.rdt is not np.float64
        for m in ms:
            if m not in facs:
                L = self.linear_matrix(m, terms)
                Id = np.eye(L.shape[0], dtype=self.grid.rdt)
                lhs = Id - alpha * L
                facs[m] = (Id + alpha * L, scipy.linalg.lu_factor(lhs.astype(np.complex128)),
                           lhs if ext else None)
            sl = m_slice(self.M, m)
            K = self.M - m + 1
            v = np.concatenate([U[0, sl], U[1, sl], U[2, sl]])
            rhs_mat, lu, lhs = facs[m]
            rhs = rhs_mat @ v
            x = scipy.linalg.lu_solve(lu, rhs.astype(np.complex128)).astype(out.dtype)
            if ext:
                # Extended precision: the float64 LU solution refined with
                # residuals formed in extended precision.  I - alpha L has
                # Hermitian part I in energy-scaled variables (well
                # conditioned), so each pass gains about 16 digits.
                for _ in range(2):
                    r = rhs - lhs @ x
                    x = x + scipy.linalg.lu_solve(lu, r.astype(np.complex128)).astype(out.dtype)
            out[0, sl], out[1, sl], out[2, sl] = x[:K], x[K:2 * K], x[2 * K:]
        return out

    # ------------------------------------------------------------------
    # viscosity and the full step
    # ------------------------------------------------------------------
    def viscosity(self, U, dt, nu, q):
        """Backward Euler for d psi/dt = (-1)^(q/2+1) nu lap^(q/2) psi."""
        if nu == 0.0:
            return U.copy()
        nn = self.grid.n_of.astype(np.float64)
        fac = 1.0 / (1.0 + dt * nu * (nn * (nn + 1.0) / self.a ** 2) ** (q // 2))
        return U * fac[None, :]

    def explicit_rk2(self, U, dt, terms=T_ALL):
        if not terms & T_NL:
            return U.copy()
        n1 = self.tendencies(U)
        n2 = self.tendencies(U + dt * n1)
        return U + 0.5 * dt * (n1 + n2)

    def imex_step(self, U, dt, nu=0.0, q=2, terms=T_ALL):
        Ua = self.cn_half(U, dt, terms) if terms & (T_LG | T_LC) else U.copy()
        Uc = self.explicit_rk2(Ua, dt, terms)
        Ud = self.cn_half(Uc, dt, terms) if terms & (T_LG | T_LC) else Uc
        if terms & T_VISC:
            Ud = self.viscosity(Ud, dt, nu, q)
        return Ud

    def propagate(self, U, dt, nsteps, nu=0.0, q=2, terms=T_ALL):
        for _ in range(nsteps):
            U = self.imex_step(U, dt, nu, q, terms)
        return U


def packed_index(M, m, n):
    return idx(M, m, n)
