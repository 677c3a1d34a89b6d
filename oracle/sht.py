"""Oracle: spherical-harmonic transform on a Gauss grid (paper Sec. 2.2).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Conventions (the paper fixes none; this is the reading the whole project uses):

* Y_{m,n}(lambda, mu) = Pbar_n^m(mu) exp(i m lambda), mu = sin(latitude).
  Pbar is normalised so that 1/2 * int_{-1}^{1} Pbar^2 dmu = 1, without the
  Condon-Shortley phase.  The (0,0) coefficient is therefore the area mean.
* Real fields store m >= 0 only; psi_{-m,n} = conj(psi_{m,n}).
* Triangular truncation M (Sec. 2.2): 0 <= m <= n <= M.  Coefficients are stored
  m-major, idx(m, n) = m(2M+3-m)/2 + (n-m).
* Grid: lambda_k = 2 pi k / nlon, k = 0..nlon-1; latitudes are the Gauss-Legendre
  nodes ordered north to south (mu descending), weights w_j sum to 2.

Transforms (Sec. 2.2: FFT in longitude, Legendre transform in latitude):

* synthesis:  s(lambda_k, mu_j) = sum_{|m|<=M} s_m(mu_j) exp(i m lambda_k),
              s_m(mu) = sum_n s_{m,n} Pbar_n^m(mu)
* analysis:   s_m(mu_j) = 1/nlon sum_k s(lambda_k, mu_j) exp(-i m lambda_k),
              s_{m,n} = 1/2 sum_j w_j Pbar_n^m(mu_j) s_m(mu_j)

Derivative tables: Hbar_n^m(mu) := (1-mu^2) dPbar_n^m/dmu, evaluated with the
textbook identity (1-mu^2) P'_n = -n mu P_n + (2n+1) eps_n P_{n-1}, with
eps_n^m = sqrt((n^2-m^2)/(4n^2-1)).

Pins (tests/test_oracle_sht.py): Gauss nodes vs closed-form moments; Pbar vs
scipy's associated Legendre functions and discrete orthonormality; Hbar vs an
independent finite-difference derivative; analysis(synthesis) = identity; FFT
vs direct DFT; div(grad psi) and curl(k x grad psi) = Laplacian eigenvalue.
"""

import numpy as np


def ncoef(M):
    """Number of (m, n) pairs with 0 <= m <= n <= M."""
    return (M + 1) * (M + 2) // 2


def idx(M, m, n):
    """Position of coefficient (m, n) in the m-major packed layout."""
    return m * (2 * M + 3 - m) // 2 + (n - m)


def m_slice(M, m):
    """Slice of the packed array holding n = m..M for one zonal wavenumber m."""
    s = idx(M, m, m)
    return slice(s, s + (M - m + 1))


def truncate(c, M, Mc):
    """Spectral restriction (spatial coarsening of a coarse level): the
    coefficients (m, n) with n <= Mc of a truncation-M state, in the
    truncation-Mc packing.  c: (..., ncoef(M)) -> (..., ncoef(Mc))."""
    c = np.asarray(c)
    out = np.zeros(c.shape[:-1] + (ncoef(Mc),), dtype=c.dtype)
    for m in range(Mc + 1):
        for n in range(m, Mc + 1):
            out[..., idx(Mc, m, n)] = c[..., idx(M, m, n)]
    return out


def pad(c, Mc, M):
    """Spectral prolongation: a truncation-Mc state in the truncation-M packing
    with zero coefficients for n > Mc."""
    c = np.asarray(c)
    out = np.zeros(c.shape[:-1] + (ncoef(M),), dtype=c.dtype)
    for m in range(Mc + 1):
        for n in range(m, Mc + 1):
            out[..., idx(M, m, n)] = c[..., idx(Mc, m, n)]
    return out


def eps(m, n, dtype=np.float64):
    """eps_n^m = sqrt((n^2 - m^2) / (4 n^2 - 1)); zero for n <= m."""
    n = np.asarray(n, dtype=dtype)
    val = (n * n - m * m) / (4.0 * n * n - 1.0)
    return np.sqrt(np.where(n > m, val, 0.0))


def _legendre_pair(n, x):
    """P_n(x) and P_{n-1}(x) (unnormalised) by the three-term recurrence."""
    p0 = np.ones_like(x)
    p1 = x.copy()
    for k in range(2, n + 1):
        p0, p1 = p1, ((2 * k - 1) * x * p1 - (k - 1) * p0) / k
    return p1, p0


def gauss_nodes(nlat, with_coslat2=False, extended=False):
    """Gauss-Legendre nodes mu_j (north to south) and weights w_j (sum 2).

    Starts from numpy's ``leggauss`` nodes, polishes them with Newton steps on
    P_nlat in x87 extended precision and evaluates the weights there with
    w = 2 / ((1 - x^2) P'_nlat(x)^2).  (numpy's own weights lose about three
    digits at nlat = 384.)  With ``with_coslat2`` also returns 1 - mu^2,
    formed in extended precision (in float64 it cancels near the poles).
    ``extended`` returns x87 extended-precision arrays (used only to
    calibrate the rounding floor of the float64 path).
    """
    x0, _ = np.polynomial.legendre.leggauss(nlat)
    x = x0.astype(np.longdouble)
    for _ in range(3):
        pn, pn1 = _legendre_pair(nlat, x)
        dp = nlat * (x * pn - pn1) / (x * x - 1)
        x = x - pn / dp
    pn, pn1 = _legendre_pair(nlat, x)
    dp = nlat * (x * pn - pn1) / (x * x - 1)
    w = 2 / ((1 - x * x) * dp * dp)
    dt = np.longdouble if extended else np.float64
    mu, w = x[::-1].astype(dt), w[::-1].astype(dt)
    if with_coslat2:
        return mu, w, (1 - x * x)[::-1].astype(dt)
    return mu, w


def pbar_table(nmax, mu, coslat2=None):
    """Normalised associated Legendre functions.

    Returns a list P with P[m] of shape (nmax-m+1, nlat): rows n = m..nmax.
    Recurrences: Pbar_0^0 = 1; Pbar_m^m = sqrt((2m+1)/(2m)) sqrt(1-mu^2)
    Pbar_{m-1}^{m-1}; Pbar_{m+1}^m = sqrt(2m+3) mu Pbar_m^m; and the three-term
    recurrence mu Pbar_n = eps_{n+1} Pbar_{n+1} + eps_n Pbar_{n-1} solved for
    Pbar_{n+1}.
    """
    mu = np.asarray(mu)
    if mu.dtype != np.longdouble:
        mu = mu.astype(np.float64)
    s = np.sqrt(1.0 - mu * mu if coslat2 is None else coslat2)
    out = []
    pmm = np.ones_like(mu)
    for m in range(nmax + 1):
        if m > 0:
            pmm = np.sqrt(mu.dtype.type(2 * m + 1) / mu.dtype.type(2 * m)) * s * pmm
        rows = np.zeros((nmax - m + 1, mu.size), dtype=mu.dtype)
        rows[0] = pmm
        if m + 1 <= nmax:
            rows[1] = np.sqrt(mu.dtype.type(2 * m + 3)) * mu * pmm
        for n in range(m + 2, nmax + 1):
            rows[n - m] = (mu * rows[n - m - 1]
                           - eps(m, n - 1, mu.dtype) * rows[n - m - 2]) / eps(m, n, mu.dtype)
        out.append(rows)
    return out


def hbar_table(P, mu, nmax):
    """Hbar_n^m = (1-mu^2) dPbar_n^m/dmu for n = m..nmax-1 (needs P to nmax-1).

    Uses (1-mu^2) P'_n = -n mu P_n + (2n+1) eps_n P_{n-1}.
    """
    out = []
    for m in range(nmax):
        rows = np.zeros((nmax - m, mu.size), dtype=mu.dtype)
        for n in range(m, nmax):
            h = -n * mu * P[m][n - m]
            if n > m:
                h = h + (2 * n + 1) * eps(m, n, mu.dtype) * P[m][n - m - 1]
            rows[n - m] = h
        out.append(rows)
    return out


class Grid:
    """Gauss grid plus Legendre tables for truncation M (Sec. 2.2)."""

    def __init__(self, M, nlon, nlat, a=6.37122e6, extended=False):
        if nlat < M + 1 or nlon < 2 * M + 1:
            raise ValueError("grid too small for truncation M")
        self.rdt = np.longdouble if extended else np.float64
        self.cdt = np.clongdouble if extended else np.complex128
        self.M, self.nlon, self.nlat = M, nlon, nlat
        self.a = self.rdt(a)
        self.mu, self.w, self.coslat2 = gauss_nodes(nlat, with_coslat2=True, extended=extended)
        self.lam = 2.0 * np.pi * np.arange(nlon) / nlon
        # Pbar for n <= M+1 (the vector transforms need one extra degree)
        self.P = pbar_table(M + 1, self.mu, self.coslat2)
        self.H = hbar_table(self.P, self.mu, M + 1)   # n = m..M
        self.nc = ncoef(M)
        self.n_of = np.zeros(self.nc, dtype=np.int64)
        self.m_of = np.zeros(self.nc, dtype=np.int64)
        for m in range(M + 1):
            sl = m_slice(M, m)
            self.m_of[sl] = m
            self.n_of[sl] = np.arange(m, M + 1)
        nn = self.n_of.astype(self.rdt)
        self.lap = -nn * (nn + 1.0) / self.a ** 2          # Laplacian eigenvalue
        self.invlap = np.zeros(self.nc, dtype=self.rdt)
        self.invlap[nn > 0] = 1.0 / self.lap[nn > 0]

    # ---- Fourier (longitude) part -------------------------------------
    def fourier_to_grid(self, fhat):
        """fhat[..., j, m] (m = 0..M) -> real grid [..., j, k]."""
        spec = np.zeros(fhat.shape[:-1] + (self.nlon // 2 + 1,), dtype=self.cdt)
        spec[..., :self.M + 1] = fhat
        return self.nlon * np.fft.irfft(spec, n=self.nlon, axis=-1)

    def grid_to_fourier(self, g):
        """real grid [..., j, k] -> fhat[..., j, m], m = 0..M."""
        return np.fft.rfft(g, axis=-1)[..., :self.M + 1] / self.nlon

    # ---- Legendre (latitude) part -------------------------------------
    def legendre_synth(self, c, table=None):
        """packed coefficients c[ncoef] -> Fourier coefficients [nlat, M+1]."""
        table = self.P if table is None else table
        out = np.zeros((self.nlat, self.M + 1), dtype=self.cdt)
        for m in range(self.M + 1):
            K = self.M - m + 1
            out[:, m] = c[m_slice(self.M, m)] @ table[m][:K]
        return out

    def legendre_anal(self, fhat, weight=None, table=None):
        """Fourier coefficients [nlat, M+1] -> packed coefficients, with
        s_{m,n} = 1/2 sum_j wq_j T_n^m(mu_j) fhat_m(mu_j), wq = w (default)."""
        table = self.P if table is None else table
        wq = self.w if weight is None else weight
        out = np.zeros(self.nc, dtype=self.cdt)
        for m in range(self.M + 1):
            K = self.M - m + 1
            out[m_slice(self.M, m)] = 0.5 * (table[m][:K] @ (wq * fhat[:, m]))
        return out

    # ---- full scalar transforms ---------------------------------------
    def synth(self, c):
        return self.fourier_to_grid(self.legendre_synth(c))

    def anal(self, g):
        return self.legendre_anal(self.grid_to_fourier(g))

    def im(self):
        """i*m for every packed coefficient (longitude derivative)."""
        return 1j * self.m_of.astype(self.rdt)

    # ---- vector transforms (integration by parts in mu) ----------------
    def div_curl_from_fourier(self, A_hat, B_hat):
        """Spectral divergence and curl of the vector (p, q) given the Fourier
        coefficients of A = p cos(lat), B = q cos(lat) on the Gauss latitudes:

        div_{m,n}  = 1/(2a) sum_j w_j/(1-mu_j^2) [ i m A_m Pbar_n - B_m Hbar_n ]
        curl_{m,n} = 1/(2a) sum_j w_j/(1-mu_j^2) [ i m B_m Pbar_n + A_m Hbar_n ]
        """
        wq = self.w / self.coslat2
        div = np.zeros(self.nc, dtype=self.cdt)
        curl = np.zeros(self.nc, dtype=self.cdt)
        for m in range(self.M + 1):
            K = self.M - m + 1
            P = self.P[m][:K]
            H = self.H[m][:K]
            a_m = wq * A_hat[:, m]
            b_m = wq * B_hat[:, m]
            div[m_slice(self.M, m)] = (1j * m * (P @ a_m) - H @ b_m) / (2.0 * self.a)
            curl[m_slice(self.M, m)] = (1j * m * (P @ b_m) + H @ a_m) / (2.0 * self.a)
        return div, curl

    def uv_fourier_from_psichi(self, psi, chi):
        """Fourier coefficients of U = u cos(lat), V = v cos(lat) from
        streamfunction psi and velocity potential chi:
        U = (1/a)[d(chi)/dlambda - (1-mu^2) d(psi)/dmu],
        V = (1/a)[d(psi)/dlambda + (1-mu^2) d(chi)/dmu]."""
        imf = self.im()
        U = (self.legendre_synth(imf * chi) - self.legendre_synth(psi, self.H)) / self.a
        V = (self.legendre_synth(imf * psi) + self.legendre_synth(chi, self.H)) / self.a
        return U, V
