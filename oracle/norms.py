"""Oracle: norms used for parity, stopping and error reporting (paper Sec. 5).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

* ``spectral_norm``: ||x||^2 = sum_n |x_{0,n}|^2 + 2 sum_{m>=1,n} |x_{m,n}|^2,
  which by Parseval equals the area-weighted mean of x^2 over the sphere.  For
  Phi the (0,0) coefficient is excluded (the norm is taken of Phi').
  Pinned against the grid quadrature of x^2 in tests.
* ``rel_err``: per field ||a - b|| / ||b|| (parity metric).
* ``max_increment``: stopping test, max over slices of the relative change
  ||U^{k+1}_n - U^k_n|| / ||U^{k+1}_n|| of Phi' and of the wind.
* ``wind_norm`` / ``state_rel_err``: the velocity field induced by vorticity
  and divergence, |V|^2 averaged over the sphere = sum_{n>=1} w_m a^2/(n(n+1))
  (|xi_{m,n}|^2 + |delta_{m,n}|^2) (Parseval with xi = lap psi, delta =
  lap chi).  ``state_rel_err`` returns the relative L2 error of Phi' and of
  the wind.  Divergence of a nearly balanced flow is a small residual of
  cancelling terms, and the Laplacian of the kinetic energy in its tendency
  multiplies FP64 rounding by n(n+1); in the plain spectral norm its
  float64 rounding floor (this oracle against itself in extended precision)
  reaches ~3e-12 at T127 and ~1.5e-11 at T255 for one tendency evaluation
  of a balanced jet, in the wind norm 1.5-4e-13.  Pinned
  against the grid quadrature of u^2 + v^2 in tests.
* The paper's E_{psi,R} (Sec. 5, eq. error_definition) is in
  ``oracle/diagnostics.py`` with its pins.
"""

import numpy as np


def _weights(M, exclude_mean):
    w = np.empty((M + 1) * (M + 2) // 2)
    k = 0
    for m in range(M + 1):
        K = M - m + 1
        w[k:k + K] = 1.0 if m == 0 else 2.0
        k += K
    if exclude_mean:
        w[0] = 0.0
    return w


def spectral_norm(x, M, exclude_mean=False):
    w = _weights(M, exclude_mean)
    return float(np.sqrt(np.sum(w * np.abs(x) ** 2)))


def field_norms(U, M):
    """Norms of (Phi', xi, delta) for a state U[3, ncoef]."""
    return np.array([spectral_norm(U[0], M, True), spectral_norm(U[1], M),
                     spectral_norm(U[2], M)])


def wind_norm(xi, de, M, a):
    w = _weights(M, True)
    n = np.concatenate([np.arange(m, M + 1) for m in range(M + 1)]).astype(np.float64)
    k = np.zeros_like(n)
    k[n > 0] = a * a / (n[n > 0] * (n[n > 0] + 1.0))
    return float(np.sqrt(np.sum(w * k * (np.abs(xi) ** 2 + np.abs(de) ** 2))))


def state_rel_err(A, B, M, a=6.37122e6):
    """(relative L2 error of Phi', relative L2 error of the wind) of A vs B."""
    d = A - B
    ph = spectral_norm(d[0], M, True) / max(spectral_norm(B[0], M, True), 1e-300)
    wn = wind_norm(B[1], B[2], M, a)
    wd = wind_norm(d[1], d[2], M, a)
    return np.array([ph, wd / wn if wn > 0 else wd])


def rel_err(A, B, M):
    """Per-field relative L2 error of A against reference B."""
    d = field_norms(A - B, M)
    r = field_norms(B, M)
    return d / np.where(r > 0, r, 1.0)


def max_increment(new, old, M, a=6.37122e6):
    """max over slices n >= 1 of the relative change of Phi' and of the wind,
    ||new_n - old_n|| / ||new_n||."""
    worst = 0.0
    for n in range(1, len(new)):
        worst = max(worst, float(np.max(state_rel_err(old[n], new[n], M, a))))
    return worst
