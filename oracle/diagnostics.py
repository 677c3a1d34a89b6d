"""Oracle: the diagnostics of paper Sec. 5 and Sec. 5.1 -- kinetic-energy
spectrum, spectral max-norm errors per resolution, physical-space L2 errors.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

* ``ke_spectrum``: the kinetic-energy spectrum of a triangular truncation
  (Sec. 5.1, Gaussian bumps test case, after Koshyk and Hamilton),
      E(n) = 1/4 * a^2 / (n (n+1)) * sum_{m=-n..n} (|xi_{m,n}|^2 + |delta_{m,n}|^2),
  E(0) = 0.  The fields are real, so xi_{-m,n} = conj(xi_{m,n}) and the sum
  over m = -n..n is |.|_{0,n}^2 + 2 sum_{m=1..n} |.|_{m,n}^2.  With the
  normalisation of ``sht`` (Y_{m,n} has unit area mean square) the sum of
  E(n) over n is a quarter of the area mean of u^2 + v^2.
* ``spectral_errors``: E_{psi,R} of Sec. 5 (eq. error_definition) for
  psi = Phi', xi, delta and every R = 0..M: the largest modulus of the
  coefficient difference over 0 <= m <= n <= R divided by the largest
  reference modulus over the same modes.  Phi' = Phi - Phibar (reading
  R28: the geopotential perturbation, so the fixed mean does not swamp the
  reference norm).  A zero reference norm gives 0 for a zero difference and
  inf otherwise.  The paper uses 0 < R <= M; R = 0 (the mean alone) is
  included for completeness.
* ``grid_l2_errors``: E_{psi,L2} of Sec. 5 (unnumbered equation after
  error_definition), the root mean square of psi - psi_ref over the nodes
  of a grid divided by that of psi_ref, unweighted as printed.  Reading
  R28: the grid is the model's Gauss grid; psi = Phi', xi, delta.

Pins: tests/test_oracle_diagnostics.py -- the spectrum of solid-body
rotation in closed form, single harmonics with m = 0 and m > 0, the sum of
the spectrum against the Gauss-quadrature mean of the synthesised wind;
E_{psi,R} against hand-worked small cases; E_{psi,L2} against fields
evaluated in closed form on the grid nodes.
"""

import numpy as np

from .sht import idx


def ke_spectrum(U, M, a):
    """E(n), n = 0..M, of the state U = (Phi, xi, delta) (packed, complex)."""
    xi, de = U[1], U[2]
    E = np.zeros(M + 1)
    for n in range(1, M + 1):
        s = 0.0
        for m in range(0, n + 1):
            k = idx(M, m, n)
            v = abs(xi[k]) ** 2 + abs(de[k]) ** 2
            s += v if m == 0 else 2.0 * v
        E[n] = 0.25 * a * a / (n * (n + 1.0)) * s
    return E


def _perturbation(U, phibar):
    V = np.array(U, dtype=np.complex128, copy=True)
    V[0, 0] -= phibar
    return V


def spectral_errors(U, Ref, M, phibar):
    """E[f, R] for fields f = (Phi', xi, delta) and R = 0..M."""
    X = _perturbation(U, phibar)
    Y = _perturbation(Ref, phibar)
    out = np.zeros((3, M + 1))
    for f in range(3):
        for R in range(M + 1):
            num = 0.0
            den = 0.0
            for m in range(R + 1):
                for n in range(m, R + 1):
                    k = idx(M, m, n)
                    num = max(num, abs(X[f, k] - Y[f, k]))
                    den = max(den, abs(Y[f, k]))
            if den > 0.0:
                out[f, R] = num / den
            else:
                out[f, R] = 0.0 if num == 0.0 else np.inf
    return out


def grid_l2_errors(U, Ref, grid, phibar):
    """(E_Phi', E_xi, E_delta) in the physical-space L2 norm on ``grid`` (an
    ``sht.Grid``): sqrt(sum (psi - psi_ref)^2 / sum psi_ref^2) over its
    nodes (the 1 / (nlat nlon) of both means cancels)."""
    X = _perturbation(U, phibar)
    Y = _perturbation(Ref, phibar)
    out = np.zeros(3)
    for f in range(3):
        d = grid.synth(X[f] - Y[f])
        r = grid.synth(Y[f])
        num = np.sum(d * d)
        den = np.sum(r * r)
        out[f] = np.sqrt(num / den) if den > 0 else (0.0 if num == 0 else np.inf)
    return out
