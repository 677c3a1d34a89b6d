"""Oracle: stability functions of the time steppers, Parareal and two-level
MGRIT on the scalar test equation u' = (lambda_L + lambda_N) u (Sec. 4).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

xi_L = lambda_L dt and xi_N = lambda_N dt, complex.

* ``imex_amp``: IMEX (Sec. 4.1.1) = CN half step, Heun step, CN half step:
  ((4 + xi_L) / (4 - xi_L))^2 (1 + xi_N (2 + xi_N) / 2).  The printed explicit
  factor drops the leading 1 (reading R1: Heun keeps U*).
* ``settls_roots``: SL-SI-SETTLS (Sec. 4.1.2, eq. stability_SL_SI_SETTLS):
  the two roots A of
      (1 - xi_L/2) A^2 - (e^{-i ks} (1 + xi_L/2 + xi_N) + xi_N/2) A
          + (xi_N/2) e^{-i ks} = 0,
  ks = kappa s the phase of the departure-point shift.
* ``mgrit_stability``: two-level MGRIT with F(CF)^nu relaxation (Sec. 4.3):
  the iterate of the recurrence (eq. parareal_FCF_nrelax_B)
      u^k_n = R u^k_{n-1} + S u^{k-1}_{n-nu-1},  S = F^nu (F - R),
  u^k_0 = u_0, u^0_n = R^n u_0, terms with a negative slice index zero, is
      sum_{i=0}^{k} C(n - i nu, i) S^i R^(n - i(nu+1)) u_0
  (terms with n - i(nu+1) < 0 vanish).  nu = 0 is Parareal (eq.
  parareal_stability_function).  The printed upper limit floor(k/(nu+1))
  does not solve the printed recurrence for nu >= 1 (reading R32: the
  recurrence decides); F = A_f^{N_f}, R = A_c^{N_c}.
* ``stability_map``: max |A| over a grid of xi_N for a scheme alone, or for
  Parareal / MGRIT with an IMEX fine propagator and an IMEX or SL-SI-SETTLS
  coarse one.  xi_L and the grid's xi_N are taken on the coarse step
  dt_c = cfactor dt_f (reading R31): the fine propagator takes
  N_f = cfactor N_c steps at xi / cfactor.  For SL-SI-SETTLS the map is the
  maximum over both roots and over ks = 2 pi j / n_ks, j = 0..n_ks (the
  stability region is the intersection over roots and phases).

Pins: tests/test_oracle_stability.py -- the IMEX factor against the steps of
the scheme on the scalar equation; the SETTLS roots against the growth of
the two-step scheme run on a Fourier mode with exact shifts, and the
Crank-Nicolson limit; the MGRIT function against brute-force iteration of
the recurrence and, at nu = 0, against the Parareal iteration; Parareal at
k = n against the fine propagator alone.
"""

import cmath
from math import comb


def imex_amp(xl, xn):
    ai = (4.0 + xl) / (4.0 - xl)
    return ai * ai * (1.0 + xn * (2.0 + xn) / 2.0)


def settls_roots(xl, xn, ks):
    e = cmath.exp(-1j * ks)
    a = 1.0 - xl / 2.0
    b = -(e * (1.0 + xl / 2.0 + xn) + xn / 2.0)
    c = xn / 2.0 * e
    d = cmath.sqrt(b * b - 4.0 * a * c)
    return ((-b + d) / (2.0 * a), (-b - d) / (2.0 * a))


def mgrit_stability(n, k, F, R, nu):
    S = F ** nu * (F - R)
    s = 0.0 + 0.0j
    for i in range(0, k + 1):
        if n - i * (nu + 1) < 0:
            break
        s += comb(n - i * nu, i) * S ** i * R ** (n - i * (nu + 1))
    return s


def _coarse_amps(coarse, xl, xn, n_ks):
    if coarse == "imex":
        return [imex_amp(xl, xn)]
    out = []
    for j in range(n_ks + 1):
        out.extend(settls_roots(xl, xn, 2.0 * cmath.pi * j / n_ks))
    return out


def stability_map(kind, coarse, xl, re, im, n=100, k=5, cfactor=2, n_c=1, nu=0, n_ks=20):
    """max |A| on the grid xi_N = re[j] + i im[i] (rows over im).
    kind: "scheme" (the coarse scheme alone, one step), "mgrit" (nu = 0:
    Parareal)."""
    out = [[0.0] * len(re) for _ in im]
    for r, y in enumerate(im):
        for c, x in enumerate(re):
            xn = complex(x, y)
            amps = _coarse_amps(coarse, xl, xn, n_ks)
            if kind == "scheme":
                out[r][c] = max(abs(a) for a in amps)
                continue
            F = imex_amp(xl / cfactor, xn / cfactor) ** (cfactor * n_c)
            out[r][c] = max(abs(mgrit_stability(n, k, F, a ** n_c, nu)) for a in amps)
    return out
