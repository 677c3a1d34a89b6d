"""Oracle: Parareal and two-level MGRIT (paper Sec. 3).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Both drivers take propagators as plain callables, so the same code runs on
the SWE model and on a scalar test equation (Sec. 4.2).

Parareal (Sec. 3.1, eq. parareal_description):
    U^0_0 = U_0,  U^0_{n+1} = G(U^0_n)                       (serial coarse sweep)
    U^{k+1}_{n+1} = (G(U^{k+1}_n) - G(U^k_n)) + F(U^k_n)
The coarse difference is formed first, so that wherever U^{k+1}_n equals U^k_n
bitwise the update returns F(U^k_n) bitwise; slices n < k are already exact
and are not recomputed.  Converges to the serial fine solution in at most N
iterations (Sec. 3.1).

Two-level MGRIT with F(CF)^nu relaxation and FAS (Sec. 3.2):
    fine grid t_j = j dt_0 with one-step propagator Phi_0, C-points every m
    fine points, coarse propagator Phi_1 over one C-interval.
    1. relaxation: F-relaxation (Phi_0 from each C-point through its F-points),
       then nu times (C-relaxation: C-point <- Phi_0(last F-point before it);
       F-relaxation).
    2-4. residual at C-points r_i = Phi_0(u_{mi-1}) - u_{mi}, injection
       v_i = u_{mi}, coarse right-hand side g_i = r_i + v_i - Phi_1(v_{i-1}).
    5. serial coarse solve w_0 = v_0, w_i = Phi_1(w_{i-1}) + g_i.
    6. correction u_{mi} <- w_i (injection of the coarse error w - v).
Reading: with injection, r_i + v_i equals Phi_0(u_{mi-1}) exactly, so the
update is formed as w_i = (Phi_1(w_{i-1}) - Phi_1(v_{i-1})) + Phi_0(u_{mi-1}),
the same floating-point order as Parareal.  With nu = 0 the iteration is then
identical to Parareal with G = Phi_1 and F = Phi_0^m (Sec. 3.2.4).  Exact
convergence after at most N_1/(nu+1) iterations (Sec. 3.2.3).

Pins: tests/test_oracle_pint.py (Parareal stability function on the scalar
test equation, finite termination, MGRIT(2,0) = Parareal, MGRIT termination).
"""

import numpy as np


def parareal(u0, n_slices, fine, coarse, n_iter, record=False, incr_fn=None,
             tol=0.0):
    """Return (U, history) with U the slice-boundary states after n_iter
    iterations (or earlier stop when the increment <= tol > 0)."""
    N = n_slices
    U = [u0] + [None] * N
    G = [None] * N
    for n in range(N):
        G[n] = coarse(U[n])
        U[n + 1] = G[n]
    history = [list(U)] if record else None
    incrs = []
    for k in range(n_iter):
        if k >= N:
            break
        F = [None] * N
        for n in range(k, N):
            F[n] = fine(U[n])
        Unew = list(U)
        Gnew = list(G)
        for n in range(k, N):
            if n > k:
                Gnew[n] = coarse(Unew[n])
            # n == k: U^{k+1}_k = U^k_k, so G is unchanged bitwise
            Unew[n + 1] = (Gnew[n] - G[n]) + F[n]
        if incr_fn is not None:
            incrs.append(incr_fn(Unew, U))
        U, G = Unew, Gnew
        if record:
            history.append(list(U))
        if tol > 0 and incrs and incrs[-1] <= tol:
            break
    return U, (history, incrs)


def mgrit2(u0, n_coarse, m, phi0, phi1, nu, n_iter, record=False,
           incr_fn=None, tol=0.0):
    """Two-level MGRIT, F(CF)^nu relaxation.  Returns C-point states
    [u_0, u_m, ..., u_{m N_1}] after n_iter iterations."""
    N1 = n_coarse
    # iteration 0: serial coarse sweep for the C-points
    C = [u0] + [None] * N1
    for i in range(N1):
        C[i + 1] = phi1(C[i])
    history = [list(C)] if record else None
    incrs = []

    def f_relax(Cpts):
        """Returns, for each interval i = 0..N1-1, the last F-point
        u_{m(i+1)-1} propagated from C-point i."""
        last = [None] * N1
        for i in range(N1):
            u = Cpts[i]
            for _ in range(m - 1):
                u = phi0(u)
            last[i] = u
        return last

    for _ in range(n_iter):
        C_start = C
        last = f_relax(C)
        for _ in range(nu):
            # C-relaxation then F-relaxation
            C = [C[0]] + [phi0(last[i]) for i in range(N1)]
            last = f_relax(C)
        Fv = [phi0(last[i]) for i in range(N1)]        # Phi_0(u_{m(i+1)-1})
        Gv = [phi1(C[i]) for i in range(N1)]           # Phi_1(v_i)
        W = [C[0]] + [None] * N1
        for i in range(N1):
            Gw = Gv[i] if i == 0 else phi1(W[i])
            W[i + 1] = (Gw - Gv[i]) + Fv[i]
        if incr_fn is not None:
            incrs.append(incr_fn(W, C_start))
        C = W
        if record:
            history.append(list(C))
        if tol > 0 and incrs and incrs[-1] <= tol:
            break
    return C, (history, incrs)


def serial(u0, n, prop):
    out = [u0]
    for _ in range(n):
        out.append(prop(out[-1]))
    return out


def parareal_stability(n, k, R, F):
    """Closed form of the Parareal iterate on the scalar test equation
    (Sec. 4.2, eq. recurrence_parareal): sum_{i=0}^{k} C(n,i) (F-R)^i R^(n-i)."""
    from math import comb
    s = 0.0 + 0.0j
    for i in range(0, min(k, n) + 1):
        s += comb(n, i) * (F - R) ** i * R ** (n - i)
    return s
