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

Parareal with a two-step coarse scheme (SL-SI-SETTLS, Sec. 2.3.2) follows
the rule of Sec. 3.2.4 for the coarsest level: the two-step scheme runs in
every step of the serial sweep, the one-step variant only where two
consecutive steps belong to different processors -- which never happens in
a sweep on one device.  Reading: the coarse propagator maps (U_n, P_{n-1})
to (G_n, P_n), P_n being the last state before the end of its run, and the
sweep hands P_{n-1} of the slice before to the coarse run of slice n (the
solution at t_{n-1} carried with the one at t_n).  The very first step of
the run has no history and takes the one-step variant.  Slice k's G and P
are unchanged in iteration k (its input and the carried state are those of
the previous sweep), so they are kept, as in the one-step case.

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

Three-level MGRIT (Sec. 3.2, multilevel recursion): the two-level iteration
with step 5 replaced by `cycles` two-level iterations of the level-1 problem
on levels (1, 2).  The level-1 problem is w_0 = v_0,
    w_i = psi_i(w_{i-1}) = (Phi_1(w_{i-1}) - Phi_1(v_{i-1})) + Phi_0(u_{mi-1}),
i.e. Phi_1 plus the FAS forcing, with initial guess v.  Its level-2 points
are every m1-th level-1 point; Phi_2 spans m1 level-1 intervals.  One
iteration on levels (1, 2): F(CF)^nu relaxation with psi; level-2 FAS with
F2_j = psi_{m1 j}(w_{m1 j - 1}), v2_j = w_{m1 j}; serial level-2 solve
z_0 = v2_0, z_j = (Phi_2(z_{j-1}) - Phi_2(v2_{j-1})) + F2_j; w_{m1 j} <- z_j;
F-relaxation with psi.  Then u_{mi} <- w_i for every level-1 point.  The
paper runs F-cycles followed by one post-V-cycle (Sec. 3.2, deferring the
definition to XBraid); reading: `cycles` = 1 is a V-cycle, 2 adds the post
cycle.  Every update keeps the difference-first order, so an exact prefix
stays bitwise exact and the finite termination bound of the two-level
iteration holds.

Pins: tests/test_oracle_pint.py (Parareal stability function on the scalar
test equation, finite termination, MGRIT(2,0) = Parareal, MGRIT termination;
carried two-step coarse scheme: the first sweep is the uninterrupted serial
two-step run, a coarse scheme ignoring its carried state gives Parareal,
finite termination;
three-level: one level-2 interval = two-level bitwise, exact level-2
propagator on a linear problem = two-level, finite termination).
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


def parareal_carry(u0, n_slices, fine, coarse, n_iter, record=False):
    """Parareal whose coarse propagator carries its previous state across
    slices: coarse(U, P) -> (G, P'), P = None for the first slice of the
    horizon.  Returns (U, history) as ``parareal``."""
    N = n_slices
    U = [u0] + [None] * N
    G = [None] * N
    P = [None] * N
    prev = None
    for n in range(N):
        G[n], P[n] = coarse(U[n], prev)
        U[n + 1] = G[n]
        prev = P[n]
    history = [list(U)] if record else None
    for k in range(n_iter):
        if k >= N:
            break
        F = [None] * N
        for n in range(k, N):
            F[n] = fine(U[n])
        Unew, Gnew, Pnew = list(U), list(G), list(P)
        for n in range(k, N):
            if n > k:
                Gnew[n], Pnew[n] = coarse(Unew[n], Pnew[n - 1])
            Unew[n + 1] = (Gnew[n] - G[n]) + F[n]
        U, G, P = Unew, Gnew, Pnew
        if record:
            history.append(list(U))
    return U, (history, [])


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


def mgrit2_sl(u0, n_coarse, m, phi0, coarse2, nu, n_iter, record=False):
    """Two-level MGRIT, F(CF)^nu relaxation, with a two-step coarse scheme
    (SL-SI-SETTLS, Sec. 2.3.2) of one step per C-interval: coarse2(u, p) is
    that step from u with p the state one coarse step earlier (None: the
    one-step variant).  The coarse level is the coarsest one, so the
    two-step scheme runs in all its steps (Sec. 3.2.4; one device: no
    processor boundaries).  Reading: the history of a coarse step from a
    point of a coarse sequence is the sequence's previous point -- v_{i-1}
    for Phi_1(v_i) in the FAS term, w_{i-1} for Phi_1(w_i) in the serial
    solve, u_{i-1} in the initial coarse sweep -- and the first point has
    none.  With w = v on a prefix both steps are the same step, so the
    correction vanishes there exactly and the finite termination of the
    two-level iteration holds.  Returns C-point states as ``mgrit2``."""
    N1 = n_coarse
    C = [u0] + [None] * N1
    for i in range(N1):
        C[i + 1] = coarse2(C[i], C[i - 1] if i > 0 else None)
    history = [list(C)] if record else None

    def f_relax(Cpts):
        last = [None] * N1
        for i in range(N1):
            u = Cpts[i]
            for _ in range(m - 1):
                u = phi0(u)
            last[i] = u
        return last

    for _ in range(n_iter):
        last = f_relax(C)
        for _ in range(nu):
            C = [C[0]] + [phi0(last[i]) for i in range(N1)]
            last = f_relax(C)
        Fv = [phi0(last[i]) for i in range(N1)]
        Gv = [coarse2(C[i], C[i - 1] if i > 0 else None) for i in range(N1)]
        W = [C[0]] + [None] * N1
        for i in range(N1):
            Gw = Gv[i] if i == 0 else coarse2(W[i], W[i - 1])
            W[i + 1] = (Gw - Gv[i]) + Fv[i]
        C = W
        if record:
            history.append(list(C))
    return C, (history, [])


def _two_level_on_level1(W, psi, phi2, m1, nu, cycles):
    """`cycles` two-level MGRIT iterations on levels (1, 2) of the level-1
    problem w_i = psi(i, w_{i-1}) (i = 1..N1), starting from the list W
    (W[0] fixed).  Returns the new list."""
    N1 = len(W) - 1
    N2 = N1 // m1

    def f_relax(W):
        W = list(W)
        for j in range(N2):
            for s in range(1, m1):
                i = m1 * j + s
                W[i] = psi(i, W[i - 1])
        return W

    def c_relax(W):
        W = list(W)
        for j in range(1, N2 + 1):
            i = m1 * j
            W[i] = psi(i, W[i - 1])
        return W

    for _ in range(cycles):
        W = f_relax(W)
        for _ in range(nu):
            W = c_relax(W)
            W = f_relax(W)
        F2 = [None] + [psi(m1 * j, W[m1 * j - 1]) for j in range(1, N2 + 1)]
        V2 = [W[m1 * j] for j in range(N2 + 1)]
        G2 = [None] + [phi2(V2[j - 1]) for j in range(1, N2 + 1)]
        Z = [V2[0]] + [None] * N2
        for j in range(1, N2 + 1):
            Gz = G2[j] if j == 1 else phi2(Z[j - 1])
            Z[j] = (Gz - G2[j]) + F2[j]
        W = list(W)
        for j in range(1, N2 + 1):
            W[m1 * j] = Z[j]
        W = f_relax(W)
    return W


def mgrit3(u0, n_coarse, m, phi0, phi1, phi2, nu, n_iter, m1=None, cycles=1,
           record=False, incr_fn=None, tol=0.0):
    """Three-level MGRIT, F(CF)^nu relaxation on levels 0 and 1.  n_coarse =
    N_1 level-1 points (C-points of level 0, m fine points apart); level-2
    points every m1 (default m) level-1 points (N_1 divisible by m1); phi2
    spans m1 level-1 intervals.  Returns the level-0 C-point states after
    n_iter iterations, as mgrit2."""
    m1 = m if m1 is None else m1
    N1 = n_coarse
    assert N1 % m1 == 0, "level-1 points must fill whole level-2 intervals"
    C = [u0] + [None] * N1
    for i in range(N1):
        C[i + 1] = phi1(C[i])
    history = [list(C)] if record else None
    incrs = []

    def f_relax(Cpts):
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
            C = [C[0]] + [phi0(last[i]) for i in range(N1)]
            last = f_relax(C)
        Fv = [phi0(last[i]) for i in range(N1)]        # Phi_0(u_{m(i+1)-1})
        Gv = [phi1(C[i]) for i in range(N1)]           # Phi_1(v_i)

        def psi(i, w, Fv=Fv, Gv=Gv):                   # level-1 map into point i
            return (phi1(w) - Gv[i - 1]) + Fv[i - 1]

        W = _two_level_on_level1(list(C), psi, phi2, m1, nu, cycles)
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
