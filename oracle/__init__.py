"""Plain FP64 CPU oracle for the rotating shallow-water IMEX/Parareal/MGRIT path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product
(``paper_2306_09497_amd``) never imports it, and this package never imports
the product: the two share no code.

Everything here is written from the paper (arXiv 2306.09497) in the most direct
form, in float64 / complex128, with NumPy/SciPy library primitives (rfft/irfft,
Gauss-Legendre nodes, dense LU) as the only building blocks:

* ``sht``   -- Gauss grid, normalised associated Legendre functions, scalar and
               vector spherical-harmonic transforms (Sec. 2.2).
* ``swe``   -- the SWE operators L = L_G + L_C, N = N_A + N_R, the
               Crank-Nicolson half step, RK2 explicit step, backward-Euler
               (hyper)viscosity and the Strang-split IMEX step (Sec. 2.1, 2.3.1,
               App. A).
* ``pint``  -- Parareal (Sec. 3.1) and two-level MGRIT with F(CF)^nu
               relaxation and FAS coarse correction (Sec. 3.2).
* ``sl``    -- the SL-SI-SETTLS step (Sec. 2.3.2) and its one-step variant
               (Sec. 3.2.4): trajectories, bicubic interpolation, the
               semi-implicit solve.
* ``norms`` -- spectral (area-weighted) L2 norms and the paper's spectral
               max-norm error (Sec. 5).

Parity status per function is stated in each module header; everything that is
not pinned by a test against closed forms, library routines or invariants says
"parity unpinned" there.
"""

from . import sht, swe, pint, norms, sl  # noqa: F401
