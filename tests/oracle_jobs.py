"""Long oracle runs for the GPU parity tests, executed in worker processes
(spawned, so they never touch the GPU the test process uses).  Every
function is importable at top level so that a spawned worker can run it."""

import os

import numpy as np

JET_PHIBAR = 9.80616e4
_models = {}


def model(M, nlon, nlat, phibar=JET_PHIBAR):
    from oracle.swe import Model
    k = (M, nlon, nlat, phibar)
    if k not in _models:
        _models[k] = Model(M, nlon, nlat, phibar=phibar)
    return _models[k]


def jet_state(M, nlon, nlat, lam_c=1.0, amp=120.0):
    """Jet + height bump on the oracle grid (seeded inputs of the parity tests)."""
    from paper_2306_09497_amd import workloads
    md = model(M, nlon, nlat)
    G = workloads.jet_bump_grid(md.grid.mu, md.grid.nlon, phibar=JET_PHIBAR, amp=amp, lam_c=lam_c)
    return np.stack([md.grid.anal(G[f]) for f in range(3)])


def perturb_ulp(U, seed):
    """U with every real and imaginary part moved by one unit in the last
    place, in a random direction (the chaos calibration of the parity bar)."""
    rng = np.random.default_rng(seed)
    re = U.real + rng.choice([-1.0, 1.0], U.shape) * np.spacing(U.real)
    im = U.imag + rng.choice([-1.0, 1.0], U.shape) * np.spacing(U.imag) * (U.imag != 0)
    return re + 1j * im


def propagate(job):
    """job = (grid, U, dt, nsteps, nu, q): the oracle's IMEX propagation."""
    (M, nlon, nlat), U, dt, nsteps, nu, q = job
    from oracle.swe import T_ALL
    return model(M, nlon, nlat).propagate(U, dt, nsteps, nu, q, T_ALL)


def parareal(job):
    """job = (grid, u0, n_slices, fine (dt, steps, nu, q), coarse (...), n_iter):
    the oracle's Parareal, every iterate's slice-boundary states."""
    (M, nlon, nlat), u0, N, fine, coarse, n_iter = job
    from oracle import pint as opint
    from oracle.swe import T_ALL
    md = model(M, nlon, nlat)

    def prop(st):
        dt, n, nu, q = st
        return lambda U: md.propagate(U, dt, n, nu, q, T_ALL)

    _, (hist, _) = opint.parareal(u0, N, prop(fine), prop(coarse), n_iter, record=True)
    return [np.array(h) for h in hist]


def run_all(fn, jobs):
    """Run fn over jobs in spawned worker processes, the host's cores shared
    between them; results in job order."""
    import multiprocessing as mp
    ncpu = len(os.sched_getaffinity(0))
    per = str(max(1, ncpu // len(jobs)))
    keys = ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")
    saved = {k: os.environ.get(k) for k in keys}
    for k in keys:
        os.environ[k] = per
    try:
        with mp.get_context("spawn").Pool(len(jobs)) as pool:
            return pool.map(fn, jobs)
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
