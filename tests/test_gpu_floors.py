"""The GPU's float64 rounding floor against the oracle evaluated in x87
extended precision, beside the float64 oracle's own floor, for one nonlinear
tendency evaluation (Sec. 2.1, N = N_A + N_R) and one IMEX step (Sec. 2.3.1,
eq. IMEX) at every configured truncation.  The GPU path must sit at the
float64 floor: per field (Phi', vorticity, divergence, wind) its error
against extended precision is at most three times the float64 oracle's (or a
few ulps where both are at machine precision).  These floors set the
divergence bars of tests/gpu_util.py."""

import numpy as np
import pytest

from gpu_util import from_dev, per_m_errors, to_dev
from oracle.norms import rel_err, state_rel_err
from oracle.swe import Model, T_ALL
from paper_2306_09497_amd import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2306_09497_amd import pint  # noqa: E402

PB = 9.80616e4
CONFIGS = {21: (64, 32, 600.0), 63: (192, 96, 240.0), 127: (384, 192, 30.0),
           255: (768, 384, 45.0), 340: (1024, 512, 30.0)}
ULPS = 5e-16        # a few units of float64 rounding: below it errors are noise


def states(md):
    """Two test states: the jet + bump as analysed (divergence zero, the
    worst-conditioned case) and a second jet with a white-noise layer."""
    out = []
    for lam_c, amp, noise, seed in ((1.0, 120.0, 0.0, 0), (4.0, 80.0, 1e-3, 3)):
        G = workloads.jet_bump_grid(md.grid.mu, md.grid.nlon, phibar=PB, amp=amp, lam_c=lam_c)
        U = np.stack([md.grid.anal(G[f]) for f in range(3)])
        if noise > 0:
            U = workloads.white_noise(md.M, U, noise, seed)
        out.append(U)
    return out


def errors(x, ref, M):
    """(Phi', xi, delta, wind) relative L2 errors."""
    pl = rel_err(x, ref, M)
    st = state_rel_err(x, ref, M)
    return np.array([pl[0], pl[1], pl[2], st[1]])


@pytest.mark.parametrize("M,what", [(M, w) for w in ("neval", "step") for M in (21, 63, 127, 255)]
                         + [(340, "neval")])
def test_gpu_at_the_float64_floor(M, what):
    nlon, nlat, dt = CONFIGS[M]
    md = Model(M, nlon, nlat, phibar=PB)
    mx = Model(M, nlon, nlat, phibar=PB, extended=True)
    pl = pint.Plan(M, nlon, nlat, phibar=PB, max_batch=2)
    Us = states(md)
    u = to_dev(np.stack(Us), torch)
    out = torch.zeros_like(u)
    nu = 1e15 if M <= 127 else 1e14
    if what == "neval":
        pl.tendency(u, out, 2)
    else:
        pl.step(pint.stepper(dt, 4, nu, T_ALL), u, out, 2, 1)
    torch.cuda.synchronize()
    got = from_dev(out)
    pl.close()
    for b, U in enumerate(Us):
        if what == "neval":
            ref = md.tendencies(U)
            ext = mx.tendencies(U.astype(np.clongdouble)).astype(np.complex128)
        else:
            ref = md.imex_step(U, dt, nu, 4, T_ALL)
            ext = mx.imex_step(U.astype(np.clongdouble), dt, nu, 4, T_ALL).astype(np.complex128)
        e_gpu, e_orc = errors(got[b], ext, M), errors(ref, ext, M)
        pm_gpu, pm_orc = per_m_errors(got[b] - ext, ext, M), per_m_errors(ref - ext, ext, M)
        print(f"floor T{M} {what} state{b}: gpu-ext {e_gpu} oracle-ext {e_orc} "
              f"gpu-oracle {errors(got[b], ref, M)} per-m gpu {pm_gpu} oracle {pm_orc}", flush=True)
        assert np.all(e_gpu <= 3.0 * np.maximum(e_orc, ULPS)), (e_gpu, e_orc)
        assert np.all(pm_gpu <= 10.0 * np.maximum(pm_orc, 1e-14)), (pm_gpu, pm_orc)
