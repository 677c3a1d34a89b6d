"""pint_step_noalloc (the propagator for callers that cannot allocate) against
pint_step through the C ABI: bitwise the same states, on two calls in a row
(the second with a smaller input), without any device allocation by the
plan.  Marked gpu; collected last so that a failure hides no other test."""

import ctypes

import numpy as np
import pytest

from gpu_util import to_dev
from paper_2306_09497_amd import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2306_09497_amd import pint  # noqa: E402


def jets(M, nlon, nlat, count, seed):
    from oracle.sht import Grid
    g = Grid(M, nlon, nlat)
    out = []
    for i in range(count):
        G = workloads.jet_bump_grid(g.mu, nlon, phibar=9.80616e4, amp=60.0 + 13.0 * i,
                                    lam_c=0.7 * i + 0.1 * seed)
        out.append(np.stack([g.anal(G[f]) for f in range(3)]))
    return np.stack(out)


@pytest.mark.parametrize("M,nlon,nlat,counts,nsteps", [
    (63, 192, 96, (9, 4), 3),          # chunks of max_batch, then a smaller call
    (255, 768, 384, (3, 1), 2),        # two states per chunk fit the scratch
])
def test_noalloc_matches_pint_step(M, nlon, nlat, counts, nsteps):
    pl = pint.Plan(M, nlon, nlat, phibar=9.80616e4, max_batch=4)
    st = pint.stepper(240.0 if M < 255 else 45.0, 4, 1e15, pint.T_ALL)
    lib = pint.load()
    for call, B in enumerate(counts):
        U = to_dev(jets(M, nlon, nlat, B, call), torch)
        print(f"noalloc T{M} call {call} B={B} nsteps={nsteps}", flush=True)
        before = pl.info().allocations
        a = torch.zeros_like(U)
        pl.step_noalloc(st, U, a, B, nsteps)
        torch.cuda.synchronize()
        assert pl.info().allocations == before
        b = torch.zeros_like(U)
        pl.step(st, U, b, B, nsteps)
        torch.cuda.synchronize()
        assert torch.equal(a, b), (call, float((a - b).abs().max()))
        # in place, and the plan's workspace untouched by the scratch path
        c = U.clone()
        pl.step_noalloc(st, c, c, B, nsteps)
        torch.cuda.synchronize()
        assert torch.equal(c, b)
    # argument errors come back as statuses
    u = torch.zeros((1, 3, pl.ncoef, 2), dtype=torch.float64, device="cuda")
    bad = pint.stepper(-1.0)
    assert lib.pint_step_noalloc(pl._h, ctypes.byref(bad), u.data_ptr(), u.data_ptr(), 1, 1,
                                 None) == -1
    pl.close()


def test_noalloc_refuses_a_state_beyond_the_scratch():
    """T500 on 1024 x 512: one state's workspace plus factors (82 MiB)
    exceeds the 64 MiB scratch."""
    pl = pint.Plan(500, 1024, 512, phibar=9.80616e4, max_batch=1)
    u = torch.zeros((1, 3, pl.ncoef, 2), dtype=torch.float64, device="cuda")
    with pytest.raises(pint.PintError) as e:
        pl.step_noalloc(pint.stepper(30.0), u, u, 1, 1)
    assert "maximum" in str(e.value)
    pl.close()
