"""Parity at the benchmark's own size and launch configuration: T255 on
768 x 384, 64 states per launch, fine IMEX dt 45 s, coarse IMEX dt 180 s
with q = 4, nu = 1e17, two-level MGRIT FCF over 64 C-intervals x 4.

* One batched fine step of 64 states against the oracle on sampled states.
* The MGRIT iteration pint_solve runs (chunked fine propagation, serial sweep
  on a second stream) against the same iteration composed here from single
  pint_step calls and elementwise updates: bitwise, on every slice.
* Batch invariance at this size in every precision: a state stepped in a
  shuffled 64-state launch, in a 16-state launch and alone gives bitwise the
  same result (64- and 16-column GEMM tiles, both ring workgroup shapes,
  packed spectral tasks at four waves and at one wave per workgroup)."""

import numpy as np
import pytest

from gpu_util import assert_parity, from_dev, to_dev
from oracle.swe import Model
from paper_2306_09497_amd import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2306_09497_amd import pint  # noqa: E402

M, NLON, NLAT = 255, 768, 384
PHIBAR = 9.80616e4
GROUP, CFACTOR = 64, 4
DT_F, DT_C, NU_C, Q_C = 45.0, 180.0, 1.0e17, 4


@pytest.fixture(scope="module")
def model():
    return Model(M, NLON, NLAT, phibar=PHIBAR)


@pytest.fixture(scope="module")
def plan():
    pl = pint.Plan(M, NLON, NLAT, phibar=PHIBAR, max_batch=GROUP)
    yield pl
    pl.close()


def batch_states(md, n):
    """n jet + bump states: one analysed base plus seeded spectral noise of
    relative size 1e-3 per state (vectorised; m = 0 coefficients real)."""
    G = workloads.jet_bump_grid(md.grid.mu, NLON, phibar=PHIBAR, **workloads.jet_bump_params(0))
    base = np.stack([md.grid.anal(G[f]) for f in range(3)])
    rng = np.random.default_rng(7)
    m0 = md.grid.m_of == 0
    out = []
    for _ in range(n):
        z = rng.standard_normal(base.shape) + 1j * rng.standard_normal(base.shape)
        z[:, m0] = z[:, m0].real
        z[:, 0] = 0.0
        scale = np.array([np.abs(base[f, 1:]).max() for f in range(3)])[:, None]
        scale[2] = scale[1]
        out.append(base + 1e-3 * scale * z)
    return out


def test_batched_fine_step_vs_oracle(model, plan):
    """One fine IMEX step (no viscosity) of 64 states in one launch sequence;
    states 0, 37 and 63 against the oracle."""
    Us = batch_states(model, GROUP)
    u = to_dev(np.stack(Us), torch)
    out = torch.zeros_like(u)
    plan.step(pint.stepper(DT_F, 2, 0.0, pint.T_ALL), u, out, GROUP, 1)
    torch.cuda.synchronize()
    got = from_dev(out)
    for b in (0, 37, 63):
        ref = model.imex_step(Us[b], DT_F)
        assert_parity(got[b], ref, M)


def test_bench_iteration_composed_bitwise(model, plan):
    """pint_solve's MGRIT iteration (F-relaxation, coarse values of the
    relaxed C-points, chunked fine propagation with the serial correction
    sweep beside it) equals, bitwise, the iteration written out with
    pint_step at batch 64 and 1 and the update (G_new - G_old) + F."""
    fine = pint.stepper(DT_F, 2, 0.0, pint.T_ALL)
    coarse = pint.stepper(DT_C, Q_C, NU_C, pint.T_ALL)
    U0 = batch_states(model, 1)[0]
    u0 = to_dev(U0, torch)
    N = GROUP
    slices = torch.zeros((N + 1, 3, plan.ncoef, 2), dtype=torch.float64, device="cuda")
    plan.solve(pint.params(pint.MGRIT, N, fine, CFACTOR, coarse, 1, nrelax=1, max_iter=0),
               u0, slices)
    torch.cuda.synchronize()
    # iteration 0 by hand: U_{n+1} = G(U_n), one state at a time
    U = torch.zeros_like(slices)
    U[0] = u0[0]
    for n in range(N):
        plan.step(coarse, U[n:n + 1], U[n + 1:n + 2], 1, 1)
    torch.cuda.synchronize()
    assert torch.equal(U, slices)
    # iteration 1 by pint_solve
    it = pint.params(pint.MGRIT, N, fine, CFACTOR, coarse, 1, nrelax=1, max_iter=1, resume=True)
    plan.solve(it, u0, slices)
    torch.cuda.synchronize()
    # iteration 1 by hand
    V = U.clone()
    Fv = torch.zeros_like(U[:N])
    plan.step(fine, U[:N].contiguous(), Fv, N, CFACTOR)       # F-relaxation
    V[1:] = Fv
    Gold = torch.zeros_like(Fv)
    plan.step(coarse, V[:N].contiguous(), Gold, N, 1)        # Phi_1 of relaxed C-points
    plan.step(fine, V[:N].contiguous(), Fv, N, CFACTOR)      # F of the relaxed C-points
    W = V.clone()
    g = torch.zeros_like(U[:1])
    for n in range(N):
        if n == 0:
            gnew = Gold[0:1]
        else:
            plan.step(coarse, W[n:n + 1].contiguous(), g, 1, 1)
            gnew = g
        W[n + 1] = (gnew[0] - Gold[n]) + Fv[n]
    torch.cuda.synchronize()
    assert torch.equal(W, slices)


@pytest.mark.parametrize("precision", [pint.FP64, pint.LEG_FP32, pint.LEG_BF16X3])
def test_batch_invariance_bench_size_bitwise(model, precision):
    """Two coarse IMEX steps of T255 states: in a shuffled 64-state launch,
    a 16-state launch and alone, bitwise the same in each precision."""
    Us = batch_states(model, GROUP)
    st = pint.stepper(DT_C, Q_C, NU_C, pint.T_ALL)
    pl = pint.Plan(M, NLON, NLAT, phibar=PHIBAR, max_batch=GROUP, precision=precision)
    try:
        order = np.random.default_rng(3).permutation(GROUP)
        u64 = to_dev(np.stack([Us[i] for i in order]), torch)
        pl.step(st, u64, u64, GROUP, 2)
        u16 = to_dev(np.stack(Us[:16]), torch)
        pl.step(st, u16, u16, 16, 2)
        alone = {}
        for i in (0, 5, 37, 63):
            u1 = to_dev(Us[i], torch)
            pl.step(st, u1, u1, 1, 2)
            alone[i] = u1
        torch.cuda.synchronize()
        pos = {int(b): k for k, b in enumerate(order)}
        for i in range(16):
            assert torch.equal(u16[i], u64[pos[i]]), i
        for i, u1 in alone.items():
            assert torch.equal(u1[0], u64[pos[i]]), i
    finally:
        pl.close()
