"""GPU parity of every hot-path row against the FP64 CPU oracle, through the
C ABI (libpint.so).  Bar: relative L2 error per field <= 1e-11 for the FP64
path (tighter bounds where the arithmetic allows)."""

import math

import numpy as np
import pytest

from gpu_util import assert_parity, field_rel, from_dev, to_dev
from oracle import sht
from oracle.swe import Model, T_ALL, T_LC, T_LG, T_NL, T_VISC
from paper_2306_09497_amd import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2306_09497_amd import pint  # noqa: E402

JET_PHIBAR = 9.80616e4
CONFIGS = {
    "T21": (21, 64, 32),
    "T63": (63, 192, 96),
    "T127": (127, 384, 192),
    "T255": (255, 768, 384),
}

_models = {}
_plans = {}


def model(key, phibar=JET_PHIBAR, omega=7.292e-5):
    k = (key, phibar, omega)
    if k not in _models:
        M, nlon, nlat = CONFIGS[key]
        _models[k] = Model(M, nlon, nlat, phibar=phibar, omega=omega)
    return _models[k]


def plan(key, phibar=JET_PHIBAR, omega=7.292e-5, max_batch=8):
    k = (key, phibar, omega, max_batch)
    if k not in _plans:
        M, nlon, nlat = CONFIGS[key]
        _plans[k] = pint.Plan(M, nlon, nlat, phibar=phibar, omega=omega, max_batch=max_batch)
    return _plans[k]


def jet(key, lam_c=1.0, amp=120.0, extra_noise=0.0, seed=0):
    md = model(key)
    G = workloads.jet_bump_grid(md.grid.mu, md.grid.nlon, phibar=JET_PHIBAR, amp=amp,
                                lam_c=lam_c)
    U = np.stack([md.grid.anal(G[f]) for f in range(3)])
    if extra_noise > 0:
        U = workloads.white_noise(md.M, U, extra_noise, seed)
    return U


def test_library_symbols():
    lib = pint.load()
    for name in pint.EXPORTS:
        assert hasattr(lib, name)


@pytest.mark.parametrize("key", ["T21", "T63", "T127", "T255"])
def test_gauss_grid(key):
    """Row a0: Gauss nodes and weights generated on the device."""
    md, pl = model(key), plan(key)
    mu, w = pl.grid_coords()
    assert np.max(np.abs(mu - md.grid.mu)) < 4e-16
    assert np.max(np.abs(w - md.grid.w) / md.grid.w) < 2e-14
    assert abs(w.sum() - 2.0) < 1e-14


@pytest.mark.parametrize("key", ["T21", "T63", "T127", "T255"])
def test_scalar_transforms(key):
    """Rows a0, a2, a3, a5, a6: synthesis and analysis against the oracle
    and the round trip on the truncation."""
    md, pl = model(key), plan(key)
    g = md.grid
    rng = np.random.default_rng(7)
    B = 3
    c = rng.standard_normal((B, g.nc)) + 1j * rng.standard_normal((B, g.nc))
    c[:, :g.M + 1] = c[:, :g.M + 1].real
    n = g.n_of.astype(float)
    c = c / (1.0 + n)                                  # decaying spectrum
    spec = torch.from_numpy(np.stack([c.real, c.imag], -1).copy()).cuda()
    grid = torch.zeros((B, g.nlat, g.nlon), dtype=torch.float64, device="cuda")
    pl.synthesis(spec, grid, B)
    back = torch.zeros_like(spec)
    pl.analysis(grid, back, B)
    torch.cuda.synchronize()
    G = grid.cpu().numpy()
    for b in range(B):
        ref = g.synth(c[b])
        assert np.max(np.abs(G[b] - ref)) < 1e-13 * np.max(np.abs(ref))
    bk = back.cpu().numpy()
    bk = bk[..., 0] + 1j * bk[..., 1]
    assert np.max(np.abs(bk - c)) < 1e-13 * np.max(np.abs(c))
    # analysis of an arbitrary (not band-limited) grid field
    x = rng.standard_normal((1, g.nlat, g.nlon))
    gx = torch.from_numpy(x).cuda()
    sx = torch.zeros((1, g.nc, 2), dtype=torch.float64, device="cuda")
    pl.analysis(gx, sx, 1)
    ref = g.anal(x[0])
    got = sx.cpu().numpy()[0]
    got = got[:, 0] + 1j * got[:, 1]
    assert np.max(np.abs(got - ref)) < 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("key", ["T21", "T63", "T127", "T255"])
def test_tendency(key):
    """Rows a1-a7: nonlinear tendencies N(U) (one N-eval) of two states."""
    md, pl = model(key), plan(key)
    U1 = jet(key, lam_c=1.0)
    U2 = jet(key, lam_c=4.0, amp=80.0, extra_noise=1e-3, seed=3)
    u = to_dev(np.stack([U1, U2]), torch)
    out = torch.zeros_like(u)
    pl.tendency(u, out, 2)
    torch.cuda.synchronize()
    got = from_dev(out)
    for b, U in enumerate((U1, U2)):
        assert_parity(got[b], md.tendencies(U), md.M, "neval")


@pytest.mark.parametrize("key", ["T21", "T63", "T127"])
@pytest.mark.parametrize("terms", [T_LG | T_LC, T_LG, T_LC, T_ALL])
def test_implicit(key, terms):
    """Rows a8, a9: Crank-Nicolson half step with implicit Coriolis (two
    tridiagonal chains per m) and the fused viscosity factor."""
    md, pl = model(key), plan(key)
    U = jet(key, extra_noise=1e-2, seed=1)
    dt, nu, q = 450.0, 2e15, 4
    st = pint.stepper(dt, q, nu, terms)
    u = to_dev(U, torch)
    x = torch.zeros_like(u)
    pl.implicit(st, u, x, 1)
    torch.cuda.synchronize()
    ref = md.cn_half(U, dt, terms)
    if terms & T_VISC:
        ref = md.viscosity(ref, dt, nu, q)
    assert_parity(from_dev(x)[0], ref, md.M, "step", (1e-13, 1e-13), 1e-13, 1e-12)


@pytest.mark.parametrize("key,dt,nsteps", [("T21", 600.0, 20), ("T63", 240.0, 10),
                                           ("T127", 30.0, 4), ("T255", 45.0, 1)])
def test_step(key, dt, nsteps):
    """Row a10: full IMEX steps on a batch of 2 slices, with viscosity."""
    md, pl = model(key), plan(key)
    U1 = jet(key, lam_c=2.0)
    U2 = jet(key, lam_c=5.0, amp=150.0, extra_noise=1e-4, seed=5)
    nu = 1e15 if md.M <= 127 else 1e14
    st = pint.stepper(dt, 4, nu, T_ALL)
    u = to_dev(np.stack([U1, U2]), torch)
    out = torch.zeros_like(u)
    pl.step(st, u, out, 2, nsteps)
    torch.cuda.synchronize()
    got = from_dev(out)
    for b, U in enumerate((U1, U2)):
        assert_parity(got[b], md.propagate(U, dt, nsteps, nu, 4, T_ALL), md.M)


def test_step_in_place_and_chunks():
    """u_out may alias u_in; batches larger than max_batch are chunked."""
    pl = plan("T21", max_batch=3)
    md = model("T21")
    Us = [jet("T21", lam_c=0.5 * i, amp=60.0 + 10 * i) for i in range(7)]
    u = to_dev(np.stack(Us), torch)
    st = pint.stepper(600.0, 2, 1e5, T_ALL)
    pl.step(st, u, u, 7, 3)
    torch.cuda.synchronize()
    got = from_dev(u)
    for b in range(7):
        assert_parity(got[b], md.propagate(Us[b], 600.0, 3, 1e5, 2, T_ALL), md.M)


def test_batch_invariance_bitwise():
    """A slice's result is bitwise independent of batch size and order."""
    pl = plan("T63", max_batch=16)
    Us = [jet("T63", lam_c=0.3 * i, amp=50.0 + 7 * i) for i in range(9)]
    st = pint.stepper(240.0, 4, 1e15, T_ALL)
    single = []
    for U in Us[:3]:
        u = to_dev(U, torch)
        pl.step(st, u, u, 1, 2)
        single.append(u.clone())
    order = [4, 0, 8, 2, 1, 7, 3, 5, 6]
    u = to_dev(np.stack([Us[i] for i in order]), torch)
    pl.step(st, u, u, 9, 2)
    torch.cuda.synchronize()
    for i in range(3):
        pos = order.index(i)
        assert torch.equal(u[pos], single[i][0])


def test_rel_diff():
    pl, md = plan("T63"), model("T63")
    A = jet("T63", extra_noise=1e-3, seed=2)
    Bv = A + 1e-3 * jet("T63", lam_c=3.0, extra_noise=1e-2, seed=4)
    got = pl.rel_diff(to_dev(A, torch), to_dev(Bv, torch), 1)[0]
    from oracle.norms import rel_err, state_rel_err
    pr = rel_err(Bv, A, md.M)
    sr = state_rel_err(Bv, A, md.M)
    ref = np.array([pr[0], pr[1], pr[2], sr[1]])
    assert np.allclose(got, ref, rtol=1e-12)


def test_step_chaining_bitwise():
    """n IMEX steps in one call (each step's first half step made by the
    previous step's closing kernel) equal n single-step calls, bitwise, at
    every SEG width of the spectral kernels."""
    for key in ("T21", "T63", "T127", "T255"):
        M, nlon, nlat = CONFIGS[key]
        pl = pint.Plan(M, nlon, nlat, phibar=9.80616e4, max_batch=2)
        U = workloads.solid_body(M, noise=1e-3, seed=3)
        u = to_dev(U, torch)
        for st in (pint.stepper(45.0, 2, 0.0, T_ALL), pint.stepper(180.0, 4, 1e16, T_ALL)):
            a, b = torch.zeros_like(u), torch.zeros_like(u)
            pl.step(st, u, a, 1, 3)
            pl.step(st, u, b, 1, 1)
            pl.step(st, b, b, 1, 1)
            pl.step(st, b, b, 1, 1)
            torch.cuda.synchronize()
            assert torch.equal(a, b), key
        pl.close()
