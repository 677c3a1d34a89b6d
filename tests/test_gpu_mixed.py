"""GPU tests of the mixed-precision modes.  PINT_LEG_FP32: the Legendre GEMMs,
the Fourier rows and the ring FFT + pointwise tendencies run in FP32, while
the state, the implicit solve, viscosity, the RK combine, the tables and the
PinT corrections stay FP64.  PINT_LEG_BF16X3: the same, with each GEMM
product as three BF16 matrix-core products of split FP32 operands.

The error of this mode against the FP64 oracle is stated, not pinned by the
paper: the bounds below are measured on MI355X with a margin, per field and
per truncation.  Each case also checks that the error is above the FP64
rounding floor, so that a silent FP64 path would fail it."""

import numpy as np
import pytest

from gpu_util import from_dev, to_dev
from oracle.norms import rel_err, state_rel_err
from oracle.swe import Model, T_ALL
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
# Stated per-field relative L2 bounds (Phi', xi, delta) of the FP32 mode
# against the FP64 oracle, per truncation: one tendency evaluation, and the
# IMEX steps of test_fp32_step.  Phi' and xi sit near FP32 rounding; the
# divergence carries n(n+1)/a^2 times the FP32 rounding of the analysed
# kinetic energy, which grows with the truncation and is large against the
# small divergence tendency of a balanced jet.
TOL = {
    "fp32": {
        "tend": {"T63": (2e-6, 2e-6, 2e-4), "T127": (2e-6, 2e-6, 1e-3),
                 "T255": (2e-6, 2e-6, 5e-3)},
        "step": {"T63": (2e-7, 2e-7, 5e-5), "T127": (2e-7, 2e-7, 2e-4),
                 "T255": (2e-7, 2e-7, 2e-3)},
        "state": 2e-7,            # (Phi', wind) after the steps
    },
    "bf16x3": {
        "tend": {"T63": (1e-4, 1e-4, 3e-3), "T127": (1e-4, 1e-4, 2e-2),
                 "T255": (1e-4, 1e-4, 6e-2)},
        "step": {"T63": (5e-6, 5e-6, 1e-3), "T127": (5e-6, 5e-6, 1e-2),
                 "T255": (5e-6, 5e-6, 5e-2)},
        "state": 5e-6,
    },
}
MODES = {"fp32": pint.LEG_FP32, "bf16x3": pint.LEG_BF16X3}
FLOOR = 1e-10                 # FP32 arithmetic must show above FP64 rounding

_models, _plans = {}, {}


def model(key):
    if key not in _models:
        M, nlon, nlat = CONFIGS[key]
        _models[key] = Model(M, nlon, nlat, phibar=JET_PHIBAR)
    return _models[key]


def plan(key, precision=pint.LEG_FP32, max_batch=8):
    k = (key, precision, max_batch)
    if k not in _plans:
        M, nlon, nlat = CONFIGS[key]
        _plans[k] = pint.Plan(M, nlon, nlat, phibar=JET_PHIBAR, max_batch=max_batch,
                              precision=precision)
    return _plans[k]


def jet(key, lam_c=1.0, amp=120.0, extra_noise=0.0, seed=0):
    md = model(key)
    G = workloads.jet_bump_grid(md.grid.mu, md.grid.nlon, phibar=JET_PHIBAR, amp=amp,
                                lam_c=lam_c)
    U = np.stack([md.grid.anal(G[f]) for f in range(3)])
    if extra_noise > 0:
        U = workloads.white_noise(md.M, U, extra_noise, seed)
    return U


def mixed_errors(got, ref, M, what):
    e = rel_err(got, ref, M)
    print(f"{what}: rel L2 (Phi', xi, delta) = {e}", flush=True)
    return e


def check_mixed(errs, tol):
    """All bounds, and FP32 rounding visible in every case (a field whose
    tendency is identically zero, like N_xi of a zonal jet, is exact)."""
    for what, e in errs:
        assert np.all(e < np.asarray(tol)), (what, e, tol)
        assert np.max(e) > FLOOR, (what, "error at FP64 level: FP32 path not taken?", e)


@pytest.mark.parametrize("mode", list(MODES))
@pytest.mark.parametrize("key", ["T63", "T127", "T255"])
def test_mixed_tendency(key, mode):
    """Rows a1-a7 in the mixed modes: one N-eval of two states."""
    md, pl = model(key), plan(key, MODES[mode])
    U1 = jet(key, lam_c=1.0)
    U2 = jet(key, lam_c=4.0, amp=80.0, extra_noise=1e-3, seed=3)
    u = to_dev(np.stack([U1, U2]), torch)
    out = torch.zeros_like(u)
    pl.tendency(u, out, 2)
    torch.cuda.synchronize()
    got = from_dev(out)
    errs = [(f"{mode} {key} tendency b={b}",
             mixed_errors(got[b], md.tendencies(U), md.M, f"{mode} {key} tendency b={b}"))
            for b, U in enumerate((U1, U2))]
    check_mixed(errs, TOL[mode]["tend"][key])
    if mode == "bf16x3":
        # the split-BF16 products round near 2^-16: well above the FP32 mode
        o32 = torch.zeros_like(u)
        plan(key, pint.LEG_FP32).tendency(u, o32, 2)
        torch.cuda.synchronize()
        g32 = from_dev(o32)
        for b, U in enumerate((U1, U2)):
            e32 = rel_err(g32[b], md.tendencies(U), md.M)
            assert np.max(errs[b][1]) > 4 * np.max(e32), (errs[b][1], e32)


@pytest.mark.parametrize("mode", list(MODES))
@pytest.mark.parametrize("key,dt,nsteps", [("T63", 240.0, 10), ("T127", 30.0, 4),
                                           ("T255", 45.0, 1)])
def test_mixed_step(key, dt, nsteps, mode):
    """Row a10 in the mixed modes: IMEX steps with viscosity."""
    md, pl = model(key), plan(key, MODES[mode])
    U1 = jet(key, lam_c=2.0)
    U2 = jet(key, lam_c=5.0, amp=150.0, extra_noise=1e-4, seed=5)
    nu = 1e15 if md.M <= 127 else 1e14
    st = pint.stepper(dt, 4, nu, T_ALL)
    u = to_dev(np.stack([U1, U2]), torch)
    out = torch.zeros_like(u)
    pl.step(st, u, out, 2, nsteps)
    ref64 = torch.zeros_like(u)
    plan(key, pint.FP64).step(st, u, ref64, 2, nsteps)
    torch.cuda.synchronize()
    got, g64 = from_dev(out), from_dev(ref64)
    errs = []
    for b, U in enumerate((U1, U2)):
        ref = md.propagate(U, dt, nsteps, nu, 4, T_ALL)
        e = mixed_errors(got[b], ref, md.M, f"{mode} {key} {nsteps} steps b={b}")
        st_e = state_rel_err(got[b], ref, md.M)
        print(f"  state (Phi', wind) rel L2 = {st_e}", flush=True)
        # the FP64 GPU path is at the oracle to 1e-11, so both differences agree
        e64 = rel_err(got[b], g64[b], md.M)
        assert np.allclose(e, e64, rtol=1e-2, atol=1e-11), (e, e64)
        assert np.all(st_e < TOL[mode]["state"]), st_e
        errs.append((f"{mode} {key} {nsteps} steps b={b}", e))
    check_mixed(errs, TOL[mode]["step"][key])


@pytest.mark.parametrize("mode", list(MODES))
def test_mixed_batch_invariance_bitwise(mode):
    """The mixed modes keep a slice's result bitwise independent of the
    batch (the narrow and the wide GEMM tiles sum in the same k-order)."""
    pl = plan("T63", MODES[mode], max_batch=16)
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
        assert torch.equal(u[order.index(i)], single[i][0])


@pytest.mark.parametrize("mode", list(MODES))
def test_mixed_parareal_exact_bitwise(mode):
    """Parareal after N iterations reproduces the serial fine states bitwise
    in the mixed modes too (the fine propagator is deterministic and batch
    invariant)."""
    M, nlon, nlat = CONFIGS["T21"]
    pl = pint.Plan(M, nlon, nlat, phibar=2.94e4, max_batch=8, precision=MODES[mode])
    U0 = workloads.solid_body(M, noise=1e-6, seed=0)
    f = pint.stepper(60.0, 2, 0.0, T_ALL)
    c = pint.stepper(3600.0, 2, 0.0, T_ALL)
    prm = pint.params(pint.PARAREAL, 8, f, 180, c, 3, max_iter=8)
    out = torch.zeros((9, 3, pl.ncoef, 2), dtype=torch.float64, device="cuda")
    pl.solve(prm, to_dev(U0, torch), out)
    u = to_dev(U0, torch)
    for n in range(1, 9):
        pl.step(f, u, u, 1, 180)
        torch.cuda.synchronize()
        assert torch.equal(u[0], out[n])
    pl.close()


@pytest.mark.parametrize("mode", list(MODES))
def test_mixed_mode_keeps_fp64_parts(mode):
    """The implicit solve and the public scalar transforms stay FP64 in the
    mixed modes: bitwise equal to the FP64 plan's."""
    p32, p64 = plan("T63", MODES[mode]), plan("T63", pint.FP64)
    U = jet("T63", extra_noise=1e-3, seed=1)
    st = pint.stepper(240.0, 4, 1e15, T_ALL)
    u = to_dev(U, torch)
    a, b = torch.zeros_like(u), torch.zeros_like(u)
    p32.implicit(st, u, a, 1)
    p64.implicit(st, u, b, 1)
    g = model("T63").grid
    spec = u[:, 0].contiguous()
    ga = torch.zeros((1, g.nlat, g.nlon), dtype=torch.float64, device="cuda")
    gb = torch.zeros_like(ga)
    p32.synthesis(spec, ga, 1)
    p64.synthesis(spec, gb, 1)
    sa, sb = torch.zeros_like(spec), torch.zeros_like(spec)
    p32.analysis(ga, sa, 1)
    p64.analysis(gb, sb, 1)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert torch.equal(ga, gb)
    assert torch.equal(sa, sb)
