"""Batching: PinT iterations replayed from a captured HIP graph, and the
Legendre GEMM launch shapes chosen by the plan's autotuner.  Both are
matters of speed only: iterates replayed from a graph are bitwise the
iterates of plain launches (Sec. 3.2, MGRIT; Sec. 3.1, Parareal), and every
GEMM shape gives bitwise the same transforms (Sec. 2.2)."""

import numpy as np
import pytest

from gpu_util import to_dev
from paper_2306_09497_amd import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2306_09497_amd import pint  # noqa: E402

M, NLON, NLAT = 21, 64, 32


def plan_with(monkeypatch, env, M=M, nlon=NLON, nlat=NLAT, max_batch=8):
    for k, v in env.items():
        monkeypatch.setenv(k, v)
    pl = pint.Plan(M, nlon, nlat, phibar=2.94e4, max_batch=max_batch)
    for k in env:
        monkeypatch.delenv(k)
    return pl


def solve(pl, q, U0):
    u0 = to_dev(U0, torch)
    us = torch.zeros((q.n_intervals + 1, 3, pl.ncoef, 2), dtype=torch.float64, device="cuda")
    rep = pl.solve(q, u0, us)
    torch.cuda.synchronize()
    return us, rep


def c1(method, k, **kw):
    return pint.params(method, 8, pint.stepper(60.0, 2, 0.0, pint.T_ALL), 180,
                       pint.stepper(3600.0, 2, 0.0, pint.T_ALL), 3, max_iter=k, **kw)


@pytest.mark.parametrize("q", [
    c1(pint.MGRIT, 5, nrelax=1),       # (relaxation not pipelined: PINT_PIPELINE=0 below)
    c1(pint.MGRIT, 4, nrelax=0),
    pint.params(pint.MGRIT, 8, pint.stepper(60.0, 2, 0.0, pint.T_ALL), 180,
                pint.stepper(3600.0, 2, 1e5, pint.T_ALL), 3, nrelax=1, max_iter=4, levels=3,
                cfactor1=2, coarse2=pint.stepper(7200.0, 2, 1e5, pint.T_ALL), coarse2_steps=3),
], ids=["mgrit_fcf", "mgrit_f", "mgrit3"])
def test_graph_replay_is_bitwise_the_plain_launches(monkeypatch, q):
    U0 = workloads.solid_body(M, noise=1e-3, seed=4)
    a, ra = solve(plan_with(monkeypatch, {"PINT_GRAPHS": "0", "PINT_PIPELINE": "0"}), q, U0)
    b, rb = solve(plan_with(monkeypatch, {"PINT_PIPELINE": "0"}), q, U0)
    print(f"graph iterations {rb.graph_iters} of {rb.iters}; seconds plain "
          f"{list(ra.seconds[:ra.iters])} graph {list(rb.seconds[:rb.iters])}", flush=True)
    assert ra.graph_iters == 0 and rb.graph_iters == q.max_iter - 1
    assert torch.equal(a, b)
    assert [ra.incr[i] for i in range(ra.iters)] == [rb.incr[i] for i in range(rb.iters)]
    assert ra.fine_slice_steps == rb.fine_slice_steps and ra.coarse_steps == rb.coarse_steps
    for i in range(rb.iters):
        assert 0.0 < rb.fine_seconds[i] <= rb.seconds[i]


def test_graph_replay_of_a_resumed_parareal(monkeypatch):
    """Parareal resumed from an iterate recomputes every slice, so its
    iterations repeat and replay from a graph too."""
    U0 = workloads.solid_body(M, noise=1e-3, seed=5)
    pa = plan_with(monkeypatch, {"PINT_GRAPHS": "0"})
    pb = plan_with(monkeypatch, {})
    a, _ = solve(pa, c1(pint.PARAREAL, 2), U0)
    b = a.clone()
    u0 = to_dev(U0, torch)
    ra = pa.solve(c1(pint.PARAREAL, 3, resume=True), u0, a)
    rb = pb.solve(c1(pint.PARAREAL, 3, resume=True), u0, b)
    torch.cuda.synchronize()
    assert ra.graph_iters == 0 and rb.graph_iters == 2
    assert torch.equal(a, b)


@pytest.mark.parametrize("B", [1, 2, 9, 16])
@pytest.mark.parametrize("variant", [1, 2])
def test_every_gemm_shape_gives_the_same_step(monkeypatch, B, variant):
    """Launch shapes with k-slabs of 16 and of 32 and column tiles of 64 and
    128, and ring workgroups of 128 and 256 threads (both launch classes),
    give bitwise the same steps."""
    pa = plan_with(monkeypatch, {"PINT_GEMM_VARIANT": "0"}, 63, 192, 96, 16)
    pb = plan_with(monkeypatch, {"PINT_GEMM_VARIANT": str(variant)}, 63, 192, 96, 16)
    assert pb.info().gemm_shape[0][0] == 1 and pb.info().gemm_shape[1][1] == variant
    assert list(pb.info().ring_threads) == [128, 256]
    U = np.stack([workloads.solid_body(63, noise=1e-3, seed=s) for s in range(B)])
    u = to_dev(U, torch)
    st = pint.stepper(240.0, 4, 1e15, pint.T_ALL)
    a, b = torch.zeros_like(u), torch.zeros_like(u)
    pa.step(st, u, a, B, 2)
    pb.step(st, u, b, B, 2)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_reserve_tunes_the_gemm_shapes():
    pl = pint.Plan(127, 384, 192, phibar=9.80616e4, max_batch=16)
    q = pint.params(pint.MGRIT, 16, pint.stepper(30.0, 2, 0.0, pint.T_ALL), 4,
                    pint.stepper(120.0, 4, 1e15, pint.T_ALL), 1, nrelax=1, max_iter=1)
    pl.reserve(q)
    info = pl.info()
    us = np.array([[info.gemm_us[k][c] for c in range(2)] for k in range(2)])
    shapes = np.array([[info.gemm_shape[k][c] for c in range(2)] for k in range(2)])
    print(f"tuned T127: shapes {shapes.tolist()} us {us.tolist()}", flush=True)
    assert np.all(us > 0.0)
    pl.close()
