#!/usr/bin/env python3
"""Throughput of the MI355X shallow-water PinT path on one GPU.

One step = one two-level MGRIT iteration with FCF relaxation (Sec. 3.2) over
one T255 slice group: 64 C-intervals x cfactor 4 = 256 fine time points,
fine IMEX dt = 45 s, coarse IMEX dt = 180 s with 4th-order hyperviscosity
nu = 1e17 m^4/s on the coarse level (paper's table for IMEX coarse levels).
Each step runs every row of the hot path: the batched fine propagator (CN
solve, Legendre synthesis GEMM, ring FFT + tendencies, Legendre analysis
GEMM, RK assembly, viscosity) over the 64 intervals for the F- and
C-relaxations and the fine propagation, the batched coarse propagator on the
relaxed C-points, the serial coarse correction sweep and the increment norms.

value = fine slice-steps executed / wall time of the timed steps.
Inputs are synthetic (jet + height bump shaped like the paper's unstable-jet
test), generated on the device before timing.  The dominant kernel's
roofline figure is timed live with HIP events on the library's stream; the
CPU baseline is the FP64 oracle timed on this host on a bounded sample.
"""

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

M, NLON, NLAT = 255, 768, 384
GROUP = 64                  # C-intervals per slice group (one launch batch)
CFACTOR = 4
DT_FINE, DT_COARSE = 45.0, 180.0
NU_COARSE, Q_COARSE = 1.0e17, 4
PHIBAR = 9.80616e4          # g * 10 km mean depth
PEAK_FP64 = 78.6e12         # MI355X dense FP64 (matrix and vector), FLOP/s
PEAK_FP32 = 157.3e12        # MI355X dense FP32 matrix, FLOP/s
PEAK_BF16 = 2.5e15          # MI355X dense BF16 matrix (3 products per useful one)
PEAK_HBM = 8.0e12           # MI355X HBM3E, B/s


def algorithmic_work(kind, B, prec=0):
    """Algorithmic FLOPs and HBM bytes of one launch over B states (T255).

    Legendre GEMMs (N/S folded): rows n = m..M+1 per m, parity-split, against
    the nlat/2 northern latitudes; synthesis has 6 fields x (re, im) columns
    per state, analysis 4.  Bytes: table once + operands + result once, at 8
    bytes per value (FP64) or 4 (the mixed modes, prec = 1 or 2).
    """
    w = 4.0 if prec in (1, 2) else 8.0
    nrows = (M + 1) * (M + 4) // 2          # sum_m (M - m + 2)
    nl2 = NLAT // 2
    if kind == "legendre_synth":
        cols = 12 * B
        flops = 2.0 * nl2 * nrows * cols
        byts = w * (nrows * nl2 + nrows * cols + 2 * (M + 1) * nl2 * cols)
    elif kind == "legendre_anal":
        cols = 8 * B
        flops = 2.0 * nl2 * nrows * cols
        byts = w * (nrows * nl2 + (M + 1) * NLAT * cols + nrows * cols)
    elif kind == "ring_tendency":
        # read the Fourier rows of the 6 fields once, write the 4 analysis fields once
        flops = 0.0
        byts = w * (2 * (M + 1) * nl2 * 12 * B + (M + 1) * NLAT * 8 * B)
    else:
        flops, byts = 0.0, 0.0
    return flops, byts


# HBM bytes per launch (64 states) measured with rocprofv3 --pmc FETCH_SIZE and
# WRITE_SIZE on `python -m paper_2306_09497_amd.profile_drivers tendency 64 3
# <precision>`, each counter scaled by what it reads for a plain 1 GiB copy
# (FETCH x 2.0, WRITE x 1.0), keyed by (kernel, precision), together with the
# SHA-256 prefixes of the sources the kernel is compiled from (its own file and
# the shared device header) when the counters were taken: a changed kernel
# reports traffic null until measured again.
_RING = {"ring.hip": "693ad39752d31eca", "device_common.h": "10c8dcd59ab35273"}
_LEG = {"legendre.hip": "18d2d21a361db2f0", "device_common.h": "10c8dcd59ab35273"}
MEASURED_TRAFFIC = {
    ("ring_tendency", 0): (546784 * 1024 * 2.0 + 478097 * 1024 * 1.0, _RING),
    ("legendre_synth", 0): (139917 * 1024 * 2.0 + 589824 * 1024 * 1.0, _LEG),
    ("legendre_anal", 0): (251583 * 1024 * 2.0 + 132608 * 1024 * 1.0, _LEG),
    ("ring_tendency", 1): (184225 * 1024 * 2.0 + 204433 * 1024 * 1.0, _RING),
    ("legendre_synth", 1): (63803 * 1024 * 2.0 + 296218 * 1024 * 1.0, _LEG),
    ("legendre_anal", 1): (114968 * 1024 * 2.0 + 66308 * 1024 * 1.0, _LEG),
    ("ring_tendency", 2): (184240 * 1024 * 2.0 + 205072 * 1024 * 1.0, _RING),
    ("legendre_synth", 2): (64658 * 1024 * 2.0 + 295429 * 1024 * 1.0, _LEG),
    ("legendre_anal", 2): (115175 * 1024 * 2.0 + 66304 * 1024 * 1.0, _LEG),
}


def measured_traffic(kind, prec=0, states=64):
    """Counter-measured HBM bytes per launch of `kind` at precision `prec` over
    `states` states, or None if absent (the counters were taken on 64-state
    launches) or if its sources changed since the counters were taken."""
    import hashlib
    if states != 64 or (kind, prec) not in MEASURED_TRAFFIC:
        return None
    byts, srcs = MEASURED_TRAFFIC[(kind, prec)]
    csrc = os.path.join(ROOT, "paper_2306_09497_amd", "csrc")
    for name, digest in srcs.items():
        with open(os.path.join(csrc, name), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest()[:16] != digest:
                return None
    return byts


def cpu_baseline(seconds):
    """The FP64 oracle on this host: fine IMEX steps of one T255 slice (the
    headline's unit of work), each step timed, for about `seconds`; the median
    step time at T21 and T127 (5 steps each); the end-to-end C1 Parareal run
    (T21 on 64x32, solid body + 1e-6 noise, 8 slices of 180 fine steps of
    60 s, coarse 3 x 3600 s, 8 iterations); and the serial-fine times of C2
    (11 520 steps at T127) and C3 (3 840 steps at T255) extrapolated from the
    median step times."""
    import numpy as np
    from threadpoolctl import threadpool_info
    from oracle import pint as opint
    from oracle.swe import Model
    from paper_2306_09497_amd import workloads

    md = Model(M, NLON, NLAT, phibar=PHIBAR)
    G = workloads.jet_bump_grid(md.grid.mu, NLON, phibar=PHIBAR, **workloads.jet_bump_params(0))
    U = np.stack([md.grid.anal(G[f]) for f in range(3)])
    md.imex_step(U, DT_FINE)                  # untimed: builds the per-m LU factors
    ts = []
    t0 = time.perf_counter()
    while True:
        a = time.perf_counter()
        U = md.imex_step(U, DT_FINE)
        ts.append(time.perf_counter() - a)
        if time.perf_counter() - t0 >= seconds and len(ts) >= 5:
            break
    dt = time.perf_counter() - t0
    n = len(ts)
    threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    per = {"T255": 1e3 * float(np.median(ts))}
    spread = {"T255": [1e3 * float(np.percentile(ts, 10)), 1e3 * float(np.percentile(ts, 90))]}
    for Mt, nl, nt in ((21, 64, 32), (127, 384, 192)):
        mt = Model(Mt, nl, nt, phibar=PHIBAR)
        Gt = workloads.jet_bump_grid(mt.grid.mu, nl, phibar=PHIBAR, **workloads.jet_bump_params(0))
        Ut = mt.imex_step(np.stack([mt.grid.anal(Gt[f]) for f in range(3)]), DT_FINE)
        tt = []
        for _ in range(5):
            a = time.perf_counter()
            Ut = mt.imex_step(Ut, DT_FINE)
            tt.append(time.perf_counter() - a)
        per[f"T{Mt}"] = 1e3 * float(np.median(tt))
    # C1 end to end
    m1 = Model(21, 64, 32, phibar=2.94e4)
    u0 = workloads.solid_body(21, noise=1e-6, seed=0)
    m1.imex_step(u0, 60.0)
    m1.imex_step(u0, 3600.0)
    a = time.perf_counter()
    opint.parareal(u0, 8, lambda u: m1.propagate(u, 60.0, 180),
                   lambda u: m1.propagate(u, 3600.0, 3), 8)
    c1_s = time.perf_counter() - a
    cpu = ""
    try:
        with open("/proc/cpuinfo") as f:
            cpu = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    return {"value": 1e3 / per["T255"], "unit": "fine slice-steps/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{n} fine IMEX steps (dt {DT_FINE:g} s) of one T255 768x384 jet+bump "
                      f"slice after LU setup, {dt:.1f} s, value from the median step; host has "
                      f"{len(os.sched_getaffinity(0))} cores available",
            "ms_per_fine_step_median": per, "ms_per_fine_step_p10_p90": spread,
            "c1_parareal_end_to_end_s": c1_s,
            "serial_fine_extrapolated_s": {"C2_T127_11520_steps": 11520 * per["T127"] * 1e-3,
                                           "C3_T255_3840_steps": 3840 * per["T255"] * 1e-3},
            "cpu": cpu}


def e_phi_r(phi, ref, mmax, R=32):
    """max_{m <= n <= R} |Phi_mn - ref_mn| / max_{m <= n <= R} |ref_mn| (spectral
    error of the geopotential up to total wavenumber R, Sec. 5)."""
    import numpy as np
    sel = []
    for m in range(R + 1):
        base = m * (2 * mmax + 3 - m) // 2
        sel.extend(base + (n - m) for n in range(m, R + 1))
    sel = np.array(sel)
    d = np.abs(phi[sel] - ref[sel]).max()
    return float(d / np.abs(ref[sel]).max())


def time_to_tol(per_slice_iters=2):
    """Parareal to a relative increment of 1e-8 in the C2 shape: T127
    (384x192), 64 slices of 5400 s (4 days), fine IMEX 30 s x 180, jet +
    bump.  The coarse level C2 specifies (IMEX 900 s x 6, q = 4, nu = 1e17:
    nu = 1e15 makes that step unstable for the jet) does not converge: the
    coarse viscosity damps the high modes that the fine level keeps, whose
    error then moves one slice per iteration (its increments are reported).
    The timed run uses a coarse level that converges: IMEX 100 s x 54 without
    viscosity.  Timed against (i) serial fine propagation (batch 1, 11 520
    steps) and (ii) the plain FP64 per-slice method: the same Parareal with
    every slice propagated by its own launches (a plan of max_batch 1; batch
    invariance makes its iterates bitwise those of the batched run, checked
    on its first iterations, whose time per iteration is carried over to the
    batched run's iteration count)."""
    import numpy as np
    import torch
    from paper_2306_09497_amd import pint, workloads

    Mc, nlon, nlat, N = 127, 384, 192, 64
    fine = pint.stepper(30.0, 2, 0.0, pint.T_ALL)
    conv = pint.stepper(100.0, 2, 0.0, pint.T_ALL)
    spec = pint.stepper(900.0, 4, 1.0e17, pint.T_ALL)
    prm = pint.params(pint.PARAREAL, N, fine, 180, conv, 54, max_iter=N, tol=1e-8)
    torch.cuda.init()
    plans = {b: pint.Plan(Mc, nlon, nlat, phibar=PHIBAR, max_batch=b) for b in (N, 1)}
    pl = plans[N]
    for p_ in plans.values():
        p_.reserve(prm)
    mu, _ = pl.grid_coords()
    G = workloads.jet_bump_grid(mu, nlon, phibar=PHIBAR, **workloads.jet_bump_params(0))
    grid = torch.from_numpy(np.ascontiguousarray(G)).cuda()
    u0 = torch.zeros((1, 3, pl.ncoef, 2), dtype=torch.float64, device="cuda")
    pl.analysis(grid, u0, 3)
    # (i) serial fine, every slice boundary kept
    ref = torch.zeros((N + 1, 3, pl.ncoef, 2), dtype=torch.float64, device="cuda")
    ref[0] = u0[0]
    u = u0.clone()
    plans[1].step(fine, u, u, 1, 180)                    # warm-up (code)
    u.copy_(u0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for n in range(N):
        plans[1].step(fine, u, u, 1, 180)
        ref[n + 1] = u[0]
    torch.cuda.synchronize()
    t_ref = time.perf_counter() - t0
    rf = ref[N].cpu().numpy()
    phr = rf[0, :, 0] + 1j * rf[0, :, 1]

    def errors(slices):
        d = pl.rel_diff(slices[1:], ref[1:], N)          # [N][4] vs serial fine
        fin = slices[N].cpu().numpy()
        return {"E_phi_32_final": e_phi_r(fin[0, :, 0] + 1j * fin[0, :, 1], phr, Mc),
                "max_rel_l2_phi_prime": float(d[:, 0].max()),
                "max_rel_l2_wind": float(d[:, 3].max())}

    out = {"config": "T127 384x192, 64 slices x 5400 s (4 days), fine IMEX 30 s x 180, coarse "
                     "IMEX 100 s x 54 without viscosity, jet + bump, Parareal to increment 1e-8 "
                     "(cap 64 = N)",
           "serial_fine_s": t_ref, "serial_fine_steps": N * 180}
    slices = torch.zeros((N + 1, 3, pl.ncoef, 2), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, rep, msg = pl.solve_status(prm, u0, slices)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    iters = rep.iters
    out["parareal_batched"] = {
        "status": st, "iters": iters, "seconds": el, "time_to_tol_vs_serial_fine": el / t_ref,
        "speedup_vs_serial_fine": t_ref / el, "fine_slice_steps": rep.fine_slice_steps,
        "fine_slice_steps_per_s": rep.fine_slice_steps / el,
        "increments": [rep.incr[i] for i in range(iters)], **errors(slices)}
    # (ii) per-slice launches: the first iterations, timed, and bitwise the
    # batched run's iterates at that count
    k = min(per_slice_iters, iters)
    short = pint.params(pint.PARAREAL, N, fine, 180, conv, 54, max_iter=k)
    a = torch.zeros_like(slices)
    b = torch.zeros_like(slices)
    pl.solve(short, u0, a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rp = plans[1].solve(short, u0, b)
    torch.cuda.synchronize()
    el1 = time.perf_counter() - t0
    # a Parareal iteration k recomputes N - k slices: scale by the work
    work_k = sum(N - i for i in range(k))
    work_all = sum(N - i for i in range(iters))
    t_ps = el1 * work_all / work_k
    out["parareal_per_slice"] = {
        "iterations_timed": k, "seconds_timed": el1, "seconds_extrapolated": t_ps,
        "iterates_bitwise_equal_to_batched": bool(torch.equal(a, b)),
        "note": "time of the first iterations scaled by the fine work of the batched run's "
                "iteration count (iteration k recomputes N - k slices)"}
    out["batched_vs_per_slice_speedup"] = t_ps / el
    # the coarse level as specified for C2: increments of its first iterations
    q2 = pint.params(pint.PARAREAL, N, fine, 180, spec, 6, max_iter=8)
    s2 = torch.zeros_like(slices)
    r2 = pl.solve(q2, u0, s2)
    out["c2_specified_coarse_increments"] = {
        "coarse": "IMEX 900 s x 6, q=4, nu=1e17",
        "increments": [r2.incr[i] for i in range(r2.iters)]}
    for p_ in plans.values():
        p_.close()
    return out


def measure(precision, steps, warmup, levels=2, coarse_grid=None, coarse_precision=None):
    """Time `steps` MGRIT iterations at the given Legendre precision (levels 2,
    or 3 with level-2 points every CFACTOR level-1 points, one level-2 step of
    CFACTOR * DT_COARSE, two cycles on levels 1 and 2 per iteration); return
    the throughput, the per-kernel profile of the batched transform kernels,
    the increments and the slice states after warmup + steps + 2 iterations
    (two more iterations time the Legendre GEMMs).
    coarse_grid = (Mc, nlon, nlat): coarse level on a plan of that truncation
    (spatial coarsening); coarse_precision: the coarse plan's transform
    precision (default: the fine plan's)."""
    import numpy as np
    import torch
    from paper_2306_09497_amd import pint, workloads

    plan = pint.Plan(M, NLON, NLAT, phibar=PHIBAR, max_batch=GROUP, precision=precision)
    # synthetic jet + bump initial state, analysed on the device
    mu, _ = plan.grid_coords()
    G = workloads.jet_bump_grid(mu, NLON, phibar=PHIBAR, **workloads.jet_bump_params(0))
    grid = torch.from_numpy(np.ascontiguousarray(G)).cuda()
    u0 = torch.zeros((1, 3, plan.ncoef, 2), dtype=torch.float64, device="cuda")
    plan.analysis(grid, u0, 3)
    slices = torch.zeros((GROUP + 1, 3, plan.ncoef, 2), dtype=torch.float64, device="cuda")
    fine = pint.stepper(DT_FINE, 2, 0.0, pint.T_ALL)
    coarse = pint.stepper(DT_COARSE, Q_COARSE, NU_COARSE, pint.T_ALL)
    extra = {}
    cplan = None
    if coarse_grid is not None:
        cplan = pint.Plan(*coarse_grid, phibar=PHIBAR, max_batch=GROUP,
                          precision=precision if coarse_precision is None else coarse_precision)
        extra["coarse_plan"] = cplan
    if levels == 3:
        extra.update(levels=3, cfactor1=CFACTOR, coarse2_steps=1, cycles1=2,
                     coarse2=pint.stepper(DT_COARSE * CFACTOR, Q_COARSE, NU_COARSE, pint.T_ALL))
    # the timed iterations are one solve of `steps` iterations resumed from
    # the warmed-up iterate (with two levels the relaxation of each iteration
    # after the first then runs beside the previous iteration's sweep)
    it = pint.params(pint.MGRIT, GROUP, fine, CFACTOR, coarse, 1, nrelax=1, max_iter=steps,
                     resume=True, **extra)
    plan.reserve(it)            # scratch and factors allocated, GEMM launch shapes tuned
    plan.solve(pint.params(pint.MGRIT, GROUP, fine, CFACTOR, coarse, 1, nrelax=1, max_iter=0,
                           coarse_plan=cplan), u0, slices)     # initial coarse sweep
    if warmup > 0:
        plan.solve(pint.params(pint.MGRIT, GROUP, fine, CFACTOR, coarse, 1, nrelax=1,
                               max_iter=warmup, resume=True, **extra), u0, slices)
    torch.cuda.synchronize()

    # timed region: exactly `steps` MGRIT iterations; the batched launches (two
    # states or more) of the dominant kernel, the ring, are bracketed by HIP
    # events (on the streams they run on)
    plan.profile(["ring_tendency"], min_batch=2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rep = plan.solve(it, u0, slices)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    fine_steps = rep.fine_slice_steps
    incr = [rep.incr[i] for i in range(rep.iters)]
    prof = plan.profile_read()
    # the Legendre GEMMs' launches, timed the same way in two more iterations
    # after the timed region (events on every launch slow the iteration)
    plan.profile(["legendre_synth", "legendre_anal"], min_batch=2)
    plan.solve(pint.params(pint.MGRIT, GROUP, fine, CFACTOR, coarse, 1, nrelax=1, max_iter=2,
                           resume=True, **extra), u0, slices)
    torch.cuda.synchronize()
    prof.update(plan.profile_read())
    plan.profile([])
    info = plan.info()
    names = {(0, 0): ["k-slab 16", "k-slab 32"], (1, 0): ["k-slab 16", "k-slab 32"],
             (0, 1): ["64 columns", "128 columns"],
             (1, 1): ["64 columns", "64 columns, k-slab 32", "128 columns"]}
    shapes = {}
    for (k, c), label in (((0, 0), "synthesis_1_state"), ((0, 1), "synthesis_64_states"),
                          ((1, 0), "analysis_1_state"), ((1, 1), "analysis_64_states")):
        v = info.gemm_shape[k][c]
        shapes[label] = {"shape": names[(k, c)][v] if v < len(names[(k, c)]) else v,
                         "tuned_us_per_launch": info.gemm_us[k][c]}
    for c, label in ((0, "ring_1_state"), (1, "ring_64_states")):
        shapes[label] = {"workgroup_threads": info.ring_threads[c],
                         "tuned_us_per_launch": info.ring_us[c]}
    plan.close()
    if cplan is not None:
        cplan.close()
    elapsed = t1 - t0
    return {"value": fine_steps / elapsed, "elapsed": elapsed, "fine_steps": fine_steps,
            "prof": prof, "incr": incr, "slices": slices, "gemm_shapes": shapes}


def measure_diagnostics(slices, reps=20):
    """Time the device diagnostics over the GROUP slice states (the states of
    slices 1..GROUP against those of 0..GROUP-1): KE spectrum, E_{psi,R} for
    every R, physical-space L2 errors.  Algorithmic bytes: every coefficient
    read once (complex128)."""
    import torch
    from paper_2306_09497_amd import pint

    plan = pint.Plan(M, NLON, NLAT, phibar=PHIBAR, max_batch=GROUP)
    u = slices[1:].contiguous()
    ref = slices[:-1].contiguous()
    B = u.shape[0]
    e = torch.zeros((B, M + 1), dtype=torch.float64, device="cuda")
    es = torch.zeros((B, 3, M + 1), dtype=torch.float64, device="cuda")
    calls = {
        "ke_spectrum": (lambda: plan.ke_spectrum(u, e, B), B * 2 * plan.ncoef * 16),
        "spectral_errors": (lambda: plan.spectral_errors(u, ref, es, B),
                            B * 2 * 3 * plan.ncoef * 16),
        "grid_l2_errors": (lambda: plan.grid_l2_errors(u, ref, B), None),
    }
    out = {}
    for name, (fn, byts) in calls.items():
        fn()
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(reps):
            fn()
        t1.record()
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1) / reps
        out[name] = {"states": B, "ms_per_call": ms}
        if byts is not None:
            out[name]["gbps_algorithmic"] = byts / (ms * 1e-3) / 1e9
            out[name]["hbm_frac"] = byts / (ms * 1e-3) / PEAK_HBM
    out["grid_l2_errors"]["note"] = ("scalar synthesis of 6 fields per state (difference and "
                                     "reference) and per-ring sums of squares; synchronises")
    plan.close()
    # stability map (Sec. 4): two-level MGRIT (nu = 1) with an SL-SI-SETTLS
    # coarse scheme, 21 phases x 2 roots per point, on a 2048 x 2048 grid
    smap = torch.zeros((2048, 2048), dtype=torch.float64, device="cuda")
    run = lambda: pint.stability_map(smap, "mgrit", "settls", 0.248j, (-2.0, 0.5), (-3.0, 3.0),
                                     n=100, k=5, cfactor=2, n_c=1, nrelax=1, n_ks=20)
    run()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(5):
        run()
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / 5
    out["stability_map"] = {"points": smap.numel(), "ms_per_call": ms,
                            "points_per_s": smap.numel() / (ms * 1e-3),
                            "stable_fraction": float((smap <= 1.0).double().mean())}
    return out


def measure_sl(reps=10):
    """SL-SI-SETTLS coarse steps (Sec. 2.3.2) at T127 (384 x 192), dt = 1800 s,
    second-order viscosity 1e5, two trajectory iterations: the coarse
    configuration of the paper's SL runs.  Three steps per call (one slice),
    the first in the one-step variant; batches of 5 instances and of 1 (the
    serial sweep).  Grid-point kernels: algorithmic bytes per arrival point
    and state = 17 doubles for the right-hand-side fields (10 read, 7
    written) + 14 for the trajectories (4 arrival values, 7 gathered fields
    once, 3 written)."""
    import numpy as np
    import torch
    from paper_2306_09497_amd import pint, workloads

    Mc, nlon, nlat = 127, 384, 192
    plan = pint.Plan(Mc, nlon, nlat, phibar=PHIBAR, max_batch=10)
    mu, _ = plan.grid_coords()
    grids = [workloads.jet_bump_grid(mu, nlon, phibar=PHIBAR, **workloads.jet_bump_params(i))
             for i in range(5)]
    grid = torch.from_numpy(np.ascontiguousarray(np.stack(grids))).cuda()
    u = torch.zeros((5, 3, plan.ncoef, 2), dtype=torch.float64, device="cuda")
    plan.analysis(grid, u, 15)                       # 5 states x 3 fields
    st = pint.sl_stepper(1800.0, 2, 2, 1.0e5)
    imex = pint.stepper(1800.0, 2, 1.0e5, pint.T_ALL)
    out = {}
    o = torch.empty_like(u)
    for B in (5, 1):
        plan.sl_steps(st, u[:B], o[:B], B, 3)
        torch.cuda.synchronize()
        plan.profile(["sl_points"], min_batch=B)
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(reps):
            plan.sl_steps(st, u[:B], o[:B], B, 3)
        t1.record()
        torch.cuda.synchronize()
        prof = plan.profile_read()
        plan.profile([])
        ms = t0.elapsed_time(t1) / (3 * reps)
        rec = {"ms_per_step": ms, "state_steps_per_s": B / (ms * 1e-3)}
        pk = prof.get(("sl_points", B))
        if pk:
            pms = pk[1] / pk[0]
            byts = (17 + 14) * 8.0 * nlat * nlon * B
            rec["grid_point_kernels_ms"] = pms
            rec["grid_point_gbps_algorithmic"] = byts / (pms * 1e-3) / 1e9
        plan.step(imex, u[:B], o[:B], B, 3)
        torch.cuda.synchronize()
        t0.record()
        for _ in range(reps):
            plan.step(imex, u[:B], o[:B], B, 3)
        t1.record()
        torch.cuda.synchronize()
        rec["imex_ms_per_step_same_dt"] = t0.elapsed_time(t1) / (3 * reps)
        out["B%d" % B] = rec
    out["config"] = "T127 384x192, dt 1800 s, q 2, nu 1e5, 2 trajectory iterations"
    # Parareal with the SL coarse propagator (Sec. 3.1, C4 shape): 64 slices
    # of 4 days / 64, fine IMEX 30 s x 180 per slice, coarse SL 1800 s x 3;
    # one instance, and the five instances together
    fplan = pint.Plan(Mc, nlon, nlat, phibar=PHIBAR, max_batch=64)
    fine = pint.stepper(30.0, 2, 0.0, pint.T_ALL)
    N = 64
    for I in (1, 5):
        slices = torch.zeros((N + 1, I, 3, plan.ncoef, 2), dtype=torch.float64, device="cuda")
        times = {}
        for it in (0, 0, 2):
            t0 = torch.cuda.Event(enable_timing=True)
            t1 = torch.cuda.Event(enable_timing=True)
            t0.record()
            fplan.parareal_sl(fine, 180, st, 3, N, it, u[:I], slices, n_inst=I, coarse_plan=plan)
            t1.record()
            torch.cuda.synchronize()
            times[it] = t0.elapsed_time(t1)
        per_it = (times[2] - times[0]) / 2
        out["parareal_sl_t127" + ("" if I == 1 else "_x%d" % I)] = {
            "instances": I, "slices": N, "fine_steps_per_slice": 180,
            "coarse_sl_steps_per_slice": 3,
            "initial_coarse_sweep_ms": times[0], "ms_per_iteration": per_it,
            # iterations 0 and 1 recompute 64 and 63 slices of every instance
            "fine_slice_steps_per_s": I * (2 * N - 1) * 180 / ((times[2] - times[0]) * 1e-3),
            "finite": bool(torch.isfinite(slices).all()),
        }
    # convergence of the SL-coarse Parareal (the paper's stability question
    # for this coarse scheme): largest relative increment over the slices of
    # Phi' and of the wind, iterations 1..4 against the iterate before
    for nu, key in ((1.0e5, "increments_phi_wind"), (1.0e6, "increments_phi_wind_nu1e6")):
        stn = pint.sl_stepper(1800.0, 2, 2, nu)
        prev = None
        incr = []
        for it in range(5):
            sl_k = torch.zeros((N + 1, 3, plan.ncoef, 2), dtype=torch.float64, device="cuda")
            fplan.parareal_sl(fine, 180, stn, 3, N, it, u[:1], sl_k, coarse_plan=plan)
            if prev is not None:
                d = fplan.rel_diff(sl_k, prev, N + 1)
                incr.append([float(d[:, 0].max()), float(d[:, 3].max())])
            prev = sl_k
        out["parareal_sl_t127"][key] = incr
    fplan.close()
    plan.close()
    return out


def serve_bench(seconds, rate, max_iter=2, seed=0, steps_per_tick=8, arena_gb=96.0,
                precision=0, tol=0.0, max_batch=GROUP, stage_states=2 * GROUP):
    """Serving with continuous batching: Poisson arrivals (rate per second for
    `seconds`) of Parareal or two-level MGRIT (FCF) requests, uniform over
    T63 192x96 / T127 384x192 / T255 768x384, 16/32/64/128 slices and 1-4 day
    horizons; fine IMEX 45 s, coarse IMEX 675 s with q = 4 and nu scaled
    with (n(n+1))^-2 from the paper's 1e17 m^4/s for IMEX coarse levels at
    T127 (T63 1.6e18, T127 1e17, T255 6.25e15; weaker values leave the 675 s
    coarse step unstable for the jet), max_iter iterations each; jet + bump initial states (amplitude U[60, 160] m, seeded
    bump longitude).  Requests are submitted at the tick after their arrival
    time; latency = completion - arrival.  precision: the plans' transform
    precision (0 FP64, 1 FP32 Legendre); tol > 0: each request stops at that
    increment (at most max_iter iterations)."""
    import numpy as np
    import torch
    from paper_2306_09497_amd import pint, workloads

    grids = [(63, 192, 96, 1.6e18), (127, 384, 192, 1.0e17), (255, 768, 384, 6.25e15)]
    plans = [pint.Plan(Mg, nl, nt, phibar=PHIBAR, max_batch=max_batch, precision=precision)
             for Mg, nl, nt, _ in grids]
    rng = np.random.default_rng(seed)
    # a few analysed initial states per truncation, made before timing
    init = []
    for pl, (Mg, nl, nt, _) in zip(plans, grids):
        mu, _ = pl.grid_coords()
        us = []
        for v in range(3):
            G = workloads.jet_bump_grid(mu, nl, phibar=PHIBAR, amp=float(rng.uniform(60, 160)),
                                        lam_c=float(rng.uniform(0, 2 * math.pi)))
            g = torch.from_numpy(np.ascontiguousarray(G)).cuda()
            u = torch.zeros((1, 3, pl.ncoef, 2), dtype=torch.float64, device="cuda")
            pl.analysis(g, u, 3)
            us.append(u)
        init.append(us)
    reqs = []
    t = 0.0
    while True:
        t += rng.exponential(1.0 / rate)
        if t > seconds:
            break
        gi = int(rng.integers(3))
        S = int(rng.choice([16, 32, 64, 128]))
        days = int(rng.integers(1, 5))
        span = days * 86400.0 / S
        fs, cs = int(round(span / 45.0)), int(round(span / 675.0))
        if cs < 1 or abs(fs * 45.0 - span) > 1e-6 or abs(cs * 675.0 - span) > 1e-6:
            continue                       # (every combination divides exactly)
        method = int(rng.integers(2))
        prm = pint.params(method, S, pint.stepper(45.0, 2, 0.0, pint.T_ALL), fs,
                          pint.stepper(675.0, 4, grids[gi][3], pint.T_ALL), cs,
                          nrelax=method, max_iter=max_iter, tol=tol)
        reqs.append((t, gi, prm, int(rng.integers(3))))
    # the plans ready for every stepper pair the requests use (factor sets,
    # GEMM launch shapes), so nothing is allocated or tuned while serving
    for pl, (_, _, _, nu) in zip(plans, grids):
        pl.reserve(pint.params(pint.MGRIT, 16, pint.stepper(45.0, 2, 0.0, pint.T_ALL), 120,
                               pint.stepper(675.0, 4, nu, pint.T_ALL), 8, nrelax=1, max_iter=1))
    srv = pint.Server(plans, int(arena_gb * 2**30), steps_per_tick=steps_per_tick,
                      stage_states=stage_states)
    torch.cuda.synchronize()
    ids, outs = [], []
    t0 = srv.clock()
    nxt, pending = 0, 1
    while nxt < len(reqs) or pending:
        now = srv.clock() - t0
        while nxt < len(reqs) and reqs[nxt][0] <= now:
            _, gi, prm, v = reqs[nxt]
            out = torch.empty((prm.n_intervals + 1, 3, plans[gi].ncoef, 2), dtype=torch.float64,
                              device="cuda")
            ids.append(srv.submit(gi, prm, init[gi][v][0], out))
            outs.append(out)
            nxt += 1
        pending = srv.tick()
        if nxt < len(reqs) and not pending:
            time.sleep(max(0.0, min(0.01, reqs[nxt][0] - (srv.clock() - t0))))
    makespan = srv.clock() - t0
    st = [srv.status(i) for i in ids]
    srv.close()
    for pl in plans:
        pl.close()
    lat = np.array([s.t_done - t0 - r[0] for s, r in zip(st, reqs)])
    queue = np.array([s.t_start - t0 - r[0] for s, r in zip(st, reqs)])
    service = np.array([s.t_done - s.t_start for s in st])
    work = sum(s.fine_slice_steps for s in st)
    per = {}
    for (_, gi, _, _), l in zip(reqs, lat):
        per.setdefault(grids[gi][0], []).append(l)
    return {
        "metric": "served fine slice-steps/s (continuous batching)",
        "value": work / makespan, "unit": "slice-steps/s", "n_gpus": 1,
        "requests": len(reqs), "completed": sum(s.state == pint.REQ_DONE for s in st),
        "diverged": sum(s.state == pint.REQ_FAILED for s in st),
        "arrival_window_s": seconds, "rate_per_s": rate, "makespan_s": makespan,
        "offered_fine_slice_steps_per_s": work / seconds,
        "achieved_fine_slice_steps_per_s": work / makespan,
        "latency_p50_s": float(np.percentile(lat, 50)),
        "latency_p99_s": float(np.percentile(lat, 99)),
        "queue_mean_s": float(queue.mean()), "service_mean_s": float(service.mean()),
        "latency_p50_by_truncation_s": {f"T{k}": float(np.percentile(v, 50))
                                        for k, v in sorted(per.items())},
        "iterations_mean": float(np.mean([s.iters for s in st])),
        "not_converged": sum(s.status == -5 for s in st),
        "config": {"workload": "Poisson arrivals, uniform T63/T127/T255, S in {16,32,64,128}, "
                               "1-4 days, fine 45 s, coarse 675 s, Parareal or MGRIT FCF, "
                               + (f"stop at increment {tol:g} (at most {max_iter} iterations)"
                                  if tol > 0 else f"{max_iter} iterations"),
                   "steps_per_tick": steps_per_tick, "max_batch": max_batch,
                   "stage_states": stage_states,
                   "legendre_precision": ["fp64", "fp32"][precision]},
        "data": "synthetic", "dtype": "f64" if precision == 0 else "f64 state, f32 transforms",
    }


def serve_c5(seconds=1.5, rate=20.0, max_iter=3, tol=1e-6):
    """The serving workload at its configured arrival rate (20/s) for a short
    window, in the north-star's mixed precision (FP32 Legendre plans) with
    each request stopping at an increment of tol (at most max_iter
    iterations), against the plain FP64 per-slice method on the same request
    stream: FP64 plans of max_batch 1 whose launches are never merged (one
    state per staging buffer), the same stopping rule."""
    merged = serve_bench(seconds, rate, max_iter=max_iter, precision=1, tol=tol)
    plain = serve_bench(seconds, rate, max_iter=max_iter, precision=0, tol=tol, max_batch=1,
                        stage_states=1)
    keep = ("requests", "completed", "diverged", "not_converged", "makespan_s",
            "offered_fine_slice_steps_per_s", "achieved_fine_slice_steps_per_s",
            "latency_p50_s", "latency_p99_s", "queue_mean_s", "service_mean_s",
            "latency_p50_by_truncation_s", "iterations_mean")
    return {"arrival_window_s": seconds, "rate_per_s": rate,
            "stopping": f"increment <= {tol:g}, at most {max_iter} iterations",
            "fp32_legendre_merged": {k: merged[k] for k in keep},
            "fp64_per_slice": {k: plain[k] for k in keep},
            "p99_ratio_per_slice_over_merged": plain["latency_p99_s"] / merged["latency_p99_s"],
            "throughput_ratio_merged_over_per_slice": (merged["achieved_fine_slice_steps_per_s"]
                                                       / plain["achieved_fine_slice_steps_per_s"])}


def c3_full_horizon(iters=2):
    """C3 at its stated horizon: two days at T255 (768x384), fine IMEX 45 s,
    960 C-intervals of cfactor 4 (15 slice groups of 64), coarse IMEX 180 s
    with q = 4, nu = 1e17; two-level MGRIT FCF over all 960 intervals (a
    959-step serial sweep), `iters` iterations after the initial coarse
    sweep, in one pint_solve call."""
    import numpy as np
    import torch
    from paper_2306_09497_amd import pint, workloads

    N = 960
    plan = pint.Plan(M, NLON, NLAT, phibar=PHIBAR, max_batch=GROUP)
    mu, _ = plan.grid_coords()
    G = workloads.jet_bump_grid(mu, NLON, phibar=PHIBAR, **workloads.jet_bump_params(0))
    grid = torch.from_numpy(np.ascontiguousarray(G)).cuda()
    u0 = torch.zeros((1, 3, plan.ncoef, 2), dtype=torch.float64, device="cuda")
    plan.analysis(grid, u0, 3)
    fine = pint.stepper(DT_FINE, 2, 0.0, pint.T_ALL)
    coarse = pint.stepper(DT_COARSE, Q_COARSE, NU_COARSE, pint.T_ALL)
    q = pint.params(pint.MGRIT, N, fine, CFACTOR, coarse, 1, nrelax=1, max_iter=iters)
    footprint = plan.workspace_query(q)
    plan.reserve(q)
    slices = torch.zeros((N + 1, 3, plan.ncoef, 2), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rep = plan.solve(q, u0, slices)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    it_s = [rep.seconds[i] for i in range(rep.iters)]
    out = {"config": "T255 768x384, 2 days, 960 C-intervals x cfactor 4, fine 45 s, coarse 180 s "
                     "q=4 nu=1e17, MGRIT FCF, one solve call",
           "iterations": rep.iters, "seconds_total": el, "seconds_per_iteration": it_s,
           "initial_sweep_s": el - sum(it_s),
           "fine_slice_steps_per_s_in_iterations": (rep.fine_slice_steps / sum(it_s)),
           "increments": [rep.incr[i] for i in range(rep.iters)],
           "device_footprint_gb": footprint / 1e9, "finite": bool(torch.isfinite(slices).all())}
    plan.close()
    return out


def field_errors(a, b):
    """Per-field relative L2 difference (Phi', xi, delta) of two (N, 3, ncoef, 2)
    device tensors over all slices."""
    import torch
    d = (a - b).double()
    out = {}
    for f, name in enumerate(("phi", "xi", "delta")):
        ref = b[:, f].clone()
        if f == 0:
            ref[:, 0, 0] = 0.0                     # Phi without its mean
        out[name] = float(torch.linalg.vector_norm(d[:, f]) / torch.linalg.vector_norm(ref))
    return out


_T_START = time.perf_counter()


def progress(what):
    """One line per finished leg on stderr (the JSON line stays on stdout)."""
    print(f"[bench] {what} ({time.perf_counter() - _T_START:.0f} s)", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-seconds", type=float, default=8.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision", choices=["fp64", "fp32", "bf16x3"], default="fp64",
                    help="transform precision of the headline (fp32: FP32 Legendre GEMMs, "
                         "Fourier rows and tendencies; bf16x3: the same with split-BF16 "
                         "GEMM products; state and solves FP64 in both)")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the FP32-Legendre side measurement of the default run")
    ap.add_argument("--no-mgrit3", action="store_true",
                    help="skip the three-level MGRIT side measurement of the default run")
    ap.add_argument("--no-diagnostics", action="store_true",
                    help="skip the diagnostics and stability-map timings of the default run")
    ap.add_argument("--no-sl", action="store_true",
                    help="skip the SL-SI-SETTLS coarse-step timing of the default run")
    ap.add_argument("--time-to-tol", action="store_true",
                    help="print the T127 Parareal time-to-tolerance measurement instead")
    ap.add_argument("--no-time-to-tol", action="store_true",
                    help="skip the T127 time-to-tolerance leg of the default run")
    ap.add_argument("--no-serve", action="store_true",
                    help="skip the bounded serving leg (20/s arrivals) of the default run")
    ap.add_argument("--no-c3-full", action="store_true",
                    help="skip the two-day, 960-interval MGRIT leg of the default run")
    ap.add_argument("--serve", type=float, nargs=2, metavar=("SECONDS", "RATE"),
                    help="print the continuous-batching serving measurement instead "
                         "(Poisson arrivals at RATE per second for SECONDS)")
    ap.add_argument("--serve-fp32", action="store_true",
                    help="serving with FP32-Legendre plans, each request stopping at an "
                         "increment of 1e-6 (at most 8 iterations)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build runs the whole PinT problem on a "
              "single MI355X (time slices are the batch dimension); --gpus must be 1.",
              file=sys.stderr)
        return 2
    if args.serve:
        kw = dict(precision=1, tol=1e-6, max_iter=8) if args.serve_fp32 else {}
        print(json.dumps(serve_bench(args.serve[0], args.serve[1], **kw)), flush=True)
        return 0
    if args.time_to_tol:
        print(json.dumps({"metric": "PinT time-to-tol vs serial fine", **time_to_tol()}),
              flush=True)
        return 0

    import torch
    from paper_2306_09497_amd import pint

    torch.cuda.init()
    prec = {"fp64": pint.FP64, "fp32": pint.LEG_FP32, "bf16x3": pint.LEG_BF16X3}[args.precision]
    res = measure(prec, args.steps, args.warmup)
    progress("headline")
    prof, elapsed, fine_steps, value = res["prof"], res["elapsed"], res["fine_steps"], res["value"]
    incr = res["incr"]
    peak_mfma = {pint.FP64: PEAK_FP64, pint.LEG_FP32: PEAK_FP32,
                 pint.LEG_BF16X3: PEAK_BF16 / 3.0}[prec]

    # dominant kernel of the timed region and its roofline
    # (the largest launches of the iteration: states per batched launch)
    bmax = max(b for (_, b) in prof)
    per_kind = {}
    for (kind, b), (n, ms) in prof.items():
        if b == bmax:
            per_kind[kind] = (n, ms)
    dom = max(per_kind, key=lambda k: per_kind[k][1])
    n_launch, tot_ms = per_kind[dom]
    avg_s = tot_ms / n_launch * 1e-3
    flops, byts = algorithmic_work(dom, bmax, prec)
    if flops > 0:
        roof = {"bound": "mfma", "achieved": flops / avg_s / 1e12, "peak": peak_mfma / 1e12,
                "unit": "TFLOP/s"}
    else:
        roof = {"bound": "hbm", "achieved": byts / avg_s / 1e9, "peak": PEAK_HBM / 1e9,
                "unit": "GB/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = measured_traffic(dom, prec, bmax)
    roof["kernel"] = dom
    roof["states_per_launch"] = bmax
    roof["avg_launch_ms"] = tot_ms / n_launch

    kernels = {}
    for kind, (n, ms) in sorted(per_kind.items()):
        f, b = algorithmic_work(kind, bmax, prec)
        avg = ms / n * 1e-3
        kernels[kind] = {"launches": n, "avg_ms": ms / n,
                         "share_of_step": ms * 1e-3 / elapsed,
                         "tflops": f / avg / 1e12 if f else None,
                         "gbps_algorithmic": b / avg / 1e9}

    out = {
        "metric": "fine slice-steps/s at T255",
        "value": value,
        "unit": "slice-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {pint.FP64: "f64", pint.LEG_FP32: "f32+f64",
                  pint.LEG_BF16X3: "bf16x3+f32+f64"}[prec],
        "data": "synthetic",
        "config": {
            "workload": "T255 768x384, two-level MGRIT FCF iteration over one slice group: "
                        "64 C-intervals x cfactor 4, fine IMEX dt 45 s, coarse IMEX dt 180 s "
                        "with q=4 nu=1e17, jet + height bump initial state",
            "truncation": M, "nlon": NLON, "nlat": NLAT, "batch": GROUP,
            "fine_slice_steps_per_step": fine_steps // args.steps,
            "parallelism": "time slices as the batch dimension, 1 GPU",
        },
        "roofline": roof,
        "kernels": kernels,
        "gemm_shapes": res["gemm_shapes"],
        "mgrit_increment": incr,
    }
    if prec == pint.FP64 and not args.no_mixed:
        # the same iterations in the mixed-precision modes (FP32 Fourier rows
        # and tendencies; FP32 or split-BF16 Legendre GEMM products):
        # throughput and per-field difference of all slice states from the
        # FP64 path after warmup + steps + 2 iterations
        mixed = {}
        for name, mode in (("fp32_legendre", pint.LEG_FP32),
                           ("bf16x3_legendre", pint.LEG_BF16X3)):
            rm = measure(mode, args.steps, args.warmup)
            mixed[name] = {
                "value": rm["value"], "unit": "slice-steps/s",
                "ms_per_step": rm["elapsed"] / args.steps * 1e3,
                "speedup_vs_fp64": rm["value"] / value,
                "rel_l2_vs_fp64_path": field_errors(rm["slices"], res["slices"]),
                "iterations_compared": args.warmup + args.steps + 2,
            }
            del rm
            progress(name)
        out["mixed_precision"] = mixed
    if prec == pint.FP64 and not args.no_mgrit3:
        # the same slice group with three MGRIT levels: the level-1 problem by
        # two cycles on levels 1 and 2 instead of the serial sweep
        try:
            r3 = measure(pint.FP64, args.steps, args.warmup, levels=3)
            out["mgrit3"] = {
                "value": r3["value"], "unit": "slice-steps/s",
                "ms_per_step": r3["elapsed"] / args.steps * 1e3,
                "increment": r3["incr"],
                "config": "levels 3: level-2 point every 4 C-points (16 level-2 intervals), "
                          "level-2 step 720 s q=4 nu=1e17, FCF on levels 0 and 1, 2 cycles "
                          "on levels (1, 2) per iteration",
            }
        except Exception as e:                      # reported, not fatal
            out["mgrit3"] = {"error": str(e)}
        progress("mgrit3")
        # two levels with spatial coarsening: the coarse level at T127 (384x192)
        try:
            rc = measure(pint.FP64, args.steps, args.warmup, coarse_grid=(127, 384, 192))
            out["mgrit2_coarse_t127"] = {
                "value": rc["value"], "unit": "slice-steps/s",
                "ms_per_step": rc["elapsed"] / args.steps * 1e3,
                "increment": rc["incr"],
                "config": "two levels, coarse level at T127 on 384x192 (truncate, step, pad), "
                          "coarse dt 180 s q=4 nu=1e17",
            }
        except Exception as e:
            out["mgrit2_coarse_t127"] = {"error": str(e)}
        progress("mgrit2_coarse_t127")
        try:
            rc3 = measure(pint.FP64, args.steps, args.warmup, levels=3,
                          coarse_grid=(127, 384, 192))
            out["mgrit3_coarse_t127"] = {
                "value": rc3["value"], "unit": "slice-steps/s",
                "ms_per_step": rc3["elapsed"] / args.steps * 1e3,
                "increment": rc3["incr"],
                "config": "three levels as mgrit3, both coarse levels at T127 on 384x192",
            }
        except Exception as e:
            out["mgrit3_coarse_t127"] = {"error": str(e)}
        progress("mgrit3_coarse_t127")
        # two levels, coarse level at the fine truncation with FP32 transforms
        # (the fine propagator stays FP64, so the iteration converges to the
        # same FP64 fine solution)
        try:
            rf = measure(pint.FP64, args.steps, args.warmup, coarse_grid=(M, NLON, NLAT),
                         coarse_precision=pint.LEG_FP32)
            out["mgrit2_coarse_fp32"] = {
                "value": rf["value"], "unit": "slice-steps/s",
                "ms_per_step": rf["elapsed"] / args.steps * 1e3,
                "increment": rf["incr"],
                "rel_l2_vs_fp64_coarse": field_errors(rf["slices"], res["slices"]),
                "config": "two levels, coarse level at T255 with FP32 Legendre GEMMs and ring "
                          "(reduced precision on the coarse level only)",
            }
        except Exception as e:
            out["mgrit2_coarse_fp32"] = {"error": str(e)}
        progress("mgrit2_coarse_fp32")
    if prec == pint.FP64 and not args.no_diagnostics:
        try:
            out["diagnostics"] = measure_diagnostics(res["slices"])
        except Exception as e:                      # reported, not fatal
            out["diagnostics"] = {"error": str(e)}
        progress("diagnostics")
    if prec == pint.FP64 and not args.no_sl:
        try:
            out["sl_settls_t127"] = measure_sl()
        except Exception as e:                      # reported, not fatal
            out["sl_settls_t127"] = {"error": str(e)}
        progress("sl_settls_t127")
    if prec == pint.FP64 and not args.no_time_to_tol:
        try:
            out["time_to_tol_t127"] = time_to_tol()
        except Exception as e:                      # reported, not fatal
            out["time_to_tol_t127"] = {"error": str(e)}
        progress("time_to_tol_t127")
    if prec == pint.FP64 and not args.no_serve:
        try:
            out["serving_c5"] = serve_c5()
        except Exception as e:
            out["serving_c5"] = {"error": str(e)}
        progress("serving_c5")
    if prec == pint.FP64 and not args.no_c3_full:
        try:
            out["c3_full_horizon"] = c3_full_horizon()
        except Exception as e:
            out["c3_full_horizon"] = {"error": str(e)}
        progress("c3_full_horizon")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
        progress("cpu_baseline")
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
