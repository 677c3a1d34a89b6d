"""Small fixed workloads for hardware-counter runs (rocprofv3 --pmc).

    python -m paper_2306_09497_amd.profile_drivers tendency [B] [reps] [precision]
        N(U) of B T255 768x384 jet + bump states, `reps` times: one spectral
        prep, Legendre synthesis GEMM, ring FFT + tendency kernel, Legendre
        analysis GEMM and assembly per call (Sec. 2.2); precision 0 (FP64),
        1 (FP32 Legendre) or 2 (split-BF16 Legendre).
    python -m paper_2306_09497_amd.profile_drivers sl [B] [reps]
        `reps` calls of three SL-SI-SETTLS steps (Sec. 2.3.2) of B T127
        384x192 jet + bump states, dt 1800 s, q 2, nu 1e5.
    python -m paper_2306_09497_amd.profile_drivers copy [reps]
        a plain 1 GiB device-to-device copy, the calibration of FETCH_SIZE and
        WRITE_SIZE against a known byte count.
"""

import sys

M, NLON, NLAT = 255, 768, 384
PHIBAR = 9.80616e4


def tendency(B=64, reps=3, precision=0):
    import numpy as np
    import torch
    from paper_2306_09497_amd import pint, workloads

    plan = pint.Plan(M, NLON, NLAT, phibar=PHIBAR, max_batch=B, precision=precision)
    mu, _ = plan.grid_coords()
    G = workloads.jet_bump_grid(mu, NLON, phibar=PHIBAR, **workloads.jet_bump_params(0))
    grid = torch.from_numpy(np.ascontiguousarray(G)).cuda()
    u0 = torch.zeros((1, 3, plan.ncoef, 2), dtype=torch.float64, device="cuda")
    plan.analysis(grid, u0, 3)
    u = u0.repeat(B, 1, 1, 1).contiguous()
    out = torch.zeros_like(u)
    for _ in range(reps):
        plan.tendency(u, out, B)
    torch.cuda.synchronize()
    plan.close()
    print(f"tendency: {reps} calls of B={B} at T{M} {NLON}x{NLAT}, precision {precision}",
          flush=True)


def sl(B=5, reps=3):
    import numpy as np
    import torch
    from paper_2306_09497_amd import pint, workloads

    plan = pint.Plan(127, 384, 192, phibar=PHIBAR, max_batch=max(2, 2 * B))
    mu, _ = plan.grid_coords()
    G = workloads.jet_bump_grid(mu, 384, phibar=PHIBAR, **workloads.jet_bump_params(0))
    grid = torch.from_numpy(np.ascontiguousarray(G)).cuda()
    u0 = torch.zeros((1, 3, plan.ncoef, 2), dtype=torch.float64, device="cuda")
    plan.analysis(grid, u0, 3)
    u = u0.repeat(B, 1, 1, 1).contiguous()
    out = torch.zeros_like(u)
    st = pint.sl_stepper(1800.0, 2, 2, 1.0e5)
    for _ in range(reps):
        plan.sl_steps(st, u, out, B, 3)
    torch.cuda.synchronize()
    plan.close()
    print(f"sl: {reps} calls of 3 steps of B={B} at T127 384x192", flush=True)


def copy(reps=3):
    import torch

    n = 1 << 27                               # 2^27 doubles = 1 GiB
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(f"copy: {reps} x 1 GiB", flush=True)


if __name__ == "__main__":
    what = sys.argv[1] if len(sys.argv) > 1 else "tendency"
    args = [int(a) for a in sys.argv[2:]]
    if what == "tendency":
        tendency(*args)
    elif what == "sl":
        sl(*args)
    elif what == "copy":
        copy(*args)
    else:
        sys.exit(f"unknown workload {what!r}: tendency | sl | copy")
