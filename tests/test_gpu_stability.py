"""GPU parity of the stability maps (Sec. 4) against the oracle: the schemes
alone (IMEX, SL-SI-SETTLS over phases and roots) and Parareal / two-level
MGRIT with either coarse scheme."""

import cmath
from math import comb

import numpy as np
import pytest

from oracle.stability import imex_amp, settls_roots, stability_map

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2306_09497_amd import pint  # noqa: E402

XI_L = 4.96e-5j            # i sqrt(Phibar / a^2) with Phibar = 1e5


def grid(lo, hi, n):
    """The device's grid formula: lo + j (hi - lo) / (n - 1)."""
    step = (hi - lo) / (n - 1)
    return [lo + j * step for j in range(n)]


def term_scale(kind, coarse, xl, re, im, n, k, cf, nc, nu, n_ks):
    """Largest sum of |terms| over roots and phases per point: the scale of
    the rounding of the MGRIT sum."""
    out = np.zeros((len(im), len(re)))
    for r, y in enumerate(im):
        for c, x in enumerate(re):
            xn = complex(x, y)
            if coarse == "imex":
                amps = [imex_amp(xl, xn)]
            else:
                amps = [a for j in range(n_ks + 1)
                        for a in settls_roots(xl, xn, 2.0 * cmath.pi * j / n_ks)]
            if kind == "scheme":
                out[r, c] = max(abs(a) for a in amps)
                continue
            F = imex_amp(xl / cf, xn / cf) ** (cf * nc)
            best = 0.0
            for a in amps:
                R = a ** nc
                S = F ** nu * (F - R)
                s = sum(comb(n - i * nu, i) * abs(S) ** i * abs(R) ** (n - i * (nu + 1))
                        for i in range(k + 1) if n - i * (nu + 1) >= 0)
                best = max(best, s)
            out[r, c] = best
    return out


CASES = [
    ("scheme", "imex", 1e4 * XI_L, (-2.0, 0.5, 41), (-3.0, 3.0, 33), 100, 5, 2, 1, 0),
    ("scheme", "settls", 1e4 * XI_L, (-2.0, 0.5, 41), (-3.0, 3.0, 33), 100, 5, 2, 1, 0),
    ("mgrit", "imex", 5e3 * XI_L, (-1.0, 0.2, 33), (-1.5, 1.5, 25), 100, 5, 2, 1, 0),
    ("mgrit", "imex", 1e4 * XI_L, (-1.0, 0.2, 33), (-1.5, 1.5, 25), 100, 5, 2, 1, 1),
    ("mgrit", "settls", 5e3 * XI_L, (-0.6, 0.1, 15), (-0.8, 0.8, 13), 100, 5, 2, 1, 1),
    ("mgrit", "settls", 0.0, (-0.6, 0.1, 15), (-0.8, 0.8, 13), 60, 10, 4, 2, 2),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}-{c[1]}-nu{c[9]}")
def test_stability_map(case):
    kind, coarse, xl, rr, ir, n, k, cf, nc, nu = case
    re, im = grid(*rr), grid(*ir)
    out = torch.full((ir[2], rr[2]), -1.0, dtype=torch.float64, device="cuda")
    pint.stability_map(out, kind, coarse, xl, rr[:2], ir[:2], n=n, k=k, cfactor=cf, n_c=nc,
                       nrelax=nu, n_ks=20)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    ref = np.array(stability_map(kind, coarse, xl, re, im, n=n, k=k, cfactor=cf, n_c=nc, nu=nu,
                                 n_ks=20))
    scale = term_scale(kind, coarse, xl, re, im, n, k, cf, nc, nu, 20)
    fin = np.isfinite(ref)
    assert np.array_equal(np.isfinite(got), fin)
    err = np.abs(got[fin] - ref[fin]) / np.maximum(scale[fin], 1e-300)
    print(f"{case[:2]} nu={nu}: max error / term scale = {err.max():.2e}, "
          f"stable points {int(np.sum(ref <= 1.0))}/{ref.size}", flush=True)
    assert err.max() < 1e-12
    # the stability region is decided the same way wherever it is not marginal
    clear = fin & (np.abs(ref - 1.0) > 1e-9 * np.maximum(scale, 1.0))
    assert np.array_equal(got[clear] <= 1.0, ref[clear] <= 1.0)


def test_stability_map_rejects():
    out = torch.zeros((4, 4), dtype=torch.float64, device="cuda")
    with pytest.raises(pint.PintError):
        pint.stability_map(out, "mgrit", "imex", 0.1j, (0, 1), (0, 1), k=65)
    with pytest.raises(pint.PintError):
        pint.stability_map(out, "scheme", "settls", 0.1j, (0, 1), (0, 1), n_ks=0)
