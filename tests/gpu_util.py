"""Helpers shared by the GPU tests: conversions between the oracle's complex
arrays and the library's (B, 3, ncoef, 2) float64 device tensors."""

import numpy as np


def to_dev(U, torch):
    """(B, 3, nc) or (3, nc) complex -> contiguous float64 cuda tensor."""
    U = np.asarray(U)
    if U.ndim == 2:
        U = U[None]
    a = np.stack([U.real, U.imag], axis=-1).astype(np.float64)
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def from_dev(t):
    a = t.detach().cpu().numpy()
    return a[..., 0] + 1j * a[..., 1]


def field_rel(A, B, M):
    """Per-field relative L2 error (spectral norm, Phi without its mean)."""
    from oracle.norms import rel_err
    return rel_err(A, B, M)


# FP64 parity bar (relative L2).  Phi' and the wind (vorticity + divergence
# through the velocity they induce) must agree to 1e-11; the plain spectral
# L2 of the divergence alone carries the float64 rounding floor of the
# Laplacian of the kinetic energy (~1e-11 at T127/T255 for any float64
# implementation, see oracle/norms.py), so it is held to a looser bound.
TOL_STATE = 1e-11
TOL_PLAIN = (1e-11, 1e-11, 2e-10)


def assert_parity(got, ref, M, tol_state=TOL_STATE, tol_plain=TOL_PLAIN):
    from oracle.norms import rel_err, state_rel_err
    st = state_rel_err(got, ref, M)
    pl = rel_err(got, ref, M)
    assert np.all(st < tol_state), ("state (Phi', wind) rel L2", st, "plain", pl)
    assert np.all(pl < np.asarray(tol_plain)), ("plain (Phi', xi, delta) rel L2", pl, st)
    return st, pl
