"""Shared helpers of the GPU parity tests: seeded inputs in both forms
(device tensor for the HIP path, complex128 numpy of the very same rounded
values for the oracle) and the comparison metric."""

import numpy as np

from paper_1908_06096_amd.inputs import grid_noise, spectral_coefficients

TOL = {"fp64": 1e-12, "fp32": 1e-5, "bf16x3": 1e-5}


def rel_l2(x, ref):
    x = np.asarray(x)
    ref = np.asarray(ref)
    den = np.linalg.norm(ref.ravel())
    return float(np.linalg.norm((x - ref).ravel()) / (den if den > 0 else 1.0))


def np_dtype(precision):
    return np.float64 if precision == "fp64" else np.float32


def spec_inputs(plan, seed=0, distinct=None):
    """Seeded coefficients for all fields of ``plan``.  With ``distinct`` = d,
    only d fields are drawn and field f is a copy of field f mod d (keeps
    large cases quick; every field is still a valid input)."""
    import torch

    F = plan.nfields
    d = F if distinct is None else min(F, distinct)
    s = spectral_coefficients(plan.truncation, d, seed=seed, dtype=np_dtype(plan.precision))
    if d < F:
        s = s[np.arange(F) % d]
    t = torch.from_numpy(np.ascontiguousarray(s)).cuda()
    c = s[..., 0].astype(np.float64) + 1j * s[..., 1].astype(np.float64)
    return t, c


def grid_inputs(plan, seed=0, distinct=None):
    import torch

    F = plan.nfields
    d = F if distinct is None else min(F, distinct)
    g = grid_noise(plan.npts, d, seed=seed, dtype=np_dtype(plan.precision))
    if d < F:
        g = g[np.arange(F) % d]
    t = torch.from_numpy(np.ascontiguousarray(g)).cuda()
    return t, g.astype(np.float64)


def spec_to_complex(t):
    a = t.detach().cpu().numpy().astype(np.float64)
    return a[..., 0] + 1j * a[..., 1]
