"""FP64 CPU oracle for spectral derivatives and the vector (wind) transforms.

TEST INFRASTRUCTURE ONLY, like the rest of this package: nothing in the
product path may import, call or execute it.

The report motivates working in spectral space because derivatives become
pointwise multiplications there (ESCAPE D3.3, section 4.4.1).  This module
writes out, in float64 and with no symmetry split, blocking or recurrence in
spectral space, the textbook relations a spectral model builds on that:

* the longitude derivative of a_n^m P_n^m e^{i m lam} is i m times it;
* the horizontal Laplacian on the unit sphere multiplies a_n^m by -n(n+1);
* H_n^m(mu) = (1 - mu^2) dPbar_n^m/dmu, evaluated from the derivative
  identity of the associated Legendre functions,
      (1 - mu^2) dPbar_n^m/dmu = -n mu Pbar_n^m
                                 + sqrt((2n+1)(n^2-m^2)/(2n-1)) Pbar_{n-1}^m;
* winds from vorticity zeta and divergence D on the unit sphere through the
  stream function psi and velocity potential chi (zeta = Lap psi,
  D = Lap chi), with U = u cos(lat), V = v cos(lat), mu = sin(lat):
      U = dchi/dlam - (1 - mu^2) dpsi/dmu,
      V = dpsi/dlam + (1 - mu^2) dchi/dmu;
* the inverse relations, integrated by parts over mu and evaluated by the
  same Gaussian quadrature as the scalar analysis:
      zeta_n^m = sum_j w_j/(1-mu_j^2) [i m V_{j,m} Pbar_n^m(mu_j) + U_{j,m} H_n^m(mu_j)],
      D_n^m    = sum_j w_j/(1-mu_j^2) [i m U_{j,m} Pbar_n^m(mu_j) - V_{j,m} H_n^m(mu_j)],
  with U_{j,m}, V_{j,m} the ring DFT coefficients (1/nlon_j) sum_k (.) e^{-i m lam_k}.

Readings (recorded with the others in the design notes): the sphere has unit
radius (multiply winds by 1/a, vorticity and divergence by 1/a, for radius
a); zeta_0^0 and D_0^0 do not enter the winds (the global mean of a curl or
a divergence vanishes) and the analysis returns them as 0; Im of every m = 0
coefficient is ignored on input and 0 on output, as for scalars.

Parity status: ``dpbar`` pinned (closed forms, SciPy's derivative of the
normalised associated Legendre functions, finite differences of ``pbar``);
``vector_inverse`` / ``gradient`` pinned (solid-body rotation in closed
form, centred differences of the pinned scalar synthesis); ``vector_direct``
pinned (closed-form solid-body rotation, exact round trip on full grids);
``spectral_op`` pinned (single harmonics against the closed-form Laplacian
of P_n^m e^{i m lam}).
"""

import math

import numpy as np

from .sht_oracle import _as_spec, dft_analysis, dft_synthesis, gauss_newton, grid_geometry, nspec_of, pbar, spec_index

__all__ = ["dpbar", "spectral_op", "vector_inverse", "vector_direct", "gradient", "degree_of_slot", "order_of_slot"]


def degree_of_slot(N):
    """n of every slot of the m-major triangular layout."""
    return np.concatenate([np.arange(m, N + 1) for m in range(N + 1)])


def order_of_slot(N):
    """m of every slot of the m-major triangular layout."""
    return np.concatenate([np.full(N - m + 1, m) for m in range(N + 1)])


def dpbar(m, N, mu):
    """H_n^m(mu) = (1 - mu^2) dPbar_n^m/dmu for n = m..N, as [len(mu), N - m + 1],
    from the derivative identity above (Pbar_{m-1}^m = 0)."""
    mu = np.asarray(mu, dtype=np.float64)
    P = pbar(m, N, mu)
    H = np.empty_like(P)
    for n in range(m, N + 1):
        h = -n * mu * P[..., n - m]
        if n > m:
            h = h + math.sqrt((2.0 * n + 1.0) * (n * n - m * m) / (2.0 * n - 1.0)) * P[..., n - m - 1]
        H[..., n - m] = h
    return H


def spectral_op(spec, N, op):
    """Pointwise spectral operators on [F, nspec] complex coefficients:
    'dlambda' (i m a_n^m), 'laplacian' (-n(n+1) a_n^m), 'inv_laplacian'
    (-a_n^m / (n(n+1)), 0 for n = 0).  Im of m = 0 coefficients is dropped
    on input."""
    a = _as_spec(spec, N).copy()
    a[:, : N + 1] = a[:, : N + 1].real
    n = degree_of_slot(N).astype(np.float64)
    m = order_of_slot(N).astype(np.float64)
    if op == "dlambda":
        return a * (1j * m)[None, :]
    if op == "laplacian":
        return a * (-n * (n + 1.0))[None, :]
    if op == "inv_laplacian":
        f = np.zeros_like(n)
        f[1:] = -1.0 / (n[1:] * (n[1:] + 1.0))
        return a * f[None, :]
    raise ValueError("op must be 'dlambda', 'laplacian' or 'inv_laplacian'")


def _winds_from_potentials(psi, chi, N, grid, geometry=None, gauss=None):
    """U, V on the grid from stream function psi and velocity potential chi
    (spectral [F, nspec], Im of m = 0 already dropped)."""
    geo = geometry or grid_geometry(N, grid)
    mu, _w = gauss if gauss is not None else gauss_newton(geo["nlat"])
    F = psi.shape[0]
    Uf = {j: np.zeros((F, geo["mmax"][j] + 1), dtype=np.complex128) for j in range(geo["nlat"])}
    Vf = {j: np.zeros((F, geo["mmax"][j] + 1), dtype=np.complex128) for j in range(geo["nlat"])}
    for m in range(N + 1):
        rows = np.nonzero(geo["mmax"] >= m)[0]
        if rows.size == 0:
            continue
        P = pbar(m, N, mu[rows])
        H = dpbar(m, N, mu[rows])
        lo = spec_index(N, m, m)
        ps = psi[:, lo:lo + N - m + 1]
        ch = chi[:, lo:lo + N - m + 1]
        U = (1j * m) * (ch @ P.T) - ps @ H.T
        V = (1j * m) * (ps @ P.T) + ch @ H.T
        for t, j in enumerate(rows):
            Uf[j][:, m] = U[:, t]
            Vf[j][:, m] = V[:, t]
    Ug = np.zeros((F, geo["npts"]))
    Vg = np.zeros((F, geo["npts"]))
    for j in range(geo["nlat"]):
        n = int(geo["nlon"][j])
        Ug[:, geo["off"][j]:geo["off"][j + 1]] = dft_synthesis(Uf[j], n)
        Vg[:, geo["off"][j]:geo["off"][j + 1]] = dft_synthesis(Vf[j], n)
    return Ug, Vg


def vector_inverse(vort, div, truncation, grid, geometry=None, gauss=None):
    """Winds U = u cos(lat), V = v cos(lat) on the grid ([F, npts] each) from
    vorticity and divergence coefficients ([F, nspec] complex), unit sphere."""
    N = int(truncation)
    vort = _as_spec(vort, N)
    div = _as_spec(div, N)
    psi = spectral_op(vort, N, "inv_laplacian")
    chi = spectral_op(div, N, "inv_laplacian")
    return _winds_from_potentials(psi, chi, N, grid, geometry, gauss)


def gradient(spec, truncation, grid, geometry=None, gauss=None):
    """cos(lat) times the gradient of a scalar field on the unit sphere:
    U = df/dlam, V = (1 - mu^2) df/dmu, on the grid ([F, npts] each)."""
    N = int(truncation)
    f = _as_spec(spec, N).copy()
    f[:, : N + 1] = f[:, : N + 1].real
    return _winds_from_potentials(np.zeros_like(f), f, N, grid, geometry, gauss)


def vector_direct(U, V, truncation, grid, geometry=None, gauss=None):
    """Vorticity and divergence coefficients ([F, nspec] complex each) from
    winds U, V on the grid ([F, npts] each), unit sphere, by the quadrature
    relations above.  zeta_0^0 = D_0^0 = 0 and Im of every m = 0 coefficient
    is 0."""
    N = int(truncation)
    geo = geometry or grid_geometry(N, grid)
    mu, w = gauss if gauss is not None else gauss_newton(geo["nlat"])
    U = np.atleast_2d(np.asarray(U, dtype=np.float64))
    V = np.atleast_2d(np.asarray(V, dtype=np.float64))
    F = U.shape[0]
    Uh, Vh = {}, {}
    for j in range(geo["nlat"]):
        n = int(geo["nlon"][j])
        ms = np.arange(geo["mmax"][j] + 1)
        Uh[j] = dft_analysis(U[:, geo["off"][j]:geo["off"][j + 1]], n, ms)
        Vh[j] = dft_analysis(V[:, geo["off"][j]:geo["off"][j + 1]], n, ms)
    vort = np.zeros((F, nspec_of(N)), dtype=np.complex128)
    div = np.zeros((F, nspec_of(N)), dtype=np.complex128)
    for m in range(N + 1):
        rows = np.nonzero(geo["mmax"] >= m)[0]
        if rows.size == 0:
            continue
        P = pbar(m, N, mu[rows])
        H = dpbar(m, N, mu[rows])
        q = w[rows] / ((1.0 - mu[rows]) * (1.0 + mu[rows]))
        Um = np.stack([Uh[j][:, m] for j in rows], axis=1) * q[None, :]
        Vm = np.stack([Vh[j][:, m] for j in rows], axis=1) * q[None, :]
        z = (1j * m) * (Vm @ P) + Um @ H
        d = (1j * m) * (Um @ P) - Vm @ H
        if m == 0:
            z = z.real.astype(np.complex128)
            d = d.real.astype(np.complex128)
            z[:, 0] = 0.0
            d[:, 0] = 0.0
        lo = spec_index(N, m, m)
        vort[:, lo:lo + N - m + 1] = z
        div[:, lo:lo + N - m + 1] = d
    return vort, div
