"""FP64 CPU oracle for the global spherical-harmonic transform.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module: only the test suite, the smoke check and the benchmark's
CPU-baseline leg use it.  It shares no code, table or constant generator with
the HIP library; the two meet only in the seeded inputs, which come from a
separate module holding none of the method's arithmetic.

What it computes is the plain definition of the transform, written out in
float64 with no blocking, fusion or symmetry tricks:

* synthesis ("inverse", spectral -> grid): the double sum of the dwarf's
  defining equation (ESCAPE D3.3, section 4.4.1, and again in 4.4.2): a
  Fourier series in longitude whose coefficient for wavenumber m is a
  Legendre sum over n of the spectral coefficients times the normalised
  associated Legendre functions at cos(colatitude);
* analysis ("direct", grid -> spectral): the discrete inverse of that sum,
  a longitude DFT normalised by 1/nlon followed by Gaussian quadrature in
  latitude.  The report gives only the synthesis equation; the analysis is
  its textbook quadrature inverse (reading recorded in the design notes).

Readings of what the report leaves unstated (each also listed in the design
notes, with the reason):

* normalisation: the integral of Pbar^2 over mu in [-1, 1] is 1, and there is
  no Condon-Shortley phase (Pbar_m^m > 0);
* real fields: the coefficient of -m is the conjugate of that of m, so only
  m >= 0 is stored and Im a_n^0 is ignored on input and 0 on output;
* triangular truncation N(m) = N;
* Gaussian latitudes are the roots of the Legendre polynomial P_nlat found by
  Newton iteration, ordered north to south (mu descending); weights sum to 2;
* full grid: nlat = N + 1 rings of 2N + 2 points.  Octahedral grid O(N+1):
  nlat = 2(N + 1) rings, ring i counted from either pole has 20 + 4i points;
* longitude of point k on a ring of n points is 2 pi k / n (origin 0 on every
  ring);
* per-ring Fourier truncation mmax_j = min(N, floor((nlon_j - 1) / 2)), which
  excludes the Nyquist wavenumber.

Parity status of each function:

* ``gauss_newton``  pinned (exact quadrature identities, library nodes,
  closed forms for small nlat);
* ``pbar``          pinned (closed forms, library associated Legendre
  functions, orthonormality, parity);
* ``dft_synthesis`` / ``dft_analysis`` pinned (library real FFT);
* ``inverse`` / ``direct`` pinned (library spherical harmonics, single
  harmonic, Parseval, round trip);
* ``grid_geometry`` pinned for the ring counts and lengths (the stated
  TCo1279 shape: 2560 rings, 20 + 4i points, 5136 at the equator, 6,599,680
  points; the 80 x 160 and 400 x 800 full grids) and the offsets; the
  per-ring truncation rule is a reading with no independent source: parity
  unpinned for that rule only;
* ``spec_index`` / ``nspec_of`` pinned (a counter over the m-major
  enumeration, the stated coefficient counts).
"""

import math

import numpy as np

__all__ = [
    "grid_geometry",
    "gauss_newton",
    "pbar",
    "spec_index",
    "nspec_of",
    "dft_synthesis",
    "dft_analysis",
    "inverse",
    "direct",
]


# ----------------------------------------------------------------------------
# Grid geometry
# ----------------------------------------------------------------------------

def grid_geometry(truncation, grid):
    """Ring structure of a full or octahedral reduced Gaussian grid.

    Returns a dict with ``nlat``, ``nlon`` (int array, rings north to south),
    ``mmax`` (per-ring Fourier truncation), ``off`` (grid offset of each ring,
    length nlat + 1), ``foff`` (offset of each ring's block of Fourier
    coefficients m = 0..mmax_j, length nlat + 1), ``npts``, ``nfour``,
    ``nspec``.

    Full grid: nlat = N + 1 latitudes by 2N + 2 longitudes.  Octahedral grid
    O(N + 1): 2(N + 1) latitudes, 20 + 4i points on ring i from each pole
    (the TCo1279 shape is 2560 latitudes with 5136 points at the equator).
    """
    N = int(truncation)
    if N < 1:
        raise ValueError("truncation must be >= 1")
    if grid == "full":
        nlat = N + 1
        nlon = np.full(nlat, 2 * N + 2, dtype=np.int64)
    elif grid == "octahedral":
        nlat = 2 * (N + 1)
        half = 20 + 4 * np.arange(N + 1, dtype=np.int64)
        nlon = np.concatenate([half, half[::-1]])
    else:
        raise ValueError("grid must be 'full' or 'octahedral'")
    mmax = np.minimum(N, (nlon - 1) // 2)
    off = np.zeros(nlat + 1, dtype=np.int64)
    off[1:] = np.cumsum(nlon)
    foff = np.zeros(nlat + 1, dtype=np.int64)
    foff[1:] = np.cumsum(mmax + 1)
    return {
        "N": N,
        "grid": grid,
        "nlat": nlat,
        "nlon": nlon,
        "mmax": mmax,
        "off": off,
        "foff": foff,
        "npts": int(off[-1]),
        "nfour": int(foff[-1]),
        "nspec": nspec_of(N),
    }


def nspec_of(N):
    """Number of (n, m) pairs with 0 <= m <= n <= N (triangular truncation)."""
    return (N + 1) * (N + 2) // 2


def spec_index(N, m, n):
    """Position of a_n^m in the m-major triangular spectral layout."""
    return m * (2 * N + 3 - m) // 2 + (n - m)


# ----------------------------------------------------------------------------
# Gaussian latitudes
# ----------------------------------------------------------------------------

def _legendre_p(n, mu):
    """P_n(mu) and P_{n-1}(mu) by the three-term recurrence
    k P_k = (2k - 1) mu P_{k-1} - (k - 1) P_{k-2}."""
    p_prev = np.ones_like(mu)
    p = mu.copy()
    for k in range(2, n + 1):
        p_prev, p = p, ((2 * k - 1) * mu * p - (k - 1) * p_prev) / k
    return p, p_prev


def gauss_newton(nlat, tol=1e-15, max_iter=100):
    """Gauss-Legendre nodes and weights by Newton iteration on P_nlat.

    Nodes are ordered north to south (mu descending).  Each root of the north
    half starts from cos(pi (j - 1/4) / (nlat + 1/2)), j = 1..ceil(nlat/2),
    and is refined with P'_n = n (P_{n-1} - mu P_n) / (1 - mu^2) until the
    step falls below ``tol``.  Weight: w = 2 / ((1 - mu^2) P'_n(mu)^2).  The
    south half is the mirror image.  If nlat is odd the middle node is 0.
    """
    nlat = int(nlat)
    if nlat < 1:
        raise ValueError("nlat must be >= 1")
    nh = (nlat + 1) // 2
    j = np.arange(1, nh + 1, dtype=np.float64)
    mu = np.cos(np.pi * (j - 0.25) / (nlat + 0.5))
    for _ in range(max_iter):
        p, pm1 = _legendre_p(nlat, mu)
        one_m = (1.0 - mu) * (1.0 + mu)
        dp = nlat * (pm1 - mu * p) / one_m
        step = p / dp
        mu = mu - step
        if np.max(np.abs(step)) < tol:
            break
    if nlat % 2 == 1:
        mu[-1] = 0.0
    p, pm1 = _legendre_p(nlat, mu)
    one_m = (1.0 - mu) * (1.0 + mu)
    dp = nlat * (pm1 - mu * p) / one_m
    w = 2.0 / (one_m * dp * dp)
    if nlat % 2 == 1:
        mu_all = np.concatenate([mu, -mu[-2::-1]])
        w_all = np.concatenate([w, w[-2::-1]])
    else:
        mu_all = np.concatenate([mu, -mu[::-1]])
        w_all = np.concatenate([w, w[::-1]])
    return mu_all, w_all


# ----------------------------------------------------------------------------
# Normalised associated Legendre functions
# ----------------------------------------------------------------------------

def _sin_colat(mu):
    """sin(theta) for mu = cos(theta), formed as sqrt((1 - mu)(1 + mu)) so
    that 1 - mu is exact near the poles."""
    return np.sqrt((1.0 - mu) * (1.0 + mu))


def pbar(m, N, mu):
    """Pbar_n^m(mu) for n = m..N, as an array [len(mu), N - m + 1].

    Normalised so that the integral of Pbar^2 over [-1, 1] is 1, no
    Condon-Shortley phase.  Textbook recurrences:

    * Pbar_0^0 = 1 / sqrt(2);
    * Pbar_k^k = sqrt((2k + 1) / (2k)) sin(theta) Pbar_{k-1}^{k-1};
    * Pbar_{m+1}^m = sqrt(2m + 3) mu Pbar_m^m;
    * Pbar_n^m = a (mu Pbar_{n-1}^m - b Pbar_{n-2}^m), with
      a = sqrt((4n^2 - 1) / (n^2 - m^2)),
      b = sqrt(((n - 1)^2 - m^2) / (4 (n - 1)^2 - 1)).
    """
    mu = np.asarray(mu, dtype=np.float64)
    if not (0 <= m <= N):
        raise ValueError("need 0 <= m <= N")
    s = _sin_colat(mu)
    p_mm = np.full(mu.shape, 1.0 / math.sqrt(2.0))
    for k in range(1, m + 1):
        p_mm = math.sqrt((2.0 * k + 1.0) / (2.0 * k)) * s * p_mm
    out = np.empty(mu.shape + (N - m + 1,), dtype=np.float64)
    out[..., 0] = p_mm
    if N > m:
        out[..., 1] = math.sqrt(2.0 * m + 3.0) * mu * p_mm
    for n in range(m + 2, N + 1):
        a = math.sqrt((4.0 * n * n - 1.0) / (n * n - m * m))
        b = math.sqrt(((n - 1.0) ** 2 - m * m) / (4.0 * (n - 1.0) ** 2 - 1.0))
        out[..., n - m] = a * (mu * out[..., n - m - 1] - b * out[..., n - m - 2])
    return out


# ----------------------------------------------------------------------------
# Longitude DFT by brute force
# ----------------------------------------------------------------------------

def _phase_tables(n, ms):
    """cos and sin of 2 pi (m k mod n) / n for the requested m and k < n.
    The integer reduction keeps the phase exact before the trig call."""
    k = np.arange(n, dtype=np.int64)
    q = (np.asarray(ms, dtype=np.int64)[:, None] * k[None, :]) % n
    ang = (2.0 * np.pi / n) * q.astype(np.float64)
    return np.cos(ang), np.sin(ang)


def dft_synthesis(c, n):
    """Real values on a ring of n points from Fourier coefficients.

    ``c`` is complex [F, mmax + 1] (m = 0..mmax, mmax < n / 2).  Returns
    g[F, n] with g_k = Re c_0 + 2 sum_{m >= 1} (Re c_m cos(m lam_k)
    - Im c_m sin(m lam_k)), lam_k = 2 pi k / n: the real field whose
    coefficient of -m is conj(c_m).  Im c_0 does not enter.
    """
    c = np.atleast_2d(np.asarray(c, dtype=np.complex128))
    mmax = c.shape[1] - 1
    if 2 * mmax >= n:
        raise ValueError("mmax must be below n / 2")
    cosm, sinm = _phase_tables(n, np.arange(mmax + 1))
    scale = np.full(mmax + 1, 2.0)
    scale[0] = 1.0
    return (c.real * scale) @ cosm - (c.imag * scale) @ sinm


def dft_analysis(g, n, ms):
    """Fourier coefficients (1/n) sum_k g_k exp(-i m lam_k) for the listed m.

    ``g`` is real [F, n]; returns complex [F, len(ms)]."""
    g = np.atleast_2d(np.asarray(g, dtype=np.float64))
    cosm, sinm = _phase_tables(n, ms)
    return (g @ cosm.T - 1j * (g @ sinm.T)) / n


# ----------------------------------------------------------------------------
# The transform
# ----------------------------------------------------------------------------

def _as_spec(spec, N):
    spec = np.atleast_2d(np.asarray(spec, dtype=np.complex128))
    if spec.shape[1] != nspec_of(N):
        raise ValueError("spectral array must be [F, (N+1)(N+2)/2]")
    return spec


def inverse(spec, truncation, grid, rings=None, geometry=None, gauss=None):
    """Synthesis: spectral coefficients -> Fourier coefficients and grid.

    ``spec`` is complex [F, nspec] in the m-major triangular layout.  For
    every ring j (both hemispheres, evaluated at its own mu_j, no
    symmetric/antisymmetric split) and every m <= mmax_j:

        c_{j,m} = sum_{n=m..N} a_n^m Pbar_n^m(mu_j)     (Im a_n^0 dropped)

    then the ring's grid values are the real Fourier series of c_j.

    ``rings`` restricts the work to a subset of ring indices (for sampled
    checks at large sizes).  Returns ``(four, grid)``: ``four`` is a dict
    ring -> complex [F, mmax_j + 1], ``grid`` a dict ring -> real [F, nlon_j]
    when ``rings`` is given, else the packed arrays [F, nfour] and
    [F, npts] (ring-major, rings north to south).
    """
    geo = geometry or grid_geometry(truncation, grid)
    N = geo["N"]
    spec = _as_spec(spec, N)
    F = spec.shape[0]
    mu, _w = gauss if gauss is not None else gauss_newton(geo["nlat"])
    sel = np.arange(geo["nlat"]) if rings is None else np.asarray(rings, dtype=np.int64)
    four = {int(j): np.zeros((F, geo["mmax"][j] + 1), dtype=np.complex128) for j in sel}
    for m in range(N + 1):
        rows = sel[geo["mmax"][sel] >= m]
        if rows.size == 0:
            continue
        P = pbar(m, N, mu[rows])
        lo = spec_index(N, m, m)
        a = spec[:, lo:lo + N - m + 1]
        if m == 0:
            a = a.real.astype(np.complex128)
        c = a @ P.T
        for t, j in enumerate(rows):
            four[int(j)][:, m] = c[:, t]
    gvals = {j: dft_synthesis(four[j], int(geo["nlon"][j])) for j in four}
    if rings is not None:
        return four, gvals
    fpack = np.zeros((F, geo["nfour"]), dtype=np.complex128)
    gpack = np.zeros((F, geo["npts"]), dtype=np.float64)
    for j in four:
        fpack[:, geo["foff"][j]:geo["foff"][j + 1]] = four[j]
        gpack[:, geo["off"][j]:geo["off"][j + 1]] = gvals[j]
    return fpack, gpack


def direct(gvals, truncation, grid, ms=None, geometry=None, gauss=None):
    """Analysis: grid values -> Fourier coefficients and spectral coefficients.

    ``gvals`` is real [F, npts] (ring-major, rings north to south).  For
    every ring j and m <= mmax_j the Fourier coefficient is the brute-force
    DFT (1/nlon_j) sum_k g_{j,k} exp(-i m lam_k); then, by Gaussian
    quadrature over every ring that carries m (both hemispheres, no split):

        a_n^m = sum_{j: mmax_j >= m} w_j chat_{j,m} Pbar_n^m(mu_j).

    Im a_n^0 is exactly 0.  ``ms`` restricts the output to a subset of m
    (the other coefficients are left 0).  Returns ``(four, spec)`` with
    ``four`` as a dict ring -> complex [F, len(ms_j)] when ``ms`` is given,
    else packed [F, nfour]; ``spec`` is complex [F, nspec].
    """
    geo = geometry or grid_geometry(truncation, grid)
    N = geo["N"]
    gvals = np.atleast_2d(np.asarray(gvals, dtype=np.float64))
    if gvals.shape[1] != geo["npts"]:
        raise ValueError("grid array must be [F, npts]")
    F = gvals.shape[0]
    mu, w = gauss if gauss is not None else gauss_newton(geo["nlat"])
    mlist = np.arange(N + 1) if ms is None else np.asarray(sorted(set(int(x) for x in ms)))
    four = {}
    for j in range(geo["nlat"]):
        mj = mlist[mlist <= geo["mmax"][j]]
        g = gvals[:, geo["off"][j]:geo["off"][j + 1]]
        four[j] = (mj, dft_analysis(g, int(geo["nlon"][j]), mj))
    spec = np.zeros((F, geo["nspec"]), dtype=np.complex128)
    for m in mlist:
        rows = np.nonzero(geo["mmax"] >= m)[0]
        P = pbar(int(m), N, mu[rows])
        chat = np.empty((F, rows.size), dtype=np.complex128)
        for t, j in enumerate(rows):
            mj, cj = four[j]
            chat[:, t] = cj[:, np.searchsorted(mj, m)]
        a = (chat * w[rows][None, :]) @ P
        if m == 0:
            a = a.real.astype(np.complex128)
        lo = spec_index(N, int(m), int(m))
        spec[:, lo:lo + N - int(m) + 1] = a
    if ms is not None:
        return {j: four[j][1] for j in four}, spec
    fpack = np.zeros((F, geo["nfour"]), dtype=np.complex128)
    for j in four:
        fpack[:, geo["foff"][j]:geo["foff"][j + 1]] = four[j][1]
    return fpack, spec
