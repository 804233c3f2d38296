"""Seeded right-hand-side generators (inputs only; see the package docstring).

Every generator returns a float64 ``numpy`` array of shape ``(n, n)`` laid out
as described in the package docstring.  All randomness comes from
``numpy.random.default_rng(seed)`` with the draw order documented per
function, so a seed fixes the array bit for bit.
"""

from __future__ import annotations

import numpy as np
import scipy.fft

DIRICHLET = 0
PERIODIC = 1

# Grid sides of the batched workload: 256 periodic problems whose side is drawn
# uniformly from this set.
SIZES_BATCHED = (129, 257, 513, 1025)


def _check_n(n: int) -> None:
    m = n - 1
    if n < 5 or m % 4 != 0 or (m // 4) & (m // 4 - 1):
        raise ValueError(f"grid side n={n} must satisfy n-1 = 4*2^k, n >= 5")


def grid_unknowns(n: int, bc: int) -> int:
    """Number of unknown nodes: (n-2)^2 for zero Dirichlet, (n-1)^2 periodic."""
    return (n - 2) ** 2 if bc == DIRICHLET else (n - 1) ** 2


def _with_seam(core: np.ndarray) -> np.ndarray:
    """Embed an (N, N) periodic field into (N+1, N+1) with the duplicated seam."""
    N = core.shape[0]
    out = np.empty((N + 1, N + 1), dtype=np.float64)
    out[:N, :N] = core
    out[N, :N] = core[0, :]
    out[:N, N] = core[:, 0]
    out[N, N] = core[0, 0]
    return out


def manufactured_solution(n: int) -> np.ndarray:
    """u(x, y) = sin(pi x) sin(pi y) sampled on the grid (zero on the boundary)."""
    _check_n(n)
    x = np.arange(n, dtype=np.float64) / (n - 1)
    s = np.sin(np.pi * x)
    s[0] = 0.0
    s[-1] = 0.0
    return np.outer(s, s)


def rhs_manufactured_dirichlet(n: int, seed: int, modes: int = 8,
                               kmax: int = 8, sigma: float = 0.1) -> np.ndarray:
    """Zero-Dirichlet source: 2 pi^2 sin(pi x) sin(pi y) plus random sine modes.

    f = 2 pi^2 sin(pi x) sin(pi y) + sum_m a_m sin(k_m pi x) sin(l_m pi y),
    m = 1..modes.  Draw order from ``default_rng(seed)``: the x mode numbers
    k (``integers(1, kmax+1, modes)``), then the y mode numbers l (same call),
    then the amplitudes a (``normal(0, sigma, modes)``; sigma is a standard
    deviation).  Sine modes keep f zero on the boundary; boundary entries are
    set to exactly 0.
    """
    _check_n(n)
    rng = np.random.default_rng(seed)
    kx = rng.integers(1, kmax + 1, size=modes)
    ly = rng.integers(1, kmax + 1, size=modes)
    amp = rng.normal(0.0, sigma, size=modes)
    x = np.arange(n, dtype=np.float64) / (n - 1)
    f = 2.0 * np.pi ** 2 * np.outer(np.sin(np.pi * x), np.sin(np.pi * x))
    for k, l, a in zip(kx, ly, amp):
        f += a * np.outer(np.sin(l * np.pi * x), np.sin(k * np.pi * x))
    f[0, :] = 0.0
    f[-1, :] = 0.0
    f[:, 0] = 0.0
    f[:, -1] = 0.0
    return f


def _spectral_amplitude(kappa: np.ndarray, kmax: float) -> np.ndarray:
    """|u_hat(k)| = sqrt(E(k) / (2 pi k)) with E(k) = k^(-5/3) on 1 <= k <= kmax."""
    amp = np.zeros_like(kappa)
    band = (kappa >= 1.0) & (kappa <= kmax)
    kb = kappa[band]
    amp[band] = np.sqrt(kb ** (-5.0 / 3.0) / (2.0 * np.pi * kb))
    return amp


def rhs_divu_periodic(n: int, seed: int, kmax: float | None = None) -> np.ndarray:
    """Periodic source f = div u of a random velocity field with E(k) ~ k^(-5/3).

    The unique grid is N x N, N = n-1, on the unit torus.  The two velocity
    components are independent real fields whose Fourier amplitudes are
    sqrt(E(|k|)/(2 pi |k|)) on integer wavenumbers 1 <= |k| <= kmax (default
    kmax = (n-1)/4) with uniform random phases.  Draw order from
    ``default_rng(seed)``: the phase array of u_x, then that of u_y, each of
    shape (N, N//2+1) from ``uniform(0, 2 pi)``.  f is the spectral divergence
    (real field via ``irfft2``), its mean is removed, and it is scaled to unit
    RMS over the unique nodes.  Returned with the duplicated seam.
    """
    _check_n(n)
    return _divu_periodic(n - 1, seed, kmax)


def _divu_periodic(N: int, seed: int, kmax: float | None) -> np.ndarray:
    """rhs_divu_periodic on N unique nodes per side (any even N)."""
    if kmax is None:
        kmax = N / 4
    rng = np.random.default_rng(seed)
    ph_x = rng.uniform(0.0, 2.0 * np.pi, size=(N, N // 2 + 1))
    ph_y = rng.uniform(0.0, 2.0 * np.pi, size=(N, N // 2 + 1))
    ky = np.fft.fftfreq(N, d=1.0 / N)[:, None]
    kx = np.fft.rfftfreq(N, d=1.0 / N)[None, :]
    kappa = np.sqrt(kx * kx + ky * ky)
    amp = _spectral_amplitude(kappa, float(kmax))
    ux_hat = amp * np.exp(1j * ph_x)
    uy_hat = amp * np.exp(1j * ph_y)
    f_hat = 2j * np.pi * (kx * ux_hat + ky * uy_hat)
    f_hat[0, 0] = 0.0
    f = np.fft.irfft2(f_hat, s=(N, N))
    f -= f.mean()
    f /= np.sqrt(np.mean(f * f))
    f -= f.mean()
    return _with_seam(f)


def velocity_periodic(n: int, seed: int, kmax: float | None = None):
    """Divergence-free periodic velocity (u_x, u_y) with E(k) ~ k^(-5/3).

    The unique grid is N x N, N = n-1, on the unit torus; x runs along the
    columns (axis 1), y along the rows (axis 0).  A stream function psi has
    Fourier amplitudes sqrt(E(|k|)/(2 pi |k|)) / (2 pi |k|) on integer
    wavenumbers 1 <= |k| <= kmax (default (n-1)/4) with uniform random phases
    drawn from ``default_rng(seed)`` as one array of shape (N, N//2+1) from
    ``uniform(0, 2 pi)``; u_x = d psi/dy, u_y = -d psi/dx (spectral), scaled
    together to unit RMS speed over the unique nodes.  Returned with the
    duplicated seam, float64.
    """
    _check_n(n)
    N = n - 1
    if kmax is None:
        kmax = N / 4
    rng = np.random.default_rng(seed)
    ph = rng.uniform(0.0, 2.0 * np.pi, size=(N, N // 2 + 1))
    ky = np.fft.fftfreq(N, d=1.0 / N)[:, None]
    kx = np.fft.rfftfreq(N, d=1.0 / N)[None, :]
    kappa = np.sqrt(kx * kx + ky * ky)
    amp = _spectral_amplitude(kappa, float(kmax))
    psi_hat = np.where(kappa > 0, amp / (2.0 * np.pi * np.maximum(kappa, 1.0)), 0.0) * np.exp(1j * ph)
    ux = np.fft.irfft2(2j * np.pi * ky * psi_hat, s=(N, N))
    uy = np.fft.irfft2(-2j * np.pi * kx * psi_hat, s=(N, N))
    speed = np.sqrt(np.mean(ux * ux + uy * uy))
    return _with_seam(ux / speed), _with_seam(uy / speed)


def rhs_divu_dirichlet(n: int, seed: int, kmax: float | None = None) -> np.ndarray:
    """Zero-Dirichlet analogue of ``rhs_divu_periodic`` in the sine basis.

    u_x = sum U[p,q] sin(p pi y) cos(q pi x), u_y = sum V[p,q] cos(p pi y)
    sin(q pi x) with p, q >= 1 and kappa = sqrt(p^2+q^2) in [1, kmax] (default
    kmax = (n-1)/4), U = A(kappa) cos(phi), V = A(kappa) cos(psi),
    A = sqrt(E/(2 pi kappa)), E = kappa^(-5/3).  Then f = div u =
    -pi sum (q U + p V) sin(p pi y) sin(q pi x), synthesised with a type-I
    DST on the interior nodes and scaled to unit RMS there.  Draw order from
    ``default_rng(seed)``: phi then psi, each of shape (n-2, n-2) from
    ``uniform(0, 2 pi)``.  Boundary entries are exactly 0.
    """
    _check_n(n)
    M = n - 2
    if kmax is None:
        kmax = (n - 1) / 4
    rng = np.random.default_rng(seed)
    phi = rng.uniform(0.0, 2.0 * np.pi, size=(M, M))
    psi = rng.uniform(0.0, 2.0 * np.pi, size=(M, M))
    p = np.arange(1, M + 1, dtype=np.float64)[:, None]
    q = np.arange(1, M + 1, dtype=np.float64)[None, :]
    kappa = np.sqrt(p * p + q * q)
    amp = _spectral_amplitude(kappa, float(kmax))
    coef = -np.pi * (q * amp * np.cos(phi) + p * amp * np.cos(psi))
    interior = scipy.fft.dstn(coef, type=1) / 4.0
    interior /= np.sqrt(np.mean(interior * interior))
    f = np.zeros((n, n), dtype=np.float64)
    f[1:-1, 1:-1] = interior
    return f


# The paper's controlled two-level experiment (Section 4.1, Table 1): 192 x 192
# periodic grids, a test set of 100 sources.
TWOLEVEL_N = 192
TWOLEVEL_BATCH = 100


def rhs_twolevel_periodic(N: int, seed: int, kmax: float | None = None) -> np.ndarray:
    """Periodic source on N unique nodes per side (N even, not necessarily
    4 * 2^k; stored with the seam as (N+1, N+1)): the rhs_divu_periodic recipe
    (divergence of a k^(-5/3) velocity field, kmax = N/4 by default, mean
    removed, unit RMS)."""
    if N < 8 or N % 2:
        raise ValueError(f"unique side N={N} must be even and >= 8")
    return _divu_periodic(N, seed, kmax)


def initial_grid_periodic(N: int, seed: int, scale: float = 1e-3) -> np.ndarray:
    """The initially random pressure grid of the two-level experiment
    (Table 1's N_smooth,pre sweeps then smooth it): ``scale *
    default_rng(seed).standard_normal((N, N))``, stored with the seam.  The
    default scale is the order of the pressure a unit-RMS source of this
    kind produces on the unit torus."""
    rng = np.random.default_rng(seed)
    return _with_seam(scale * rng.standard_normal((N, N)))


def twolevel_batch(seed: int = 0, count: int = TWOLEVEL_BATCH, N: int = TWOLEVEL_N):
    """The two-level test set: problem b has source rhs_twolevel_periodic(N,
    2000 + b) and initial grid initial_grid_periodic(N, 3000 + b); ``seed``
    shifts both seed bases by 10000 * seed.  Returns (f, p0) arrays of shape
    (count, N+1, N+1)."""
    f = np.stack([rhs_twolevel_periodic(N, 10000 * seed + 2000 + b) for b in range(count)])
    p0 = np.stack([initial_grid_periodic(N, 10000 * seed + 3000 + b) for b in range(count)])
    return f, p0


def batch_sizes(seed: int, count: int = 256) -> list[int]:
    """Grid sides of the batched workload: ``default_rng(seed).integers(0, 4,
    count)`` indexes ``SIZES_BATCHED``."""
    idx = np.random.default_rng(seed).integers(0, len(SIZES_BATCHED), size=count)
    return [SIZES_BATCHED[i] for i in idx]


def workload(name: str, seed: int = 0):
    """Named workloads.  Returns ``(n, bc, f)`` or, for the batch, a list.

    * ``"dirichlet65"``: n=65, zero Dirichlet, manufactured source + 8 modes.
    * ``"periodic1025"``: n=1025 periodic, div-u source with kmax = 256.
    * ``"dirichlet4097"``: n=4097 zero Dirichlet, sine-basis div-u source,
      kmax = 1024.
    * ``"batch256"``: 256 periodic problems, sides from ``batch_sizes(seed)``,
      problem b built by ``rhs_divu_periodic`` with seed 1000+b.
    """
    if name == "dirichlet65":
        return 65, DIRICHLET, rhs_manufactured_dirichlet(65, seed)
    if name == "periodic1025":
        return 1025, PERIODIC, rhs_divu_periodic(1025, seed, kmax=256)
    if name == "dirichlet4097":
        return 4097, DIRICHLET, rhs_divu_dirichlet(4097, seed, kmax=1024)
    if name == "batch256":
        sizes = batch_sizes(seed)
        return [(n, PERIODIC, rhs_divu_periodic(n, 1000 + b)) for b, n in enumerate(sizes)]
    raise KeyError(name)
