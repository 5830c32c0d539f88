"""Morlet and Gaussian filters of the JTFS filterbanks (oracle; test infrastructure only).

Conventions (sample rate 1, frequencies in cycles per sample, Sec. 3.1):

* A band-pass filter is described by its centre ``xi`` and Gaussian width ``sigma``.
  Its Fourier transform is the Gaussian G(w - xi; sigma) = exp(-(w - xi)^2 / (2 sigma^2))
  minus a multiple kappa of G(w; sigma), kappa chosen so that the filter has a null
  average (paper Eq. 1: the corrective term gives one vanishing moment).
  In the time domain this is sigma*sqrt(2 pi) exp(-2 pi^2 sigma^2 t^2) (exp(2 pi i xi t) - kappa),
  i.e. Eq. 1 with lambda = xi and the Eq. 1 quality factor equal to xi / (2 pi sigma);
  the lambda prefactor of Eq. 1 is replaced by a unit Fourier peak.
* A low-pass filter (phi_T over time, phi_F over log-frequency bins) is the Gaussian
  G(w; sigma) normalised to unit gain at w = 0 (Sec. 2.2, Eqs. 3-4).
* A filter "at level k" is the same physical filter for a signal already subsampled
  by 2^k: parameters (2^k xi, 2^k sigma) on the coarser grid, with kappa (or the
  low-pass normalisation) recomputed on that grid (the ``levels[k]`` tables of Sec. 3.2-3.3).
* On an L-point grid, the Fourier values are the closed form periodised with period 1
  at w = m / L; the time values are the continuous filter periodised with period L at
  integer t. The two are a DFT pair by the Poisson summation formula.
"""
from __future__ import annotations

import math

import numpy as np

SIGMA0 = 0.1                # sigma0 of the Sec. 3.1 generator
R_PSI = math.sqrt(0.5)      # r_psi of the Sec. 3.1 generator: neighbours cross at -3 dB
BAND_EDGE_WIDTHS = 5.0      # a filter's band edge is xi + 5 sigma (subsampling rule)


def constant_q_count(sigma_top: float, sigma_min: float, Q: int) -> int:
    """How many constant-Q filters the Sec. 3.1 generator emits.

    Widths shrink by 2^(1/Q) per filter, sigma_k = sigma_top 2^(-k/Q), and a filter of the
    constant-Q region is kept while its width stays strictly above the floor sigma_min
    (the elbow). With R = Q log2(sigma_top / sigma_min) that is every k < R: ceil(R)
    filters, or R itself when R is an integer (the member of width exactly sigma_min
    belongs to the constant-bandwidth region). R within 1e-9 of an integer counts as
    that integer, so the decision does not hang on the last bit of a logarithm.
    No room at all (sigma_top <= sigma_min) gives 0.
    """
    if sigma_top <= sigma_min:
        return 0
    R = Q * math.log2(sigma_top / sigma_min)
    m = round(R)
    if abs(R - m) <= 1e-9 * max(1.0, R):
        return max(1, m)
    return max(1, math.ceil(R))


def morlet_bank(J: int, Q: int):
    """(xi, sigma) pairs of a wavelet filterbank (Sec. 3.1), in closed form.

    * Top filter: xi_0 = max(1 / (1 + 2^(3/Q)), 0.35). Its width sigma_0 makes two
      Gaussians a factor 2^(1/Q) apart meet at r_psi of their peak:
      sigma_0 = (1 - 2^(-1/Q)) / (1 + 2^(-1/Q)) * xi_0 / sqrt(2 ln(1 / r_psi)).
    * Constant-Q region: (xi_0 2^(-k/Q), sigma_0 2^(-k/Q)) for the k counted by
      ``constant_q_count`` against the floor sigma_min = sigma0 / 2^J.
    * Constant-bandwidth region: Q - 1 filters of width sigma_min whose centres step
      down arithmetically from the last constant-Q centre e by e / Q each,
      xi = e (1 - q / Q), q = 1 .. Q - 1. Without a constant-Q region the steps start
      from e = sigma_0.
    """
    if J < 0 or Q < 1:
        raise ValueError("need J >= 0 and Q >= 1")
    xi_top = max(1.0 / (1.0 + math.pow(2.0, 3.0 / Q)), 0.35)
    f = math.pow(2.0, -1.0 / Q)
    sigma_top = (1.0 - f) / (1.0 + f) * xi_top / math.sqrt(2.0 * math.log(1.0 / R_PSI))
    sigma_min = SIGMA0 / math.pow(2.0, J)
    n_cq = constant_q_count(sigma_top, sigma_min, Q)
    bank = []
    for k in range(n_cq):
        g = math.pow(2.0, -k / Q)
        bank.append((xi_top * g, sigma_top * g))
    elbow = bank[-1][0] if bank else sigma_top
    for q in range(1, Q):
        bank.append((elbow * (Q - q) / Q, sigma_min))
    return bank


def spun(bank):
    """Frequential band-pass list with spin: the bank, then every centre negated (Sec. 3.4)."""
    return list(bank) + [(-xi, s) for (xi, s) in bank]


def subsampling_scale(xi: float, sigma: float) -> int:
    """Largest j >= 0 whose Nyquist 2^-(j+1) still lies above the band edge |xi| + 5 sigma.

    Sec. 3.2 ties the subsampling of a filter to how fine its cut-off frequency is; the
    band edge at 5 sigma is this implementation's reading of that. Comparisons use exact powers
    of two so that the rule is decided identically everywhere.
    """
    edge = abs(xi) + BAND_EDGE_WIDTHS * sigma
    j = 0
    while edge <= math.ldexp(1.0, -(j + 2)):
        j += 1
    return j


def gauss(u, s):
    return np.exp(-(u * u) / (2.0 * s * s))


_PERIODS = 4   # period-1 images summed on each side; terms beyond are below exp(-300)


def bandpass_hat(L: int, xi: float, sigma: float, level: int = 0) -> np.ndarray:
    """Fourier values of a Morlet band-pass at ``level`` on an L-point grid (real, length L)."""
    xs = xi * 2.0 ** level
    ss = sigma * 2.0 ** level
    w = np.arange(L, dtype=np.float64) / L
    p = np.arange(-_PERIODS, _PERIODS + 1, dtype=np.float64)[:, None]
    bump = gauss(w[None, :] + p - xs, ss).sum(axis=0)
    env = gauss(w[None, :] + p, ss).sum(axis=0)
    kappa = bump[0] / env[0]
    return bump - kappa * env


def lowpass_hat(L: int, sigma: float, level: int = 0) -> np.ndarray:
    """Fourier values of a Gaussian low-pass at ``level`` on an L-point grid, unit DC gain."""
    ss = sigma * 2.0 ** level
    w = np.arange(L, dtype=np.float64) / L
    p = np.arange(-_PERIODS, _PERIODS + 1, dtype=np.float64)[:, None]
    env = gauss(w[None, :] + p, ss).sum(axis=0)
    return env / env[0]


def _time_images(L: int, ss: float) -> int:
    # Time-domain standard deviation is 1 / (2 pi ss); sum images out to 40 of them.
    width = 40.0 / (2.0 * math.pi * ss)
    return int(math.ceil(width / L)) + 1


def morlet_time_continuous(t, xi: float, sigma: float, kappa: float):
    """Continuous-time Morlet whose Fourier transform is G(w - xi; sigma) - kappa G(w; sigma)."""
    env = sigma * math.sqrt(2.0 * math.pi) * np.exp(-2.0 * math.pi ** 2 * sigma ** 2 * t * t)
    return env * (np.exp(2j * math.pi * xi * t) - kappa)


def morlet_kappa_time(xi: float, sigma: float) -> float:
    """kappa making the integer-sampled Morlet sum to zero, computed by a direct time sum."""
    half = int(math.ceil(40.0 / (2.0 * math.pi * sigma))) + 1
    t = np.arange(-half, half + 1, dtype=np.float64)
    g = np.exp(-2.0 * math.pi ** 2 * sigma ** 2 * t * t)
    num = np.sum(g * np.cos(2.0 * math.pi * xi * t))   # the sine part cancels by symmetry
    return float(num / np.sum(g))


def bandpass_time(L: int, xi: float, sigma: float, level: int = 0) -> np.ndarray:
    """Time values of the level-``level`` Morlet on an L-point grid (complex, length L).

    Built from the continuous filter, independently of ``bandpass_hat``: kappa by a
    direct sum over integer times, periodisation by summing images t + qL.
    """
    xs = xi * 2.0 ** level
    ss = sigma * 2.0 ** level
    kappa = morlet_kappa_time(xs, ss)
    n = np.arange(L, dtype=np.float64)
    q = _time_images(L, ss)
    out = np.zeros(L, dtype=np.complex128)
    for img in range(-q, q + 1):
        out += morlet_time_continuous(n + img * L, xs, ss, kappa)
    return out


def lowpass_time(L: int, sigma: float, level: int = 0) -> np.ndarray:
    """Time values of the level-``level`` Gaussian low-pass on an L-point grid, summing to 1."""
    ss = sigma * 2.0 ** level
    n = np.arange(L, dtype=np.float64)
    q = _time_images(L, ss)
    out = np.zeros(L, dtype=np.float64)
    for img in range(-q, q + 1):
        t = n + img * L
        out += np.exp(-2.0 * math.pi ** 2 * ss ** 2 * t * t)
    return out / out.sum()
