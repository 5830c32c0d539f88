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


def morlet_bank(J: int, Q: int):
    """(xi, sigma) pairs of a wavelet filterbank, Sec. 3.1.

    The top filter sits at max(1 / (1 + 2^(3/Q)), 0.35). Its width follows from the
    requirement that neighbouring Gaussians, a factor 2^(1/Q) apart, cross at r_psi
    of their peak. Centres and widths then shrink geometrically by 2^(1/Q) (constant Q)
    while the width stays above sigma0 / 2^J scaled by one step; below that "elbow"
    Q - 1 further filters are spaced arithmetically at the minimum width.

    The arithmetic is written in the same order as the paper's generator (one division
    per step) so that the number of constant-Q filters is decided the same way.
    """
    if J < 0 or Q < 1:
        raise ValueError("need J >= 0 and Q >= 1")
    step = math.pow(2.0, 1.0 / Q)
    shrink = 1.0 / step
    xi = max(1.0 / (1.0 + math.pow(2.0, 3.0 / Q)), 0.35)
    sigma = (1.0 - shrink) / (1.0 + shrink) * xi / math.sqrt(2.0 * math.log(1.0 / R_PSI))
    sigma_min = SIGMA0 / math.pow(2.0, J)

    bank = []
    if sigma <= sigma_min:
        # No room for a constant-Q region: the arithmetic region starts from xi = sigma.
        xi = sigma
    else:
        bank.append((xi, sigma))
        while sigma > sigma_min * step:
            xi = xi / step
            sigma = sigma / step
            bank.append((xi, sigma))
    elbow = xi
    for _ in range(Q - 1):
        xi = xi - elbow / Q
        bank.append((xi, sigma_min))
    return bank


def spun(bank):
    """Frequential band-pass list with spin: the bank, then every centre negated (Sec. 3.4)."""
    return list(bank) + [(-xi, s) for (xi, s) in bank]


def subsampling_scale(xi: float, sigma: float) -> int:
    """Largest j >= 0 whose Nyquist 2^-(j+1) still lies above the band edge |xi| + 5 sigma.

    Kymatio derives j from "the resolution of the cutoff frequency" (Sec. 3.2); the
    factor 5 on sigma is this implementation's reading. Comparisons use exact powers
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
