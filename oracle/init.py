"""The paper's descent start (oracle, FP64; Sec. 2.3): Gaussian noise coloured so that
its power spectral density matches the first-order coefficients S1 x.

TEST INFRASTRUCTURE ONLY (see the package header).

The paper names the start but not its construction; this module is one reading of it,
in the paper's notation (the same reading the library implements):

1. Band levels. m_lambda = mean over the kept frames of S1 x(t, lambda) (Eq. 3 before
   the phi_F averaging along lambda, i.e. U1 x averaged by phi_T).
2. Band powers. For a circular complex Gaussian z with E|z|^2 = P, E|z| = sqrt(pi P) / 2
   (Rayleigh), so noise whose band lambda carries power P_lambda = (4 / pi) m_lambda^2
   has the mean modulus m_lambda there.
3. Spectrum. On the padded DFT grid of N_pad bins, with E_lambda = (1 / N_pad)
   sum_k |psi1_lambda^(k)|^2 the energy per sample of filter lambda and
   c_lambda = P_lambda / E_lambda its level per unit energy,
       |H_k|^2 = sum_lambda c_lambda |psi1_lambda^(k')|^2
                 / (sum_lambda |psi1_lambda^(k')|^2 + 1e-12 max_k sum_lambda |psi1_lambda^(k)|^2),
   k' = min(k, N_pad - k) (the filters are analytic, so the spectrum is mirrored to the
   negative frequencies and y0 is real). Where the bands do not overlap, white noise
   shaped by H has band power exactly P_lambda; the small regulariser keeps the ratio
   smooth where every filter vanishes.
4. Noise. y0 = unpad(IDFT(H . DFT(pad(w)))) for w a vector of N independent standard
   normal draws (passed in: the generator is not part of the method).
"""
from __future__ import annotations

import math

import numpy as np

from .fftroute import FilterCache, first_layer, pad_signal
from .plan import OraclePlan

# relative floor of the summed filter energy in the spectrum's denominator (step 3)
REG = 1e-12


def band_levels(plan: OraclePlan, x: np.ndarray, fc: FilterCache = None) -> np.ndarray:
    """m_lambda: S1 x averaged over the kept frames, one value per first-order filter."""
    fc = fc or FilterCache(plan)
    S1 = first_layer(plan, x, fc)[3]
    return S1[:, plan.f_lo:plan.f_lo + plan.n_frames].mean(axis=1)


def spectrum(plan: OraclePlan, m: np.ndarray, fc: FilterCache = None) -> np.ndarray:
    """H_k (real, >= 0) on all N_pad bins for band levels m (steps 2-3)."""
    fc = fc or FilterCache(plan)
    m = np.asarray(m, dtype=np.float64)
    k = np.arange(plan.N_pad)
    kk = np.minimum(k, plan.N_pad - k)
    num = np.zeros(plan.N_pad)
    den = np.zeros(plan.N_pad)
    for n1 in range(plan.N1):
        h2 = np.abs(fc.psi1(n1)) ** 2
        E = h2.sum() / plan.N_pad
        c = (4.0 / math.pi) * m[n1] ** 2 / E
        num += c * h2[kk]
        den += h2[kk]
    return np.sqrt(num / (den + REG * den.max()))


def shape(plan: OraclePlan, H: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Step 4: white noise w (N samples) filtered by the spectrum H, unpadded."""
    y = np.fft.ifft(H * np.fft.fft(pad_signal(plan, w)))
    return y.real[plan.pad_left:plan.pad_left + plan.N]


def colored_noise(plan: OraclePlan, x: np.ndarray, w: np.ndarray, fc: FilterCache = None) -> np.ndarray:
    """The descent start y0 for target x and standard normal draws w."""
    fc = fc or FilterCache(plan)
    return shape(plan, spectrum(plan, band_levels(plan, x, fc), fc), w)
