"""The joint time--log-frequency wavelet of a scattering path (oracle, FP64; test
infrastructure only).

Sec. 2.1 (Eq. 2) filters the scalogram jointly by a time wavelet psi_alpha(t) and a
log-frequency wavelet psi_beta(log2 lambda); Fig. 1 shows the real part of their product,
the "interference pattern" of a path. Here both factors are the continuous filters of
``filterbank`` sampled and periodised in their own domain (time domain: no Fourier
table): psi_alpha is the second-order wavelet n2 at the signal's rate on the N_pad-point
grid, psi_beta the frequential filter n_fr (phi_F or a spinned band-pass) on the N_fr
log-frequency bins. Both are centred: time t maps to t - n_t / 2, bin r to r - N_fr / 2.
"""
from __future__ import annotations

import numpy as np

from . import filterbank as fb
from .plan import OraclePlan


def time_wavelet(plan: OraclePlan, n2: int) -> np.ndarray:
    """psi_alpha of the second-order filter n2, time domain, N_pad samples (complex)."""
    b = plan.psi2[n2]
    return fb.bandpass_time(plan.N_pad, b.xi, b.sigma, 0)


def freq_wavelet(plan: OraclePlan, n_fr: int) -> np.ndarray:
    """psi_beta of the frequential filter n_fr along log-frequency, N_fr bins (complex)."""
    b = plan.fr[n_fr]
    if b.lowpass:
        return fb.lowpass_time(plan.N_fr, b.sigma, 0).astype(np.complex128)
    return fb.bandpass_time(plan.N_fr, b.xi, b.sigma, 0)


def joint_wavelet_complex(plan: OraclePlan, n2: int, n_fr: int, n_t: int) -> np.ndarray:
    """psi_alpha(t - n_t/2) psi_beta(r - N_fr/2) on an N_fr x n_t grid (complex)."""
    a = time_wavelet(plan, n2)
    g = freq_wavelet(plan, n_fr)
    t = (np.arange(n_t) - n_t // 2) % plan.N_pad
    r = (np.arange(plan.N_fr) - plan.N_fr // 2) % plan.N_fr
    return g[r][:, None] * a[t][None, :]


def joint_wavelet(plan: OraclePlan, n2: int, n_fr: int, n_t: int) -> np.ndarray:
    """Fig. 1's interference pattern: the real part of the joint wavelet."""
    return joint_wavelet_complex(plan, n2, n_fr, n_t).real
