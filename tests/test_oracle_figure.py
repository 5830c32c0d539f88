"""Pins of the oracle's joint wavelet (Sec. 2.1, Fig. 1) against the mathematics (CPU)."""
import numpy as np
import pytest

from oracle import figure
from oracle import filterbank as fb
from oracle.plan import make_plan

CFG1 = (8192, 6, 8, 1, 3, 1, 9, 4.0)


def test_two_dimensional_dft_is_the_product_of_fourier_filters():
    # With n_t = N_pad the complex joint wavelet is the outer product of two periodic
    # sequences, circularly shifted: its 2-D DFT is the outer product of the closed-form
    # Fourier filters (Poisson pair of Eq. 1's Morlet) times the shift phases.
    p = make_plan(1024, 4, 4, 2, 2, 2, 5, 2, periodic=True)
    for n2 in range(len(p.psi2)):
        for n_fr in (0, 1, len(p.fr) - 1):
            F = figure.joint_wavelet_complex(p, n2, n_fr, p.N_pad)
            D = np.fft.fft2(F)
            b2, bf = p.psi2[n2], p.fr[n_fr]
            a_hat = fb.bandpass_hat(p.N_pad, b2.xi, b2.sigma, 0)
            g_hat = fb.lowpass_hat(p.N_fr, bf.sigma, 0) if bf.lowpass else fb.bandpass_hat(p.N_fr, bf.xi, bf.sigma, 0)
            # shifting t by -N/2 multiplies bin m by e^{-2 pi i m (-N/2) / N} = (-1)^m
            sa = (-1.0) ** np.arange(p.N_pad)
            sg = (-1.0) ** np.arange(p.N_fr)
            want = (g_hat * sg)[:, None] * (a_hat * sa)[None, :]
            assert np.max(np.abs(D - want)) <= 1e-10 * np.max(np.abs(want))


def test_spin_conjugates_the_log_frequency_factor():
    # The band-pass with centre -xi is the conjugate of the one with +xi (real Gaussian
    # spectra): along log-frequency the negative-spin pattern carries conj(g) where the
    # positive-spin one carries g (compared at the time where the wavelet peaks).
    p = make_plan(*CFG1)
    n_pos = [i for i, b in enumerate(p.fr) if b.spin > 0]
    n_neg = [i for i, b in enumerate(p.fr) if b.spin < 0]
    assert len(n_pos) == len(n_neg) > 0
    n2 = p.groups[0].n2
    for i, j in zip(n_pos, n_neg):
        Fp = figure.joint_wavelet_complex(p, n2, i, 2048)
        Fn = figure.joint_wavelet_complex(p, n2, j, 2048)
        t0 = int(np.argmax(np.abs(Fp).max(axis=0)))
        a0 = figure.time_wavelet(p, n2)[(t0 - 1024) % p.N_pad]
        gp, gn = Fp[:, t0] / a0, Fn[:, t0] / a0
        assert np.max(np.abs(gn - np.conj(gp))) <= 1e-12 * np.max(np.abs(gp))
        assert np.max(np.abs(gp - figure.freq_wavelet(p, i)[(np.arange(p.N_fr) - p.N_fr // 2) % p.N_fr])) \
            <= 1e-12 * np.max(np.abs(gp))


def test_pattern_peaks_at_the_centre_and_lowpass_pair_is_real_positive():
    # phi_F with the second-order wavelet: the |.| of the product peaks at the centre
    # sample of both axes (both filters peak at their origin); the real part of the
    # phi_F x phi_F-like pattern is even in log-frequency.
    p = make_plan(*CFG1)
    n2 = p.groups[-1].n2
    F = figure.joint_wavelet_complex(p, n2, 0, 4096)
    r0, t0 = np.unravel_index(np.argmax(np.abs(F)), F.shape)
    assert r0 == p.N_fr // 2 and t0 == 2048
    R = figure.joint_wavelet(p, n2, 0, 4096)
    assert np.allclose(R[1:], R[1:][::-1], atol=1e-12 * np.abs(R).max())
