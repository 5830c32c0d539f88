"""Pins of the coloured-noise descent start (oracle.init) against facts fixed outside it:
the Rayleigh mean of a circular Gaussian, the closed-form response of a pure tone, the
defining property (white noise in -> flat spectrum at the same level out; band means of
the start match those of the target) and the exactness of the shaping in periodic mode.
"""
import math

import numpy as np
import pytest

from oracle import init as OI
from oracle.fftroute import FilterCache, first_layer
from oracle.plan import make_plan


def test_rayleigh_mean_modulus():
    """E|z| = sqrt(pi P) / 2 for a circular complex Gaussian with E|z|^2 = P."""
    rng = np.random.default_rng(0)
    P = 2.7
    z = rng.normal(0, math.sqrt(P / 2), 2_000_000) + 1j * rng.normal(0, math.sqrt(P / 2), 2_000_000)
    assert abs(np.mean(np.abs(z)) - math.sqrt(math.pi * P) / 2) < 2e-3 * math.sqrt(P)


def test_band_levels_of_a_pure_tone():
    """A cos(2 pi k0 n / N) has U1 = (A / 2) |psi1^(k0)| (constant) for every filter whose
    negative-frequency response is negligible; phi_T keeps a constant (gain phi_T^(0))."""
    N = 1 << 14
    plan = make_plan(N, 8, 8, 1, 2, 1, 8, 2, periodic=True)
    fc = FilterCache(plan)
    A, k0 = 1.7, 1234
    x = A * np.cos(2 * np.pi * k0 * np.arange(N) / N)
    m = OI.band_levels(plan, x, fc)
    checked = 0
    for n1, b in enumerate(plan.psi1):
        h = fc.psi1(n1)
        if abs(h[N - k0]) > 1e-9 * max(abs(h[k0]), 1e-300) or abs(h[k0]) < 1e-3 * np.abs(h).max():
            continue
        expect = 0.5 * A * abs(h[k0]) * fc.phi_t(b.k)[0].real
        assert abs(m[n1] - expect) <= 1e-9 * expect + 1e-12, (n1, m[n1], expect)
        checked += 1
    assert checked >= 3


@pytest.mark.parametrize("periodic", [True, False])
def test_white_noise_gives_a_flat_spectrum_at_its_level(periodic):
    """For white x of variance s^2, every band's level per unit filter energy is s^2
    (Rayleigh factor and the per-sample filter energy both enter), so H^2 = s^2 wherever
    the filters have energy."""
    N = 1 << 16 if periodic else (1 << 16) - 1000
    plan = make_plan(N, 8, 8, 1, 2, 1, 6, 2, periodic=periodic)
    fc = FilterCache(plan)
    s = 0.37
    x = s * np.random.default_rng(1).normal(size=N)
    H = OI.spectrum(plan, OI.band_levels(plan, x, fc), fc)
    # bins where the filterbank carries at least 1% of its peak summed energy
    k = np.arange(plan.N_pad)
    kk = np.minimum(k, plan.N_pad - k)
    den = sum(np.abs(fc.psi1(n1)[kk]) ** 2 for n1 in range(plan.N1))
    core = den > 1e-2 * den.max()
    ratio = H[core] ** 2 / s ** 2
    assert abs(np.median(ratio) - 1.0) < 0.03, np.median(ratio)
    assert np.quantile(ratio, 0.02) > 0.8 and np.quantile(ratio, 0.98) < 1.2, np.quantile(ratio, [0.02, 0.98])


def test_start_matches_the_band_means_of_a_coloured_target():
    """The defining property: S1 of the start has (about) the band means of S1 x, for a
    target whose spectrum falls by 30 dB over the filterbank."""
    N = 1 << 16
    plan = make_plan(N, 8, 8, 1, 2, 1, 6, 2, periodic=True)
    fc = FilterCache(plan)
    rng = np.random.default_rng(2)
    f = np.fft.rfftfreq(N)
    tilt = 1.0 / (1.0 + (f / 0.02) ** 1.5)
    x = np.fft.irfft(np.fft.rfft(rng.normal(size=N)) * tilt, n=N)
    m_x = OI.band_levels(plan, x, fc)
    y0 = OI.colored_noise(plan, x, rng.normal(size=N), fc)
    m_y = OI.band_levels(plan, y0, fc)
    rel = m_y / m_x
    assert np.median(np.abs(rel - 1.0)) < 0.05, rel
    assert np.all(np.abs(rel - 1.0) < 0.35), rel


def test_shaping_is_exact_in_periodic_mode_and_linear():
    N = 1 << 12
    plan = make_plan(N, 6, 4, 1, 2, 1, 5, 2, periodic=True)
    rng = np.random.default_rng(3)
    H = np.abs(rng.normal(size=N))
    H = 0.5 * (H + np.roll(H[::-1], 1))          # H_k = H_{N-k}: a real filter
    w = rng.normal(size=N)
    y = OI.shape(plan, H, w)
    np.testing.assert_allclose(np.fft.fft(y), H * np.fft.fft(w), atol=1e-9 * np.abs(np.fft.fft(w)).max())
    np.testing.assert_allclose(OI.shape(plan, H, 2.5 * w), 2.5 * y, rtol=1e-12, atol=1e-12)
    assert np.all(OI.spectrum(plan, np.zeros(plan.N1)) == 0.0)
