"""Seeded synthetic input signals for the JTFS metamer workloads.

This module is shared by the FP64 oracle and the HIP path; it holds none of the
transform's arithmetic, only the recipes that draw test signals and initial
guesses from a seed (NumPy PCG64 through ``default_rng``).

The paper reconstructs metamers of arbitrary audio recordings (Introduction and
Conclusion) and names no dataset, so music-like synthetic signals stand in:
harmonic tones with 1/k partial amplitudes, slow amplitude modulation, an
optional linear chirp, and white noise 30 dB below the signal.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "harmonic_am_signal",
    "chirp_signal",
    "config1_signal",
    "config2_signal",
    "config4_signal",
    "concatenated_signal",
    "white_noise_like",
    "batched_workload",
    "decoder_init",
]


def harmonic_am_signal(n: int, fs: float, rng: np.random.Generator, n_tones: int = 3,
                       n_partials: int = 6, f0_lo: float = 100.0, f0_hi: float = 800.0,
                       am_lo: float = 2.0, am_hi: float = 8.0, noise_db: float = -30.0) -> np.ndarray:
    """Sum of amplitude-modulated harmonic tones plus white noise, unit RMS before noise.

    Draw order per tone (fixed so that a seed always gives the same signal):
    f0 log-uniform in [f0_lo, f0_hi], AM rate uniform in [am_lo, am_hi], AM phase,
    then one phase per partial k = 1..n_partials (drawn even when the partial is
    dropped because k*f0 reaches the Nyquist frequency). Partial k has amplitude 1/k;
    the envelope of a tone is (1 + sin(2 pi f_am t + phase)) / 2. After the tones are
    summed and scaled to unit RMS, Gaussian noise with variance 10**(noise_db/10) is added.
    """
    t = np.arange(n, dtype=np.float64) / fs
    mix = np.zeros(n, dtype=np.float64)
    for _ in range(n_tones):
        f0 = math.exp(rng.uniform(math.log(f0_lo), math.log(f0_hi)))
        f_am = rng.uniform(am_lo, am_hi)
        am_phase = rng.uniform(0.0, 2.0 * math.pi)
        envelope = 0.5 * (1.0 + np.sin(2.0 * math.pi * f_am * t + am_phase))
        phases = rng.uniform(0.0, 2.0 * math.pi, size=n_partials)
        tone = np.zeros(n, dtype=np.float64)
        for k in range(1, n_partials + 1):
            if k * f0 >= fs / 2.0:
                continue
            tone += np.sin(2.0 * math.pi * k * f0 * t + phases[k - 1]) / k
        mix += envelope * tone
    rms = math.sqrt(float(np.mean(mix * mix)))
    if rms > 0.0:
        mix /= rms
    noise_std = math.sqrt(10.0 ** (noise_db / 10.0))
    mix += rng.normal(0.0, noise_std, size=n)
    return mix


def chirp_signal(n: int, fs: float, rng: np.random.Generator, f_start: float = 200.0,
                 f_stop: float = 4000.0, amplitude: float = 1.0) -> np.ndarray:
    """Linear chirp sweeping f_start -> f_stop over the n samples, random start phase."""
    t = np.arange(n, dtype=np.float64) / fs
    dur = n / fs
    phase0 = rng.uniform(0.0, 2.0 * math.pi)
    inst = 2.0 * math.pi * (f_start * t + 0.5 * (f_stop - f_start) * t * t / dur)
    return amplitude * np.sin(inst + phase0)


def _unit_rms(x: np.ndarray) -> np.ndarray:
    rms = math.sqrt(float(np.mean(x * x)))
    return x / rms if rms > 0.0 else x


def config1_signal(seed: int = 0, n: int = 8192, fs: float = 8000.0) -> np.ndarray:
    """Three harmonic AM tones + noise at -30 dB (8 kHz, 2**13 samples by default)."""
    rng = np.random.default_rng(seed)
    return harmonic_am_signal(n, fs, rng)


def config2_signal(seed: int = 2, n: int = 65536, fs: float = 22050.0) -> np.ndarray:
    """The harmonic AM mixture plus a 200-4000 Hz linear chirp, re-normalised to unit RMS."""
    rng = np.random.default_rng(seed)
    x = harmonic_am_signal(n, fs, rng)
    x = x + chirp_signal(n, fs, rng)
    return _unit_rms(x)


def config4_signal(seed: int, n: int = 65536, fs: float = 8000.0) -> np.ndarray:
    """Config-1 generator at 2**16 samples (warm-start decoder training and held-out signals)."""
    rng = np.random.default_rng(seed)
    return harmonic_am_signal(n, fs, rng)


def concatenated_signal(seed: int, n_segments: int = 16, seg_len: int = 65536,
                        fs: float = 22050.0) -> np.ndarray:
    """Long signal: segments of the harmonic AM generator, each with fresh f0 and AM rate."""
    rng = np.random.default_rng(seed)
    parts = [harmonic_am_signal(seg_len, fs, rng) for _ in range(n_segments)]
    return _unit_rms(np.concatenate(parts))


def standard_normal(n: int, seed: int) -> np.ndarray:
    """n independent standard normal draws (the noise the coloured-noise start shapes)."""
    return np.random.default_rng(seed).standard_normal(n)


def white_noise_like(x: np.ndarray, seed: int) -> np.ndarray:
    """Initial guess of a metamer descent: white Gaussian noise with the RMS of x."""
    rng = np.random.default_rng(seed)
    rms = math.sqrt(float(np.mean(np.asarray(x, dtype=np.float64) ** 2)))
    return rng.normal(0.0, rms, size=np.asarray(x).shape[0])


def batched_workload(n_signals: int = 64, meta_seed: int = 99, first_seed: int = 100,
                     fs: float = 22050.0, log2_n_lo: int = 14, log2_n_hi: int = 17,
                     log2_T_choices=(11, 12, 13), F_choices=(12, 24, 48)):
    """Heterogeneous batch: lengths log-uniform in [2**lo, 2**hi], own T and F per signal.

    Returns a list of (signal, log2_T, F) tuples.
    """
    meta = np.random.default_rng(meta_seed)
    out = []
    for i in range(n_signals):
        n = int(round(math.exp(meta.uniform(log2_n_lo * math.log(2.0), log2_n_hi * math.log(2.0)))))
        log2_T = int(meta.choice(np.asarray(log2_T_choices)))
        F = float(meta.choice(np.asarray(F_choices)))
        rng = np.random.default_rng(first_seed + i)
        out.append((harmonic_am_signal(n, fs, rng), log2_T, F))
    return out


def decoder_init(layers, kernel: int, leak: float, seed: int) -> np.ndarray:
    """Seeded initial parameters of the warm-start decoder, packed flat.

    ``layers`` lists (C_out, C_in, stride) per layer. Layer l contributes its weights
    [C_out, C_in, kernel] (row-major) followed by its C_out biases. Weights are normal
    with standard deviation gain / sqrt(fan_in), where fan_in = C_in * ceil(kernel / stride)
    counts the taps that meet a non-zero sample after zero-stuffing, gain is
    sqrt(2 / (1 + leak^2)) for hidden layers and 1 for the last; biases start at 0.
    """
    rng = np.random.default_rng(seed)
    parts = []
    for idx, (co, ci, s) in enumerate(layers):
        fan_in = ci * (-(-kernel // s))
        gain = 1.0 if idx == len(layers) - 1 else math.sqrt(2.0 / (1.0 + leak * leak))
        parts.append(rng.normal(0.0, gain / math.sqrt(fan_in), size=co * ci * kernel))
        parts.append(np.zeros(co))
    return np.concatenate(parts)
