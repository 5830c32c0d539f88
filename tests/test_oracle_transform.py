"""Pins of the oracle's forward transform (CPU): brute force, closed forms, invariances."""
import math

import numpy as np
import pytest

from oracle import brute, fftroute
from oracle import filterbank as fb
from oracle.plan import make_plan

TINY = (512, 4, 4, 1, 2, 1, 5, 2)          # N, J, Q1, Q2, J_fr, Q_fr, log2_T, F
TINY_B = (384, 4, 3, 2, 2, 2, 4, 3)        # non power-of-two N, Q2 = Q_fr = 2, F not a power of 2


def blocks_of(plan, order=None):
    return [b for b in plan.blocks if order is None or b.order == order]


def block(plan, S, blk):
    return S[blk.offset: blk.offset + blk.n_lambda * blk.n_frames].reshape(blk.n_lambda, blk.n_frames)


def test_fourier_subsampling_equals_decimation():
    rng = np.random.default_rng(1)
    X = rng.standard_normal(256) + 1j * rng.standard_normal(256)
    for k in range(5):
        lhs = np.fft.ifft(fftroute.fold(X, k))
        rhs = np.fft.ifft(X)[:: 1 << k]
        assert np.max(np.abs(lhs - rhs)) <= 1e-14 * np.max(np.abs(rhs))


@pytest.mark.parametrize("args,periodic", [(TINY, False), (TINY_B, False), ((1024, 4, 4, 1, 2, 1, 5, 2), True)])
def test_brute_force_equals_fourier_route(args, periodic):
    p = make_plan(*args, periodic=periodic)
    rng = np.random.default_rng(2)
    x = rng.standard_normal(p.N)
    S_o1, mid = brute.forward(p, x, return_intermediates=True)
    S_o2, cache = fftroute.forward(p, x, return_cache=True)
    assert np.linalg.norm(S_o1 - S_o2) <= 1e-12 * np.linalg.norm(S_o2)
    for n1 in range(p.N1):
        assert np.max(np.abs(mid["Z1"][n1] - cache["Z1"][n1])) <= 1e-12 * np.max(np.abs(cache["Z1"][n1]))
    assert np.max(np.abs(mid["S1"] - cache["S1"])) <= 1e-12 * np.max(np.abs(cache["S1"]))


def test_impulse_response_is_the_morlet():
    # x = delta at n0 (periodic): Z1[t] = psi[(t 2^k1 - n0) mod N], the sampled Eq. 1 Morlet.
    p = make_plan(1024, 5, 4, 1, 2, 1, 6, 2, periodic=True)
    n0 = 37
    x = np.zeros(p.N)
    x[n0] = 1.0
    Z1, _, _ = fftroute.first_order_only(p, x)
    for n1, b in enumerate(p.psi1):
        h = fb.bandpass_time(p.N, b.xi, b.sigma, 0)
        t = np.arange(p.N >> b.k)
        want = h[((t << b.k) - n0) % p.N]
        assert np.max(np.abs(Z1[n1] - want)) <= 1e-12 * np.max(np.abs(want))


def test_pure_tone_scalogram_closed_form():
    # x = A cos(2 pi m0 n / N + th): Z1[t] = A/2 (psi^[m0] e^{i th} e^{2 pi i m0 t 2^k/N}
    #                                            + psi^[N-m0] e^{-i th} e^{-2 pi i m0 t 2^k/N})
    p = make_plan(2048, 6, 4, 1, 2, 1, 7, 2, periodic=True)
    A, m0, th = 1.7, 301, 0.4
    n = np.arange(p.N)
    x = A * np.cos(2 * math.pi * m0 * n / p.N + th)
    Z1, _, S1 = fftroute.first_order_only(p, x)
    for n1, b in enumerate(p.psi1):
        h = fb.bandpass_hat(p.N, b.xi, b.sigma)
        t = np.arange(p.N >> b.k) << b.k
        want = A / 2 * (h[m0] * np.exp(1j * th) * np.exp(2j * math.pi * m0 * t / p.N)
                        + h[p.N - m0] * np.exp(-1j * th) * np.exp(-2j * math.pi * m0 * t / p.N))
        assert np.max(np.abs(Z1[n1] - want)) <= 1e-12 * A
        # U1 is constant up to the negative-frequency leakage, and phi_T has unit DC gain
        lo, hi = A / 2 * (abs(h[m0]) - abs(h[p.N - m0])), A / 2 * (abs(h[m0]) + abs(h[p.N - m0]))
        assert np.all(S1[n1] >= lo - 1e-12) and np.all(S1[n1] <= hi + 1e-12)


def test_frequential_filter_orientation():
    # An impulse at log-frequency row n0 gives V[r] = g[(r 2^k - n0) mod N_fr] (convolution).
    p = make_plan(*TINY)
    fc = fftroute.FilterCache(p)
    n0 = 5
    Y = np.zeros((p.N_fr, 3), dtype=np.complex128)
    Y[n0] = 1.0
    Yh = np.fft.fft(Y, axis=0)
    for g, b in enumerate(p.fr):
        V = fftroute.freq_filter(p, Yh, g, fc)
        if b.lowpass:
            gt = fb.lowpass_time(p.N_fr, b.sigma)
        else:
            gt = fb.bandpass_time(p.N_fr, b.xi, b.sigma)
        r = np.arange(p.N_fr >> b.k)
        want = gt[((r << b.k) - n0) % p.N_fr]
        assert np.max(np.abs(V[:, 0] - want)) <= 1e-12 * np.max(np.abs(want))


def test_homogeneity_sign_and_zero():
    p = make_plan(*TINY)
    rng = np.random.default_rng(3)
    x = rng.standard_normal(p.N)
    S = fftroute.forward(p, x)
    assert np.linalg.norm(fftroute.forward(p, -2.5 * x) - 2.5 * S) <= 1e-12 * np.linalg.norm(S)
    assert np.linalg.norm(fftroute.forward(p, 0.01 * x) - 0.01 * S) <= 1e-12 * np.linalg.norm(S)
    assert np.all(fftroute.forward(p, np.zeros(p.N)) == 0.0)
    assert np.all(S >= 0)


def test_shift_by_T_rolls_frames():
    p = make_plan(1024, 4, 4, 1, 2, 1, 5, 2, periodic=True)
    rng = np.random.default_rng(4)
    x = rng.standard_normal(p.N)
    S = fftroute.forward(p, x)
    Ss = fftroute.forward(p, np.roll(x, p.T))
    for blk in p.blocks:
        assert np.max(np.abs(block(p, Ss, blk) - np.roll(block(p, S, blk), 1, axis=1))) <= 1e-12 * np.max(S)


def test_small_shift_changes_little():
    # Invariance to shifts well below T (Sec. 2.2): relative change grows with the shift.
    p = make_plan(2048, 5, 4, 1, 2, 1, 8, 2, periodic=True)
    rng = np.random.default_rng(6)
    x = rng.standard_normal(p.N)
    S = fftroute.forward(p, x)
    rel = [np.linalg.norm(fftroute.forward(p, np.roll(x, tau)) - S) / np.linalg.norm(S) for tau in (4, 16, 64)]
    assert rel[0] < rel[1] < rel[2]
    assert rel[0] < 0.63 * 4 / p.T


def test_transposition_changes_little_up_to_F():
    # Invariance to frequency transposition up to F (Sec. 2.2): moving a tone by one
    # first-order bin (a factor 2^(1/Q1)) changes S by a small fraction that grows with the
    # shift, and the change per bin shrinks as the frequential averaging F widens. Missing
    # or misplaced phi_F averaging along log-frequency makes a one-bin move large.
    N, Q1 = 1 << 13, 8

    def tone(f):
        k = round(f * N)
        return np.cos(2 * np.pi * k * np.arange(N) / N)

    def rel_change(F, bins):
        p = make_plan(N, 8, Q1, 1, 3, 1, 9, F, periodic=True)
        a = fftroute.forward(p, tone(0.04))
        return [np.linalg.norm(fftroute.forward(p, tone(0.04 * 2 ** (b / Q1))) - a) / np.linalg.norm(a)
                for b in bins]

    wide = rel_change(8, (1, 4, 16))     # F = 8 bins, one octave
    assert wide[0] < wide[1] < wide[2]
    assert wide[0] < 0.1 and wide[2] > 0.5
    narrow = rel_change(2, (1,))         # F = 2 bins
    assert narrow[0] > 2.5 * wide[0]


def test_time_reversal_swaps_spin():
    p = make_plan(1024, 4, 4, 2, 2, 2, 5, 2, periodic=True)
    rng = np.random.default_rng(7)
    x = rng.standard_normal(p.N)
    S = fftroute.forward(p, x)
    Sr = fftroute.forward(p, x[(-np.arange(p.N)) % p.N])
    n_pos = sum(1 for b in p.fr if b.spin > 0)

    def swap(g):
        s = p.fr[g].spin
        return g if s == 0 else (g + n_pos if s > 0 else g - n_pos)

    index = {(b.order, b.n2, b.n_fr): b for b in p.blocks}
    rev = lambda a: a[:, (-np.arange(a.shape[1])) % a.shape[1]]
    for blk in p.blocks:
        partner = index[(blk.order, blk.n2, blk.n_fr if blk.order == 1 else swap(blk.n_fr))]
        assert np.max(np.abs(block(p, Sr, blk) - rev(block(p, S, partner)))) <= 1e-12 * np.max(S)


def test_output_layout_counts():
    # Sizes of the JTFS output under the plan's readings, counted independently here:
    # order 1: (1 + #positive frequential wavelets) blocks of ceil(N1/2^sF) x frames;
    # order 2: for each n2 with K > 0, |fr list| blocks of ceil(K/2^sF) x frames.
    p = make_plan(8192, 6, 8, 1, 3, 1, 9, 4)
    nf = 16                              # frames f with 4096 <= 512 f < 12288
    n_pos = len(fb.morlet_bank(3, 1))
    o1 = (1 + n_pos) * math.ceil(p.N1 / 4) * nf
    Ks = [sum(1 for b1 in p.psi1 if b1.j < b2.j) for b2 in p.psi2]
    o2 = sum((1 + 2 * n_pos) * math.ceil(K / 4) * nf for K in Ks if K > 0)
    assert p.n_frames == nf and p.n_coeff == o1 + o2
