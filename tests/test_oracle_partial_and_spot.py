"""Pins of the oracle at full size (CPU): the partial forward used for sampled parity, and
direct time-domain spot checks of the Fourier route at the N = 2^16 workload."""
import numpy as np
import pytest

import jtfs_inputs as ji
from oracle import fftroute
from oracle import filterbank as fb
from oracle.plan import make_plan

TINY_B = (384, 4, 3, 2, 2, 2, 4, 3)          # N, J, Q1, Q2, J_fr, Q_fr, log2_T, F
CFG1 = (8192, 6, 8, 1, 3, 1, 9, 4.0)
CFG2 = (65536, 12, 12, 2, 4, 2, 13, 24.0)


def _subsets(groups, rng):
    n2s = [g.n2 for g in groups]
    return [[], n2s[:1], n2s[-1:], sorted(rng.choice(n2s, size=min(3, len(n2s)), replace=False).tolist()), n2s]


@pytest.mark.parametrize("args", [TINY_B, CFG1])
def test_forward_partial_equals_forward(args):
    # every block forward_partial fills equals forward's (it fills exactly the asked-for
    # blocks, the rest stays NaN), for several n2 subsets, with and without order 1
    p = make_plan(*args)
    rng = np.random.default_rng(11)
    x = rng.standard_normal(p.N)
    fc = fftroute.FilterCache(p)
    S = fftroute.forward(p, x, fc=fc)
    for n2s in _subsets(p.groups, rng):
        for order1 in (True, False):
            Sp = fftroute.forward_partial(p, x, n2s, order1=order1, fc=fc)
            for blk in p.blocks:
                sl = slice(blk.offset, blk.offset + blk.n_lambda * blk.n_frames)
                filled = (blk.order == 1 and order1) or (blk.order == 2 and blk.n2 in n2s)
                if filled:
                    assert not np.any(np.isnan(Sp[sl]))
                    assert np.max(np.abs(Sp[sl] - S[sl])) <= 1e-13 * max(np.max(np.abs(S[sl])), 1e-300)
                else:
                    assert np.all(np.isnan(Sp[sl]))


def _direct_conv_samples(sig: np.ndarray, h: np.ndarray, k: int, ts: np.ndarray) -> np.ndarray:
    """y[t] = sum_n sig[n] h[(t 2^k - n) mod L] at the listed output times, one O(L) dot
    product each (no FFT)."""
    L = sig.shape[0]
    n = np.arange(L)
    return np.array([np.dot(sig, h[((int(t) << k) - n) % L]) for t in ts])


@pytest.mark.slow
def test_config2_spot_checks_against_direct_sums():
    # 256 random first- and second-layer coefficients at N = 2^16 (J = 12, Q1 = 12): each is
    # an O(N_pad) circular sum with the time-domain filter built from the continuous Morlet,
    # compared with the Fourier route. Second-layer sums take the Fourier route's U1 row
    # as input (itself pinned by the first-layer sums).
    p = make_plan(*CFG2)
    x = ji.config2_signal(2)
    fc = fftroute.FilterCache(p)
    _, Z1, U1h, _ = fftroute.first_layer(p, x, fc)
    xp = fftroute.pad_signal(p, x)
    rng = np.random.default_rng(7)

    # first layer: Z1[n1][t] (complex) and U1 = |Z1|, 128 samples over 32 random rows
    for n1 in rng.choice(p.N1, size=32, replace=False):
        b = p.psi1[n1]
        h = fb.bandpass_time(p.N_pad, b.xi, b.sigma, 0)
        ts = rng.integers(0, p.N_pad >> b.k, size=4)
        got = _direct_conv_samples(xp, h, b.k, ts)
        ref = Z1[n1][ts]
        scale = np.max(np.abs(Z1[n1]))
        assert np.max(np.abs(got - ref)) <= 1e-12 * scale, n1
        assert np.max(np.abs(np.abs(got) - np.abs(ref))) <= 1e-12 * scale, n1

    # second layer: Y2[n2][n1][t] for 128 samples over random (n2, n1) pairs
    checked = 0
    groups = list(p.groups)
    while checked < 128:
        grp = groups[rng.integers(len(groups))]
        Y = fftroute.second_layer_group(p, grp, U1h, fc)
        b2 = p.psi2[grp.n2]
        for n1 in rng.choice(grp.K, size=min(4, grp.K), replace=False):
            k1 = p.psi1[n1].k
            L1 = p.N_pad >> k1
            u1 = np.abs(np.fft.ifft(U1h[n1]))        # U1 row of the Fourier route (real)
            h2 = fb.bandpass_time(L1, b2.xi, b2.sigma, k1)
            ts = rng.integers(0, p.N_pad >> grp.j2, size=4)
            got = _direct_conv_samples(u1, h2, grp.j2 - k1, ts)
            ref = Y[n1][ts]
            scale = np.max(np.abs(Y[n1]))
            assert np.max(np.abs(got - ref)) <= 1e-12 * scale, (grp.n2, n1)
            checked += len(ts)
