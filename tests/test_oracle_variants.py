"""Pins of the oracle's variants of the method (CPU): the zeroth order (S0 or U0), no
local time averaging of the second order, no frequential averaging (the average_local /
average_local_fr switches of the Sec. 3.3 and 3.5 listings and the Sec. 3.6 main
algorithm), and the S0 weight of the loss."""
import numpy as np
import pytest

from oracle import brute, descent, fftroute
from oracle import filterbank as fb
from oracle.plan import make_plan

TINY = (512, 4, 4, 1, 2, 1, 5, 2)
TINY_B = (384, 4, 3, 2, 2, 2, 4, 3)
FLAGS = [dict(zeroth=True), dict(zeroth=True, average_local=False), dict(average_local_fr=False),
         dict(zeroth=True, average_local=False, average_local_fr=False)]


@pytest.mark.parametrize("args", [TINY, TINY_B])
@pytest.mark.parametrize("flags", FLAGS)
def test_brute_force_equals_fourier_route(args, flags):
    # direct circular convolutions and index-stride decimation (no FFT) against the
    # Fourier route, under each variant's rules
    p = make_plan(*args, **flags)
    x = np.random.default_rng(2).standard_normal(p.N)
    S1 = brute.forward(p, x)
    S2 = fftroute.forward(p, x)
    assert S1.shape == S2.shape == (p.n_coeff,)
    assert np.linalg.norm(S1 - S2) <= 1e-12 * np.linalg.norm(S2)


def test_layout_of_the_variants():
    base = make_plan(*TINY)
    z = make_plan(*TINY, zeroth=True)
    u = make_plan(*TINY, zeroth=True, average_local=False)
    f = make_plan(*TINY, average_local_fr=False)
    # S0: one row of the kept frames first; U0: the N samples first; the rest shifted
    assert z.blocks[0].order == 0 and z.blocks[0].n_frames == base.n_frames
    assert z.n_coeff == base.n_coeff + base.n_frames
    assert u.blocks[0].n_frames == base.N and u.blocks[0].t_lo == base.pad_left
    # unaveraged second order: every path keeps its own time resolution 2^j2
    for blk in u.blocks:
        if blk.order == 2:
            assert blk.n_frames == -(-(u.pad_left + u.N) // (1 << blk.j2)) - (-(-u.pad_left // (1 << blk.j2)))
    # without frequential averaging, band-pass paths keep their own log-frequency stride
    for blk in f.blocks:
        b = f.fr[blk.n_fr]
        if blk.order >= 1 and not b.lowpass:
            K = f.N1 if blk.order == 1 else next(g.K for g in f.groups if g.n2 == blk.n2)
            assert b.k == b.j and blk.n_lambda == -(-K // (1 << b.k))


def test_s0_of_a_constant_is_that_constant_periodic():
    # phi_T has unit DC gain: in periodic mode S0 of a constant signal is the constant
    p = make_plan(1024, 4, 4, 1, 2, 1, 5, 2, periodic=True, zeroth=True)
    S = fftroute.forward(p, np.full(p.N, 0.7))
    blk = p.blocks[0]
    assert np.allclose(S[blk.offset: blk.offset + blk.n_frames], 0.7, rtol=0, atol=1e-13)


def test_s0_is_the_sampled_lowpass_of_x():
    # S0 against the time-domain phi_T (continuous Gaussian, periodised) by direct sums
    p = make_plan(*TINY_B, zeroth=True)
    x = np.random.default_rng(3).standard_normal(p.N)
    S = fftroute.forward(p, x)
    xp = np.zeros(p.N_pad)
    xp[p.pad_left: p.pad_left + p.N] = x
    h = fb.lowpass_time(p.N_pad, p.sigma_T, 0)
    blk = p.blocks[0]
    for i, f in enumerate(range(blk.t_lo, blk.t_lo + blk.n_frames)):
        want = sum(xp[n] * h[(f * p.T - n) % p.N_pad] for n in range(p.N_pad))
        assert abs(S[blk.offset + i] - want) <= 1e-12 * np.max(np.abs(xp))


@pytest.mark.parametrize("flags", FLAGS)
def test_shift_equivariance_and_homogeneity(flags):
    # periodic mode: rolling x by 2^J (a multiple of every stride of the unaveraged
    # outputs and of T here) rolls every row of every block by its own stride; and
    # S(c x) = |c| S(x) for the paths through a modulus, c S(x) for the zeroth order
    args = (1024, 4, 4, 2, 2, 2, 4, 2)
    p = make_plan(*args, periodic=True, **flags)
    x = np.random.default_rng(4).standard_normal(p.N)
    S = fftroute.forward(p, x)
    c = np.full(p.n_coeff, 2.5)
    for blk in p.blocks:
        if blk.order == 0:
            c[blk.offset: blk.offset + blk.n_frames] = -2.5
    assert np.allclose(fftroute.forward(p, -2.5 * x), c * S, rtol=1e-12, atol=1e-14 * np.abs(S).max())
    sh = 1 << max(p.J, p.log2_T)
    Ss = fftroute.forward(p, np.roll(x, sh))
    for blk in p.blocks:
        a = S[blk.offset: blk.offset + blk.n_lambda * blk.n_frames].reshape(blk.n_lambda, blk.n_frames)
        b = Ss[blk.offset: blk.offset + blk.n_lambda * blk.n_frames].reshape(blk.n_lambda, blk.n_frames)
        stride = p.N // blk.n_frames
        assert np.allclose(np.roll(a, sh // stride, axis=1), b, rtol=0, atol=1e-12 * max(np.abs(S).max(), 1e-300))


@pytest.mark.parametrize("flags", FLAGS)
def test_adjoint_and_central_differences(flags):
    # the hand-written adjoint of every variant: <J u, v> = <u, J^T v> through the
    # gradient (central differences at 12 indices, 1e-6 relative) and the Euler identity
    p = make_plan(*TINY_B, **flags)
    rng = np.random.default_rng(5)
    x = rng.standard_normal(p.N)
    y = rng.standard_normal(p.N)
    S_x = fftroute.forward(p, x)
    S_y, cache = fftroute.forward(p, y, return_cache=True)
    E, dS = descent.loss_and_grad_S(S_y, S_x)
    g = fftroute.backward(p, y, dS, cache=cache)
    h = 1e-5
    idx = rng.choice(p.N, 12, replace=False)
    fd = []
    for i in idx:
        yp, ym = y.copy(), y.copy()
        yp[i] += h
        ym[i] -= h
        fd.append((descent.loss_and_grad_S(fftroute.forward(p, yp), S_x)[0]
                   - descent.loss_and_grad_S(fftroute.forward(p, ym), S_x)[0]) / (2 * h))
    fd = np.array(fd)
    assert np.linalg.norm(fd - g[idx]) <= 1e-6 * np.linalg.norm(g[idx])
    # degree-1 homogeneity (the zeroth order is linear): <y, J^T dS> = <S(y), dS>
    assert abs(np.dot(y, g) - np.dot(S_y, dS)) <= 1e-10 * abs(np.dot(S_y, dS))


def test_weighted_loss_of_the_zeroth_order():
    # a weight w0 on the zeroth-order block: E = w0 ||S0(y) - S0(x)||^2 + the rest, and its
    # gradient; w0 = 0 drops the block exactly (Eqs. 5-7 hold S1 and S2 only)
    p = make_plan(*TINY, zeroth=True)
    rng = np.random.default_rng(6)
    S_x = rng.standard_normal(p.n_coeff)
    S_y = rng.standard_normal(p.n_coeff)
    n0 = p.blocks[0].n_frames
    for w0 in (0.0, 0.5, 1.0):
        E, dS = descent.loss_and_grad_S(S_y, S_x, weights=descent.block_weights(p, w0))
        d = S_y - S_x
        assert np.isclose(E, w0 * np.dot(d[:n0], d[:n0]) + np.dot(d[n0:], d[n0:]), rtol=1e-14)
        assert np.allclose(dS[:n0], 2 * w0 * d[:n0]) and np.allclose(dS[n0:], 2 * d[n0:])
