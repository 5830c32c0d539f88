"""Pins of the oracle's filterbanks against what the paper and the mathematics fix (CPU)."""
import math

import numpy as np
import pytest

from oracle import filterbank as fb
from oracle.plan import make_plan


# ---------------------------------------------------------------- Sec. 3.1 generator

def test_q1_bank_closed_form():
    # With Q = 1 the generator starts at xi = max(1/9, 0.35) = 0.35; the -3 dB rule gives
    # sigma = (1/3) xi / sqrt(ln 2), and both halve at every step (no linear region).
    for J in (3, 6, 9):
        bank = fb.morlet_bank(J, 1)
        for n, (xi, s) in enumerate(bank):
            assert xi == pytest.approx(0.35 * 2.0 ** -n, rel=1e-14)
            assert s == pytest.approx(0.35 / (3.0 * math.sqrt(math.log(2.0))) * 2.0 ** -n, rel=1e-14)
        # the last constant-Q width is the first one not above twice sigma0 / 2^J
        s_min = 0.1 / 2 ** J
        assert bank[-1][1] > s_min and bank[-1][1] <= 2 * s_min


def test_sigma_top_value():
    # Q = 1: sigma_0 = 0.35 / (3 sqrt(ln 2)) = 0.140131...
    assert fb.morlet_bank(4, 1)[0][1] == pytest.approx(0.1401309, abs=1e-7)


@pytest.mark.parametrize("J,Q", [(6, 8), (12, 12), (14, 16), (12, 2), (4, 2), (5, 3), (8, 1)])
def test_bank_structure_and_count(J, Q):
    bank = fb.morlet_bank(J, Q)
    xi_top = max(1.0 / (1.0 + 2.0 ** (3.0 / Q)), 0.35)
    r = 2.0 ** (1.0 / Q)
    s_top = (r - 1.0) / (r + 1.0) * xi_top / math.sqrt(math.log(2.0))
    s_min = 0.1 / 2 ** J
    # independent count: constant-Q members are the n >= 0 with s_top r^-n > s_min
    n_cq = int(math.floor(Q * math.log2(s_top / s_min))) + 1
    assert len(bank) == n_cq + (Q - 1)
    cq, lin = bank[:n_cq], bank[n_cq:]
    for a, b in zip(cq, cq[1:]):
        assert a[0] / b[0] == pytest.approx(r, rel=1e-13)
        assert a[1] / b[1] == pytest.approx(r, rel=1e-13)
        assert a[0] / a[1] == pytest.approx(xi_top / s_top, rel=1e-12)   # constant Q
    elbow = cq[-1][0]
    for q, (xi, s) in enumerate(lin, start=1):
        assert s == s_min
        assert xi == pytest.approx(elbow * (1.0 - q / Q), rel=1e-12)
    xis = [b[0] for b in bank]
    assert all(a > b > 0 for a, b in zip(xis, xis[1:]))


def _constant_q_count_decimal(J: int, Q: int):
    """Count of constant-Q members, k >= 0 with sigma_top 2^(-k/Q) > sigma0 / 2^J, evaluated
    with 60-digit decimal arithmetic (independent of the float code), and how close
    R = Q log2(sigma_top / sigma_min) lies to an integer (a tie of the rule)."""
    from decimal import Decimal, getcontext
    getcontext().prec = 60
    two = Decimal(2)
    ln2 = two.ln()
    p2 = lambda e: (Decimal(e) * ln2).exp()            # 2^e
    xi_top = max(Decimal(1) / (1 + p2(Decimal(3) / Q)), Decimal("0.35"))
    f = p2(Decimal(-1) / Q)
    # sqrt(2 ln(1 / r_psi)) with r_psi = sqrt(1/2) is sqrt(ln 2)
    s_top = (1 - f) / (1 + f) * xi_top / ln2.sqrt()
    s_min = Decimal("0.1") / (two ** J)
    if s_top <= s_min:
        return 0, None
    R = Q * (s_top / s_min).ln() / ln2
    n = int(R.to_integral_value(rounding="ROUND_CEILING"))
    return max(1, n), float(abs(R - R.to_integral_value()))


def test_constant_q_count_against_high_precision():
    # Every (J, Q) in a wide grid: the float count equals the exact one; the pairs whose
    # R lies closest to an integer (the boundary cases of the rule) are included.
    closest = []
    for J in range(0, 21):
        for Q in range(1, 33):
            n_ref, dist = _constant_q_count_decimal(J, Q)
            bank = fb.morlet_bank(J, Q)
            n_cq = sum(1 for (_, s) in bank if s > 0.1 / 2 ** J)
            assert n_cq == n_ref, (J, Q)
            assert len(bank) == n_ref + Q - 1, (J, Q)
            if dist is not None:
                closest.append((dist, J, Q))
    closest.sort()
    # the nearest approach to a tie stays far above the 1e-9 tie tolerance
    assert closest[0][0] > 1e-6


def test_bank_sizes_of_the_workloads():
    # N1 = constant-Q + (Q - 1) linear members at configs 1, 2, 5; N2 at Q2 = 1 and 2
    assert len(fb.morlet_bank(6, 8)) == 38
    assert len(fb.morlet_bank(12, 12)) == 124
    assert len(fb.morlet_bank(14, 16)) == 191
    assert len(fb.morlet_bank(6, 1)) == 7
    assert len(fb.morlet_bank(12, 2)) == 25
    assert len(fb.morlet_bank(14, 2)) == 29


def test_no_constant_q_room():
    # J = 0 with Q = 1: sigma_top = 0.14 > 0.1, so one constant-Q member; a tiny J and a
    # large Q leave none, and the linear members then step down from sigma_top
    bank = fb.morlet_bank(0, 1)
    assert len(bank) == 1
    xi_top = 1.0 / (1.0 + 2.0 ** (3.0 / 40))  # 0.487 > 0.35
    f = 2.0 ** (-1.0 / 40)
    s_top = (1 - f) / (1 + f) * xi_top / math.sqrt(math.log(2.0))
    assert s_top < 0.1                       # no room at J = 0, Q = 40
    bank = fb.morlet_bank(0, 40)
    assert len(bank) == 39
    for q, (xi, s) in enumerate(bank, start=1):
        assert s == 0.1
        assert xi == pytest.approx(s_top * (1 - q / 40), rel=1e-14)


def test_adjacent_constant_q_filters_cross_at_minus_3db():
    # r_psi = sqrt(1/2): neighbouring Gaussians intersect at sqrt(1/2) of their peak.
    for J, Q in [(6, 8), (12, 12), (10, 2), (8, 1)]:
        bank = fb.morlet_bank(J, Q)
        n_cq = sum(1 for (_, s) in bank if s > 0.1 / 2 ** J)
        for (xa, sa), (xb, sb) in zip(bank[: n_cq - 1], bank[1:n_cq]):
            w = (xa * sb + xb * sa) / (sa + sb)          # where (w-xa)/sa = (xb-w)/sb
            assert math.exp(-((w - xa) / sa) ** 2 / 2) == pytest.approx(math.sqrt(0.5), rel=1e-12)
            assert math.exp(-((w - xb) / sb) ** 2 / 2) == pytest.approx(math.sqrt(0.5), rel=1e-12)


def test_spin_negates_centres_keeps_widths():
    bank = fb.morlet_bank(4, 2)
    sp = fb.spun(bank)
    assert sp[: len(bank)] == bank
    assert sp[len(bank):] == [(-x, s) for (x, s) in bank]


def test_subsampling_scale_hand_values():
    # edge = |xi| + 5 sigma; j = largest j with edge <= 2^-(j+1)
    assert fb.subsampling_scale(0.35, 0.140131) == 0            # edge 1.05
    assert fb.subsampling_scale(0.04375, 0.0175164) == 1         # edge 0.131 in (1/8, 1/4]
    assert fb.subsampling_scale(-0.04375, 0.0175164) == 1
    assert fb.subsampling_scale(0.0, 0.1 / 4) == 2               # edge 0.125 = 2^-3 exactly
    assert fb.subsampling_scale(0.0, 0.1 / 4 * 1.0000001) == 1


# ---------------------------------------------------------------- Eq. 1 closed forms

@pytest.mark.parametrize("L,xi,sigma,level", [
    (256, 0.35, 0.14013, 0), (512, 0.1, 0.02, 0), (128, 0.0437, 0.0175, 1),
    (1024, 0.2, 0.01, 0), (64, -0.175, 0.07, 0), (2048, 0.0031, 0.00125, 3),
])
def test_morlet_time_and_fourier_forms_are_a_dft_pair(L, xi, sigma, level):
    # The time-sampled, L-periodised continuous Morlet (Eq. 1 shape) has as DFT the
    # period-1 periodised Gaussian closed form (Poisson summation).
    h_t = fb.bandpass_time(L, xi, sigma, level)
    h_f = fb.bandpass_hat(L, xi, sigma, level)
    assert np.max(np.abs(np.fft.fft(h_t) - h_f)) <= 1e-12 * np.max(np.abs(h_f))


@pytest.mark.parametrize("L,sigma,level", [(256, 0.1 / 32, 0), (512, 0.1 / 4, 1), (64, 0.1 / 24, 0), (32, 0.1 / 2, 2)])
def test_gaussian_time_and_fourier_forms_are_a_dft_pair(L, sigma, level):
    p_t = fb.lowpass_time(L, sigma, level)
    p_f = fb.lowpass_hat(L, sigma, level)
    assert np.max(np.abs(np.fft.fft(p_t) - p_f)) <= 1e-12
    assert p_f[0] == 1.0 and np.all(p_t >= 0) and np.argmax(p_t) == 0


def test_morlet_time_shape_is_equation_1():
    # Eq. 1 with lambda = xi and its Q equal to xi / (2 pi sigma): Gaussian envelope
    # exp(-lambda^2 t^2 / (2 Q^2)) times (exp(2 pi i lambda t) - kappa), up to a constant.
    xi, sigma = 0.2, 0.03
    Q_eq1 = xi / (2 * math.pi * sigma)
    kappa = fb.morlet_kappa_time(xi, sigma)
    t = np.linspace(-40, 40, 161)
    eq1 = xi * np.exp(-(xi ** 2) * t ** 2 / (2 * Q_eq1 ** 2)) * (np.exp(2j * math.pi * xi * t) - kappa)
    ours = fb.morlet_time_continuous(t, xi, sigma, kappa)
    ratio = ours / eq1
    assert np.allclose(ratio, ratio[80], rtol=1e-12)


@pytest.mark.parametrize("L,xi,sigma,level", [(256, 0.35, 0.14013, 0), (4096, 0.005, 0.00244, 0), (512, 0.0437, 0.0175, 2)])
def test_vanishing_moment(L, xi, sigma, level):
    h_f = fb.bandpass_hat(L, xi, sigma, level)
    assert abs(h_f[0]) <= 1e-15
    h_t = fb.bandpass_time(L, xi, sigma, level)
    assert abs(h_t.sum()) <= 1e-12 * np.max(np.abs(h_t))


def test_peak_gain_about_one():
    # Reading of Eq. 1's lambda prefactor: the Fourier peak of every band-pass is ~1.
    for xi, s in fb.morlet_bank(8, 4):
        h = fb.bandpass_hat(1 << 14, xi, s)
        assert 0.95 < np.max(np.abs(h)) <= 1.0 + 1e-12


# ---------------------------------------------------------------- Littlewood-Paley

@pytest.mark.parametrize("args,cq_lo,cq_hi", [
    ((8192, 6, 8, 1, 3, 1, 9, 4), 0.99, 1.13),
    ((65536, 12, 12, 2, 4, 2, 13, 24), 0.99, 1.13),
])
def test_littlewood_paley_sum(args, cq_lo, cq_hi):
    p = make_plan(*args)
    L = p.N_pad
    A = np.zeros(L)
    for b in p.psi1:
        h = fb.bandpass_hat(L, b.xi, b.sigma)
        A += np.abs(h) ** 2 + np.abs(np.roll(h[::-1], 1)) ** 2
    A += 2 * np.abs(fb.lowpass_hat(L, p.sigma_T)) ** 2
    w = np.arange(L) / L
    n_cq = sum(1 for b in p.psi1 if b.sigma > 0.1 / 2 ** p.J)
    band = (w >= p.psi1[n_cq - 1].xi) & (w <= p.psi1[0].xi)
    assert cq_lo <= A[band].min() and A[band].max() <= cq_hi
    # Parseval: sum_l ||x * psi_l||^2 + ||x * phi||^2 = (1/L) sum_m A'(m)|X(m)|^2
    rng = np.random.default_rng(5)
    x = rng.standard_normal(L)
    X = np.fft.fft(x)
    lhs = 0.0
    Ap = np.zeros(L)
    for b in p.psi1:
        h = fb.bandpass_hat(L, b.xi, b.sigma)
        lhs += np.sum(np.abs(np.fft.ifft(X * h)) ** 2)
        Ap += np.abs(h) ** 2
    ph = fb.lowpass_hat(L, p.sigma_T)
    lhs += np.sum(np.abs(np.fft.ifft(X * ph)) ** 2)
    Ap += ph ** 2
    rhs = np.sum(Ap * np.abs(X) ** 2) / L
    assert lhs == pytest.approx(rhs, rel=1e-12)
