"""O2: JTFS forward through the Fourier route, and its exact adjoint (oracle, FP64).

Follows the paper's implementation section step by step:
* first layer (Sec. 3.2): FFT of the padded signal, product with each first-order
  filter, Fourier-domain subsampling by 2^k1 (average of the 2^k1 aliased blocks),
  inverse FFT, modulus, FFT again;
* first-order averaging S1 = U1 * phi_T subsampled to T (Eq. 3);
* frequential scattering (Sec. 3.5): the log-frequency axis is zero-padded to N_fr,
  transformed, multiplied by each frequential filter, Fourier-subsampled by 2^k_fr and
  inverse-transformed; real inputs (alpha = 0) use phi_F and the positive spins only;
* second layer in width-first order (Sec. 3.3): for each n2, all rows n1 with j2 > j1
  are filtered by the second-order wavelet at level k1 and stacked;
* modulus and phi_T / phi_F averaging of every joint path (Eq. 2, Eq. 4).

The adjoint composes the Hermitian adjoints of these linear steps in reverse order
with the derivative of the modulus (Sec. 2.3, Eqs. 5-7); it is the exact gradient of
the forward, with the subgradient 0 where a modulus argument is exactly 0.

Fourier subsampling normalisation: X_sub[m] = 2^-k sum_b X[m + b L / 2^k], so that
ifft(X_sub) equals the 2^k-decimation of ifft(X) exactly.
"""
from __future__ import annotations

import numpy as np

from . import filterbank as fb
from .plan import OraclePlan


# ----------------------------------------------------------------------------- helpers

def fold(z: np.ndarray, k: int, axis: int = -1) -> np.ndarray:
    """Fourier-domain subsampling by 2^k along ``axis``: mean of the 2^k aliased blocks."""
    if k == 0:
        return z
    z = np.moveaxis(z, axis, -1)
    L = z.shape[-1]
    out = z.reshape(z.shape[:-1] + (1 << k, L >> k)).mean(axis=-2)
    return np.moveaxis(out, -1, axis)


def tile(z: np.ndarray, k: int, axis: int = -1) -> np.ndarray:
    """Periodic extension by 2^k along ``axis`` (the transpose of a block sum)."""
    if k == 0:
        return z
    reps = [1] * z.ndim
    reps[axis] = 1 << k
    return np.tile(z, reps)


def _bcast(h: np.ndarray, ndim: int, axis: int) -> np.ndarray:
    shape = [1] * ndim
    shape[axis] = h.shape[0]
    return h.reshape(shape)


def filt_dec(x: np.ndarray, hhat: np.ndarray, k: int, axis: int = -1) -> np.ndarray:
    """Circular convolution with the filter of Fourier values ``hhat``, then keep every 2^k-th sample."""
    X = np.fft.fft(x, axis=axis)
    return np.fft.ifft(fold(X * _bcast(hhat, x.ndim, axis), k, axis), axis=axis)


def filt_dec_adj(y: np.ndarray, hhat: np.ndarray, k: int, axis: int = -1) -> np.ndarray:
    """Adjoint of ``filt_dec`` for a real filter spectrum ``hhat`` (complex result).

    With y = IDFT_L'(fold_k(h . DFT_L x)) and L = 2^k L', the adjoint is
    IDFT_L(h . tile_k(DFT_L' y)) (the 1/L', 2^-k and L factors cancel).
    """
    Y = np.fft.fft(y, axis=axis)
    return np.fft.ifft(_bcast(hhat, y.ndim, axis) * tile(Y, k, axis), axis=axis)


def phase(z: np.ndarray) -> np.ndarray:
    """z / |z|, and 0 where z == 0 (subgradient of the modulus)."""
    a = np.abs(z)
    out = np.zeros_like(z)
    nz = a > 0
    out[nz] = z[nz] / a[nz]
    return out


class FilterCache:
    """Memoised Fourier filter values (the paper's per-level filter tables)."""

    def __init__(self, plan: OraclePlan):
        self.p = plan
        self._c = {}

    def psi1(self, n1):
        key = ("psi1", n1)
        if key not in self._c:
            b = self.p.psi1[n1]
            self._c[key] = fb.bandpass_hat(self.p.N_pad, b.xi, b.sigma, 0)
        return self._c[key]

    def psi2(self, n2, level):
        key = ("psi2", n2, level)
        if key not in self._c:
            b = self.p.psi2[n2]
            self._c[key] = fb.bandpass_hat(self.p.N_pad >> level, b.xi, b.sigma, level)
        return self._c[key]

    def phi_t(self, level):
        key = ("phiT", level)
        if key not in self._c:
            self._c[key] = fb.lowpass_hat(self.p.N_pad >> level, self.p.sigma_T, level)
        return self._c[key]

    def fr(self, g):
        key = ("fr", g)
        if key not in self._c:
            b = self.p.fr[g]
            if b.lowpass:
                self._c[key] = fb.lowpass_hat(self.p.N_fr, b.sigma, 0)
            else:
                self._c[key] = fb.bandpass_hat(self.p.N_fr, b.xi, b.sigma, 0)
        return self._c[key]

    def phi_f(self, level):
        key = ("phiF", level)
        if key not in self._c:
            self._c[key] = fb.lowpass_hat(self.p.N_fr >> level, self.p.sigma_F, level)
        return self._c[key]


def pad_signal(plan: OraclePlan, x: np.ndarray) -> np.ndarray:
    x = np.asarray(x, dtype=np.float64)
    if x.shape != (plan.N,):
        raise ValueError(f"signal must have shape ({plan.N},)")
    xp = np.zeros(plan.N_pad, dtype=np.float64)
    xp[plan.pad_left:plan.pad_left + plan.N] = x
    return xp


def _block_view(plan, blk, S):
    return S[blk.offset: blk.offset + blk.n_lambda * blk.n_frames].reshape(blk.n_lambda, blk.n_frames)


def _keep(plan, blk, full):
    """Unpad a (bins x padded times) array to the block's kept bins and times."""
    return full[:blk.n_lambda, blk.t_lo: blk.t_lo + blk.n_frames]


def _unkeep(plan, blk, block, n_bins, n_times=None):
    full = np.zeros((n_bins, plan.nf_pad if n_times is None else n_times), dtype=np.float64)
    full[:blk.n_lambda, blk.t_lo: blk.t_lo + blk.n_frames] = block
    return full


def _fr_pooled(plan, b) -> bool:
    """Whether the path of frequential filter b is averaged by phi_F (every band-pass
    path unless frequential averaging is off; phi_F itself is already a low-pass)."""
    return (not b.lowpass) and plan.average_local_fr


def zeroth_order(plan: OraclePlan, x: np.ndarray, fc: "FilterCache") -> np.ndarray:
    """The zeroth-order block: S0 = (x_pad * phi_T) at stride T when averaging is local,
    else U0 = x (Sec. 3.6 main algorithm)."""
    if not plan.average_local:
        return np.asarray(x, dtype=np.float64).copy()
    S0 = filt_dec(pad_signal(plan, x), fc.phi_t(0), plan.log2_T).real
    return S0[plan.f_lo: plan.f_lo + plan.n_frames]


# ----------------------------------------------------------------------------- stages

def first_layer(plan: OraclePlan, x: np.ndarray, fc: FilterCache):
    """Z1 (complex scalogram before modulus, subsampled by 2^k1), U1hat = DFT(|Z1|), S1."""
    Xh = np.fft.fft(pad_signal(plan, x))
    Z1, U1h = [], []
    S1 = np.zeros((plan.N1, plan.nf_pad), dtype=np.float64)
    for n1, b in enumerate(plan.psi1):
        z = np.fft.ifft(fold(Xh * fc.psi1(n1), b.k))
        uh = np.fft.fft(np.abs(z))
        Z1.append(z)
        U1h.append(uh)
        S1[n1] = np.fft.ifft(fold(uh * fc.phi_t(b.k), plan.log2_T - b.k)).real
    return Xh, Z1, U1h, S1


def second_layer_group(plan: OraclePlan, grp, U1h, fc: FilterCache) -> np.ndarray:
    """Width-first stack Y2 (K rows, zero-padded to N_fr) for one second-order filter n2."""
    L2 = plan.N_pad >> grp.j2
    Y = np.zeros((plan.N_fr, L2), dtype=np.complex128)
    for n1 in range(grp.K):
        k1 = plan.psi1[n1].k
        Y[n1] = np.fft.ifft(fold(U1h[n1] * fc.psi2(grp.n2, k1), grp.j2 - k1))
    return Y


def freq_filter(plan, Xh_fr, g, fc):
    """Frequential filter g applied along axis 0 of an already-transformed input."""
    b = plan.fr[g]
    return np.fft.ifft(fold(Xh_fr * fc.fr(g)[:, None], b.k, axis=0), axis=0)


def first_layer_cache(plan: OraclePlan, x: np.ndarray, fc: FilterCache = None) -> dict:
    """The intermediates ``backward`` needs (first layer and the transformed order-1 input)."""
    fc = fc or FilterCache(plan)
    Xh, Z1, U1h, S1 = first_layer(plan, x, fc)
    return dict(Xh=Xh, Z1=Z1, U1h=U1h, S1=S1, Ah=transformed_s1(plan, S1), fc=fc)


def order1_blocks(plan: OraclePlan, Ah: np.ndarray, fc: FilterCache, S: np.ndarray) -> None:
    """Order-1 joint paths (Sec. 3.5 on real input, Eq. 3 for phi_F) written into S.

    ``Ah`` is the DFT along log-frequency of S1 zero-padded to N_fr rows."""
    for blk in plan.blocks:
        if blk.order != 1:
            continue
        g, b = blk.n_fr, plan.fr[blk.n_fr]
        V = freq_filter(plan, Ah, g, fc)
        if b.lowpass:
            out = V.real
        elif _fr_pooled(plan, b):
            out = filt_dec(np.abs(V), fc.phi_f(b.k), plan.s_F - b.k, axis=0).real
        else:
            out = np.abs(V)
        _block_view(plan, blk, S)[:] = _keep(plan, blk, out)


def order2_group(plan: OraclePlan, grp, U1h, fc: FilterCache, S: np.ndarray) -> None:
    """Every order-2 joint path of the second-order filter ``grp.n2`` written into S:
    the width-first stack Y2 (Sec. 3.3), the frequential filters along log-frequency
    (Sec. 3.5), the modulus, then phi_T over time and (band-pass paths) phi_F (Eq. 4)."""
    Y = second_layer_group(plan, grp, U1h, fc)
    Yh = np.fft.fft(Y, axis=0)
    phT = fc.phi_t(grp.j2)
    for blk in plan.blocks:
        if blk.order != 2 or blk.n2 != grp.n2:
            continue
        g, b = blk.n_fr, plan.fr[blk.n_fr]
        W = np.abs(freq_filter(plan, Yh, g, fc))
        P = filt_dec(W, phT, plan.log2_T - grp.j2, axis=1).real if plan.average_local else W
        if _fr_pooled(plan, b):
            out = filt_dec(P, fc.phi_f(b.k), plan.s_F - b.k, axis=0).real
        else:
            out = P
        _block_view(plan, blk, S)[:] = _keep(plan, blk, out)


def transformed_s1(plan: OraclePlan, S1: np.ndarray) -> np.ndarray:
    """DFT along log-frequency of S1 with its rows zero-padded to N_fr (Sec. 3.5)."""
    A = np.zeros((plan.N_fr, plan.nf_pad), dtype=np.float64)
    A[:plan.N1] = S1
    return np.fft.fft(A, axis=0)


def forward(plan: OraclePlan, x: np.ndarray, fc: FilterCache = None, return_cache: bool = False):
    """S(x) as a flat FP64 vector in the plan's output layout."""
    fc = fc or FilterCache(plan)
    Xh, Z1, U1h, S1 = first_layer(plan, x, fc)
    S = np.zeros(plan.n_coeff, dtype=np.float64)
    for blk in plan.blocks:
        if blk.order == 0:
            _block_view(plan, blk, S)[:] = zeroth_order(plan, x, fc)
    Ah = transformed_s1(plan, S1)
    order1_blocks(plan, Ah, fc, S)
    for grp in plan.groups:
        order2_group(plan, grp, U1h, fc, S)
    if return_cache:
        return S, dict(Xh=Xh, Z1=Z1, U1h=U1h, S1=S1, Ah=Ah, fc=fc)
    return S


def order2_group_adjoint(plan: OraclePlan, grp, U1h, fc: FilterCache, dS: np.ndarray, dU1) -> None:
    """Adds to the rows dU1[n1] (n1 < K) the adjoint of ``order2_group`` applied to the
    order-2 blocks of dS for the second-order filter ``grp.n2``: back through the phi_F and
    phi_T pooling, the modulus (subgradient 0 at 0), the frequential filters and the
    second layer."""
    blocks = [blk for blk in plan.blocks if blk.order == 2 and blk.n2 == grp.n2]
    if not any(np.any(_block_view(plan, blk, dS)) for blk in blocks):
        return    # every path of this group has zero gradient: it contributes nothing
    Y = second_layer_group(plan, grp, U1h, fc)
    Yh = np.fft.fft(Y, axis=0)
    phT = fc.phi_t(grp.j2)
    L2 = plan.N_pad >> grp.j2
    dY = np.zeros_like(Y)
    for blk in blocks:
        g, b = blk.n_fr, plan.fr[blk.n_fr]
        n_rows = plan.N_fr >> (plan.s_F if _fr_pooled(plan, b) or b.lowpass else b.k)
        dout = _unkeep(plan, blk, _block_view(plan, blk, dS), n_rows, None if plan.average_local else L2)
        if not np.any(dout):
            continue
        if _fr_pooled(plan, b):
            dP = filt_dec_adj(dout, fc.phi_f(b.k), plan.s_F - b.k, axis=0).real
        else:
            dP = dout
        dW = filt_dec_adj(dP, phT, plan.log2_T - grp.j2, axis=1).real if plan.average_local else dP
        V = freq_filter(plan, Yh, g, fc)
        dY += filt_dec_adj(dW * phase(V), fc.fr(g), b.k, axis=0)
    for n1 in range(grp.K):
        k1 = plan.psi1[n1].k
        dU1[n1] += filt_dec_adj(dY[n1], fc.psi2(grp.n2, k1), grp.j2 - k1).real


def backward(plan: OraclePlan, x: np.ndarray, dS: np.ndarray, cache=None, fc: FilterCache = None) -> np.ndarray:
    """dx = J_S(x)^T dS, the exact adjoint of ``forward``."""
    dS = np.asarray(dS, dtype=np.float64)
    if cache is None:
        cache = first_layer_cache(plan, x, fc)
    fc = cache["fc"]
    Z1, U1h, Ah = cache["Z1"], cache["U1h"], cache["Ah"]
    dU1 = [np.zeros(z.shape[0], dtype=np.float64) for z in Z1]

    # order 1: back through phi_F pooling, modulus, frequential filters, onto S1
    dA = np.zeros((plan.N_fr, plan.nf_pad), dtype=np.float64)
    for blk in plan.blocks:
        if blk.order != 1:
            continue
        g, b = blk.n_fr, plan.fr[blk.n_fr]
        n_rows = plan.N_fr >> (plan.s_F if _fr_pooled(plan, b) or b.lowpass else b.k)
        dout = _unkeep(plan, blk, _block_view(plan, blk, dS), n_rows)
        if b.lowpass:
            dV = dout.astype(np.complex128)
        else:
            V = freq_filter(plan, Ah, g, fc)
            dW = filt_dec_adj(dout, fc.phi_f(b.k), plan.s_F - b.k, axis=0).real if _fr_pooled(plan, b) else dout
            dV = dW * phase(V)
        dA += filt_dec_adj(dV, fc.fr(g), b.k, axis=0).real
    for n1, b in enumerate(plan.psi1):
        dU1[n1] += filt_dec_adj(dA[n1], fc.phi_t(b.k), plan.log2_T - b.k).real

    # order 2: per n2 group, back through pooling, modulus, frequential filters, second layer
    for grp in plan.groups:
        order2_group_adjoint(plan, grp, U1h, fc, dS, dU1)

    # first layer: modulus, then the first-order filters, onto the padded signal
    dxp = np.zeros(plan.N_pad, dtype=np.float64)
    for n1, b in enumerate(plan.psi1):
        dZ = dU1[n1] * phase(Z1[n1])
        dxp += filt_dec_adj(dZ, fc.psi1(n1), b.k).real
    # zeroth order: the adjoint of phi_T at stride T (S0), or the identity (U0)
    for blk in plan.blocks:
        if blk.order != 0:
            continue
        d0 = _block_view(plan, blk, dS)[0]
        if plan.average_local:
            full = np.zeros(plan.nf_pad)
            full[blk.t_lo: blk.t_lo + blk.n_frames] = d0
            dxp += filt_dec_adj(full, fc.phi_t(0), plan.log2_T).real
        else:
            dxp[plan.pad_left: plan.pad_left + plan.N] += d0
    return dxp[plan.pad_left: plan.pad_left + plan.N].copy()


# ----------------------------------------------------------------------------- partial forward

def forward_partial(plan: OraclePlan, x: np.ndarray, n2_list, order1: bool = True, fc: FilterCache = None):
    """The order-1 blocks (if ``order1``) and the order-2 blocks of the listed n2, computed
    by the same per-block steps as ``forward``; every other coefficient is NaN. Used for
    sampled parity at full size."""
    fc = fc or FilterCache(plan)
    _, _, U1h, S1 = first_layer(plan, x, fc)
    S = np.full(plan.n_coeff, np.nan)
    if order1:
        for blk in plan.blocks:
            if blk.order == 0:
                _block_view(plan, blk, S)[:] = zeroth_order(plan, x, fc)
        order1_blocks(plan, transformed_s1(plan, S1), fc, S)
    want = set(n2_list)
    for grp in plan.groups:
        if grp.n2 in want:
            order2_group(plan, grp, U1h, fc, S)
    return S


def first_order_only(plan: OraclePlan, x: np.ndarray, fc: FilterCache = None):
    """The order-1 block and the intermediate first-layer arrays (Z1 rows, S1)."""
    fc = fc or FilterCache(plan)
    Xh, Z1, U1h, S1 = first_layer(plan, x, fc)
    return Z1, U1h, S1
