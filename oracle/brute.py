"""O1: JTFS by direct circular convolutions (oracle, FP64, tiny sizes only).

Every filter is built in the time domain from the continuous Morlet / Gaussian
(``filterbank.bandpass_time`` / ``lowpass_time``), every convolution is the plain sum
y[t] = sum_n x[n] h[(t 2^k - n) mod L] kept at every 2^k-th output sample, and the
modulus and averaging follow Eqs. 2-4 directly. No FFT is used anywhere, so agreement
with the Fourier route (O2) checks its Fourier subsampling, level filters and adjoint
bookkeeping against the plain definition.
"""
from __future__ import annotations

import numpy as np

from . import filterbank as fb
from .plan import OraclePlan


def conv_matrix(h: np.ndarray, k: int) -> np.ndarray:
    """Matrix C with (C x)[t] = sum_n x[n] h[(t 2^k - n) mod L], t < L / 2^k."""
    L = h.shape[0]
    t = np.arange(L >> k)[:, None] << k
    n = np.arange(L)[None, :]
    return h[(t - n) % L]


def _fr_time(plan, g):
    b = plan.fr[g]
    if b.lowpass:
        return fb.lowpass_time(plan.N_fr, b.sigma, 0)
    return fb.bandpass_time(plan.N_fr, b.xi, b.sigma, 0)


def forward(plan: OraclePlan, x: np.ndarray, return_intermediates: bool = False):
    x = np.asarray(x, dtype=np.float64)
    xp = np.zeros(plan.N_pad)
    xp[plan.pad_left: plan.pad_left + plan.N] = x
    Z1, U1 = [], []
    S1 = np.zeros((plan.N1, plan.nf_pad))
    for b in plan.psi1:
        z = conv_matrix(fb.bandpass_time(plan.N_pad, b.xi, b.sigma, 0), b.k) @ xp
        u = np.abs(z)
        L1 = plan.N_pad >> b.k
        S1_row = conv_matrix(fb.lowpass_time(L1, plan.sigma_T, b.k), plan.log2_T - b.k) @ u
        Z1.append(z)
        U1.append(u)
        S1[len(U1) - 1] = S1_row.real
    S = np.zeros(plan.n_coeff)

    def put(blk, full):
        blockv = S[blk.offset: blk.offset + blk.n_lambda * blk.n_frames].reshape(blk.n_lambda, blk.n_frames)
        blockv[:] = full[:blk.n_lambda, blk.t_lo: blk.t_lo + blk.n_frames]

    def fr_pooled(b):
        return (not b.lowpass) and plan.average_local_fr

    for blk in plan.blocks:
        if blk.order == 0:
            if plan.average_local:
                S0 = conv_matrix(fb.lowpass_time(plan.N_pad, plan.sigma_T, 0), plan.log2_T) @ xp
                put(blk, S0[None, :])
            else:
                put(blk, xp[None, :])   # U0: the kept samples of the padded signal

    A = np.zeros((plan.N_fr, plan.nf_pad))
    A[:plan.N1] = S1
    for blk in plan.blocks:
        if blk.order != 1:
            continue
        b = plan.fr[blk.n_fr]
        V = conv_matrix(_fr_time(plan, blk.n_fr), b.k) @ A
        if b.lowpass:
            out = V.real
        elif fr_pooled(b):
            Mg = plan.N_fr >> b.k
            out = (conv_matrix(fb.lowpass_time(Mg, plan.sigma_F, b.k), plan.s_F - b.k) @ np.abs(V)).real
        else:
            out = np.abs(V)
        put(blk, out)

    for grp in plan.groups:
        L2 = plan.N_pad >> grp.j2
        b2 = plan.psi2[grp.n2]
        Y = np.zeros((plan.N_fr, L2), dtype=np.complex128)
        for n1 in range(grp.K):
            k1 = plan.psi1[n1].k
            L1 = plan.N_pad >> k1
            h2 = fb.bandpass_time(L1, b2.xi, b2.sigma, k1)
            Y[n1] = conv_matrix(h2, grp.j2 - k1) @ U1[n1]
        Ct = conv_matrix(fb.lowpass_time(L2, plan.sigma_T, grp.j2), plan.log2_T - grp.j2)
        for blk in plan.blocks:
            if blk.order != 2 or blk.n2 != grp.n2:
                continue
            b = plan.fr[blk.n_fr]
            W = np.abs(conv_matrix(_fr_time(plan, blk.n_fr), b.k) @ Y)
            P = (W @ Ct.T).real if plan.average_local else W
            if fr_pooled(b):
                Mg = plan.N_fr >> b.k
                out = (conv_matrix(fb.lowpass_time(Mg, plan.sigma_F, b.k), plan.s_F - b.k) @ P).real
            else:
                out = P
            put(blk, out)
    if return_intermediates:
        return S, dict(Z1=Z1, U1=U1, S1=S1)
    return S
