"""Oracle plan: filterbanks, subsampling factors, path list and output layout.

Derived from the paper (Sec. 3.1-3.5) independently of the C++ plan of the HIP path.
Readings where the paper is silent, each with its reason:

* phi_T is a Gaussian of width sigma0 / T, phi_F of width sigma0 / F (F in first-order
  filter bins); both have unit DC gain. Their subsampling scales are log2 T and
  floor(log2 F). (Sec. 2.1-2.2 give only "width 1/T", "bandwidth 1/F".) Parity unpinned.
* j of a band-pass comes from its band edge |xi| + 5 sigma (see filterbank). Parity unpinned.
* First layer: k1 = min(j1, log2 T) (Sec. 3.2). Second layer: pairs with j2 > j1 and
  k2 = min(j2 - k1, log2 T) (Sec. 3.3); every admitted pair must land at a resolution
  no coarser than T, otherwise the configuration is rejected.
* Time padding: zeros to N_pad = 2^(ceil(log2 N) + 1), left pad floor((N_pad - N) / 2)
  (Sec. 3.2 says both sides, not how much). ``periodic`` skips padding (N a power of two).
* Frequential padding: the first-order axis is zero-padded on the right to
  N_fr = 2 * 2^ceil(log2 N1) (Sec. 3.5, ``phi['N']``). Parity unpinned.
* Frequential filter list: [phi_F] + band-passes with xi > 0 + band-passes with xi < 0
  (Sec. 3.4-3.5). Real (alpha = 0) inputs use the first two groups only.
* k_fr = min(j_fr, floor(log2 F)) (Sec. 3.5).
* Each axis is low-passed exactly once: alpha = 0 paths get no second phi_T, and
  beta = 0 (phi_F) paths get no second phi_F.
* Output: order-1 block, then order-2 blocks for ascending n2; inside a block the
  frequential filter (list order), then the log-frequency bin, then the frame. Only
  unpadded frames (pad_left <= f T < pad_left + N) and unpadded bins (b 2^sF < n1_max)
  are kept. Zeroth order is not part of the output (it does not enter Eqs. 5-7) unless
  ``zeroth`` asks for it; then its block comes first (the main algorithm of Sec. 3.6
  yields it before order 1).
* Variants of the Sec. 3.3 / 3.5 listings and the Sec. 3.6 main algorithm:
  - ``zeroth``: the zeroth-order block: S0 = (x * phi_T) at stride T (kept frames) when
    averaging is local, else U0 = x itself (the listing's "U_0 indexed by time");
  - ``average_local = False``: no phi_T averaging of the second order: each joint path
    keeps |Y_2_fr| at its own time resolution 2^j2 (the listing's "time[n2]"), unpadded to
    the times t with pad_left <= t 2^j2 < pad_left + N. With the second-order rule
    k1 + k2 = j2 <= log2 T of this plan, the listing's subsampling exponents coincide
    with the averaged ones. The first order stays averaged (S1 = U1 * phi_T, "time[log2_T]");
  - ``average_local_fr = False``: k_fr = j_fr instead of min(j_fr, floor(log2 F)), and no
    phi_F averaging of band-pass paths: each keeps |Y_fr| at log-frequency resolution
    2^k_fr, unpadded to the bins b with b 2^k_fr < n1_max.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List

from . import filterbank as fb


def ceil_log2(n: int) -> int:
    p = 0
    while (1 << p) < n:
        p += 1
    return p


@dataclass
class Band:
    xi: float
    sigma: float
    j: int
    k: int = 0            # subsampling actually applied (k1, or k_fr)
    spin: int = 0         # frequential filters: +1, -1, or 0 for phi_F
    lowpass: bool = False


@dataclass
class Group:
    n2: int
    j2: int
    K: int                # n1_max: number of first-order rows with j1 < j2


@dataclass
class PathBlock:
    order: int            # 0, 1 or 2
    n2: int               # -1 for orders 0 and 1
    n_fr: int             # index in the frequential filter list (-1 for order 0)
    spin: int
    j2: int               # -1 for orders 0 and 1
    j_fr: int
    n_lambda: int
    n_frames: int
    offset: int
    t_lo: int = 0         # first kept sample on the block's time grid


@dataclass
class OraclePlan:
    N: int
    J: int
    Q1: int
    Q2: int
    J_fr: int
    Q_fr: int
    log2_T: int
    F: float
    periodic: bool
    N_pad: int = 0
    pad_left: int = 0
    T: int = 0
    s_F: int = 0
    N_fr: int = 0
    sigma_T: float = 0.0
    sigma_F: float = 0.0
    psi1: List[Band] = field(default_factory=list)
    psi2: List[Band] = field(default_factory=list)
    fr: List[Band] = field(default_factory=list)
    groups: List[Group] = field(default_factory=list)
    nf_pad: int = 0       # frames on the padded axis, N_pad / T
    f_lo: int = 0
    n_frames: int = 0
    blocks: List[PathBlock] = field(default_factory=list)
    n_coeff: int = 0
    zeroth: bool = False
    average_local: bool = True
    average_local_fr: bool = True

    @property
    def N1(self) -> int:
        return len(self.psi1)

    def fr_real(self):
        """Indices of the frequential filters applied to real (alpha = 0) inputs."""
        return [g for g, b in enumerate(self.fr) if b.spin >= 0]


def make_plan(N: int, J: int, Q1: int, Q2: int, J_fr: int, Q_fr: int, log2_T: int, F: float,
              periodic: bool = False, zeroth: bool = False, average_local: bool = True,
              average_local_fr: bool = True) -> OraclePlan:
    if N < 2:
        raise ValueError("N must be >= 2")
    p = OraclePlan(N, J, Q1, Q2, J_fr, Q_fr, log2_T, float(F), bool(periodic))
    p.zeroth, p.average_local, p.average_local_fr = bool(zeroth), bool(average_local), bool(average_local_fr)
    if periodic:
        if N & (N - 1):
            raise ValueError("periodic mode needs N a power of two")
        p.N_pad, p.pad_left = N, 0
    else:
        p.N_pad = 1 << (ceil_log2(N) + 1)
        p.pad_left = (p.N_pad - N) // 2
    p.T = 1 << log2_T
    if p.T > p.N_pad:
        raise ValueError("T exceeds the padded length")
    if F < 1.0:
        raise ValueError("F must be >= 1 bin")
    p.s_F = int(math.floor(math.log2(F)))
    while (1 << (p.s_F + 1)) <= F:      # guard the float log against rounding
        p.s_F += 1
    while (1 << p.s_F) > F:
        p.s_F -= 1
    p.sigma_T = fb.SIGMA0 / p.T
    p.sigma_F = fb.SIGMA0 / F

    for xi, s in fb.morlet_bank(J, Q1):
        j = fb.subsampling_scale(xi, s)
        p.psi1.append(Band(xi, s, j, min(j, log2_T)))
    for xi, s in fb.morlet_bank(J, Q2):
        p.psi2.append(Band(xi, s, fb.subsampling_scale(xi, s)))

    p.N_fr = 2 * (1 << ceil_log2(max(p.N1, 1)))
    if (1 << p.s_F) > p.N_fr:
        raise ValueError("F exceeds the padded frequential axis")
    p.fr.append(Band(0.0, p.sigma_F, p.s_F, p.s_F, spin=0, lowpass=True))
    bank_fr = fb.morlet_bank(J_fr, Q_fr)
    for sign in (+1, -1):
        for xi, s in bank_fr:
            j = fb.subsampling_scale(xi, s)
            p.fr.append(Band(sign * xi, s, j, min(j, p.s_F) if p.average_local_fr else j, spin=sign))

    for n2, b2 in enumerate(p.psi2):
        K = 0
        for b1 in p.psi1:
            if b2.j > b1.j:
                K += 1
        # rows with j1 < j2 form a prefix because j1 never decreases along the bank
        assert all((b2.j > p.psi1[i].j) == (i < K) for i in range(p.N1))
        if K == 0:
            continue
        for b1 in p.psi1[:K]:
            k2 = min(b2.j - b1.k, log2_T)
            if b1.k + k2 > log2_T:
                raise ValueError("second-order resolution coarser than T is not supported")
            assert b1.k + k2 == b2.j
        p.groups.append(Group(n2, b2.j, K))

    p.nf_pad = p.N_pad // p.T
    if periodic:
        p.f_lo, f_hi = 0, p.nf_pad
    else:
        p.f_lo = -(-p.pad_left // p.T)
        f_hi = -(-(p.pad_left + N) // p.T)
    p.n_frames = f_hi - p.f_lo

    def bins(K, k):
        return -(-K // (1 << k))

    def kept_times(j):
        """First kept sample and count on a grid of stride 2^j (unpadded samples)."""
        if periodic:
            return 0, p.N_pad >> j
        lo = -(-p.pad_left // (1 << j))
        return lo, -(-(p.pad_left + N) // (1 << j)) - lo

    def lam(K, b):
        """Kept log-frequency bins of a path: phi_F-averaged (stride 2^sF) or, for a
        band-pass without frequential averaging, its own stride 2^k_fr."""
        return bins(K, b.k if (not b.lowpass and not p.average_local_fr) else p.s_F)

    off = 0
    if p.zeroth:
        if p.average_local:
            blk = PathBlock(0, -1, -1, 0, -1, -1, 1, p.n_frames, off, p.f_lo)
        else:
            blk = PathBlock(0, -1, -1, 0, -1, -1, 1, N, off, p.pad_left)
        p.blocks.append(blk)
        off += blk.n_lambda * blk.n_frames
    for g in p.fr_real():
        b = p.fr[g]
        blk = PathBlock(1, -1, g, b.spin, -1, b.j, lam(p.N1, b), p.n_frames, off, p.f_lo)
        p.blocks.append(blk)
        off += blk.n_lambda * blk.n_frames
    for grp in p.groups:
        t_lo, n_t = (p.f_lo, p.n_frames) if p.average_local else kept_times(grp.j2)
        for g, b in enumerate(p.fr):
            blk = PathBlock(2, grp.n2, g, b.spin, grp.j2, b.j, lam(grp.K, b), n_t, off, t_lo)
            p.blocks.append(blk)
            off += blk.n_lambda * blk.n_frames
    p.n_coeff = off
    return p
