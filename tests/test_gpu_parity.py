"""GPU parity of the HIP path against the FP64 oracle (run on an MI355X).

Tolerances (FP32 path vs FP64 oracle): relative L2 error <= 1e-5 on S(x) and on the
first-layer / second-layer intermediates, <= 1e-4 on the gradient dx.
"""
import math
import sys

import numpy as np
import pytest
import torch

import jtfs_inputs as ji
from oracle import descent, fftroute
from oracle.plan import make_plan

pytestmark = pytest.mark.gpu

J = pytest.importorskip("paper_2602_11896_amd.jtfs")

TOL_S = 1e-5
TOL_GRAD = 1e-4

TINY = (512, 4, 4, 1, 2, 1, 5, 2)
TINY_B = (384, 4, 3, 2, 2, 2, 4, 3)
CFG1 = (8192, 6, 8, 1, 3, 1, 9, 4)
CFG2 = (65536, 12, 12, 2, 4, 2, 13, 24)


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel(a, b):
    """Relative L2 error of a against b (complex arrays compared in both parts)."""
    a = np.asarray(a)
    b = np.asarray(b)
    dt = np.complex128 if (np.iscomplexobj(a) or np.iscomplexobj(b)) else np.float64
    a, b = a.astype(dt), b.astype(dt)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def assert_blocks(op, Sg, S_ref, what, tol=10 * TOL_S):
    """Relative L2 of every output block (order-1 blocks, each (n2, frequential filter)
    block) within tol, the whole vector within TOL_S; NaN entries of S_ref (blocks a
    partial oracle did not fill) are skipped."""
    worst = 0.0
    for blk in op.blocks:
        sl = slice(blk.offset, blk.offset + blk.n_lambda * blk.n_frames)
        if np.isnan(S_ref[sl]).any():
            continue
        e = rel(Sg[sl], S_ref[sl])
        worst = max(worst, e)
        assert e <= tol, f"{what}: block order={blk.order} n2={blk.n2} n_fr={blk.n_fr}: {e:.3e}"
    mask = ~np.isnan(S_ref)
    err = rel(Sg[mask], S_ref[mask])
    say(f"[parity] {what}: rel L2 {err:.3e} (worst block {worst:.3e})")
    assert err <= TOL_S
    return err


def dev(x):
    return torch.as_tensor(np.asarray(x, dtype=np.float32), device="cuda").contiguous()


def host(t):
    torch.cuda.synchronize()
    a = t.detach().cpu().numpy()
    return a.astype(np.complex128 if np.iscomplexobj(a) else np.float64)


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def run_forward(args, x, periodic=False):
    plan = J.Plan(J.Params(*args, periodic=periodic))
    ws = plan.workspace()
    S = plan.forward(dev(x), ws=ws)
    return plan, ws, S


@pytest.mark.parametrize("name,args,periodic", [("tiny", TINY, False), ("tiny_b", TINY_B, False),
                                                ("periodic", (1024, 4, 4, 2, 2, 2, 5, 2), True),
                                                ("cfg1", CFG1, False)])
def test_forward_and_intermediates(name, args, periodic):
    say(f"[parity] forward {name} {args}")
    op = make_plan(*args, periodic=periodic)
    x = ji.config1_signal(0, n=op.N) if not periodic else np.random.default_rng(9).standard_normal(op.N)
    plan, ws, S = run_forward(args, x, periodic)
    S_ref, cache = fftroute.forward(op, x, return_cache=True)
    Z1 = host(plan.ws_region(ws, 0, 0))
    U1h = host(plan.ws_region(ws, 0, 1))
    S1 = host(plan.ws_region(ws, 0, 2, torch.float32)).reshape(op.N1, op.nf_pad)
    Y2 = host(plan.ws_region(ws, 0, 3))
    off = 0
    for n1 in range(op.N1):
        L = cache["Z1"][n1].shape[0]
        assert rel(Z1[off:off + L], cache["Z1"][n1]) <= TOL_S, f"Z1 row {n1}"
        assert rel(U1h[off:off + L], cache["U1h"][n1]) <= TOL_S, f"U1hat row {n1}"
        off += L
    assert rel(S1, cache["S1"]) <= TOL_S
    off = 0
    for grp in op.groups:
        Yr = fftroute.second_layer_group(op, grp, cache["U1h"], cache["fc"])[:grp.K]
        n = Yr.size
        assert rel(Y2[off:off + n].reshape(Yr.shape), Yr) <= TOL_S, f"Y2 group n2={grp.n2}"
        off += n
    Sg = host(S)
    for blk in op.blocks:
        a = Sg[blk.offset: blk.offset + blk.n_lambda * blk.n_frames]
        b = S_ref[blk.offset: blk.offset + blk.n_lambda * blk.n_frames]
        assert rel(a, b) <= 10 * TOL_S, f"block order={blk.order} n2={blk.n2} n_fr={blk.n_fr}: {rel(a, b)}"
    err = rel(Sg, S_ref)
    say(f"[parity] forward {name}: rel L2 {err:.3e}")
    assert err <= TOL_S


@pytest.mark.parametrize("name,args", [("tiny", TINY), ("tiny_b", TINY_B), ("cfg1", CFG1)])
def test_backward(name, args):
    say(f"[parity] backward {name} {args}")
    op = make_plan(*args)
    x = ji.config1_signal(0, n=op.N)
    y = ji.white_noise_like(x, 1)
    S_x = fftroute.forward(op, x)
    S_y, cache = fftroute.forward(op, y, return_cache=True)
    dS = 2.0 * (S_y - S_x)
    g_ref = fftroute.backward(op, y, dS, cache=cache)
    plan = J.Plan(J.Params(*args))
    ws = plan.workspace()
    dx = plan.backward(dev(y), dev(dS), ws=ws)
    err = rel(host(dx), g_ref)
    say(f"[parity] backward {name}: rel L2 {err:.3e}")
    assert err <= TOL_GRAD
    # reuse of the forward intermediates gives the same gradient bit for bit
    yd = dev(y)
    plan.forward(yd, ws=ws)
    dx2 = plan.backward(yd, dev(dS), ws=ws, reuse_forward=True)
    assert torch.equal(dx, dx2)


def test_config2_full_forward_and_backward():
    # Full config-2 size: every output block of S(x) and S(y) element-wise against the
    # oracle, and the whole gradient of E(y) = ||S(y) - S(x)||^2 (dS = 2 (S(y) - S(x))).
    say("[parity] config 2 full: oracle forward of x")
    op = make_plan(*CFG2)
    x = ji.config2_signal(2)
    y = ji.white_noise_like(x, 3)
    S_x = fftroute.forward(op, x)
    say("[parity] config 2 full: oracle forward of y")
    S_y, cache = fftroute.forward(op, y, return_cache=True)
    dS = 2.0 * (S_y - S_x)
    say("[parity] config 2 full: oracle backward")
    g_ref = fftroute.backward(op, y, dS, cache=cache)
    plan = J.Plan(J.Params(*CFG2))
    ws = plan.workspace()
    assert_blocks(op, host(plan.forward(dev(x), ws=ws)), S_x, "config 2 forward S(x)")
    yd = dev(y)
    assert_blocks(op, host(plan.forward(yd, ws=ws)), S_y, "config 2 forward S(y)")
    dx = plan.backward(yd, dev(dS), ws=ws, reuse_forward=True)
    err = rel(host(dx), g_ref)
    say(f"[parity] config 2 backward (full gradient): rel L2 {err:.3e}")
    assert err <= TOL_GRAD


def test_config2_finite_differences_64_indices():
    # BASELINE config 2's check of the hand-written adjoint: central differences of
    # E(y) = ||S(y) - S(x)||^2 at 64 random sample indices (seed 4) against the device
    # gradient. S is the device's FP32 transform, E is summed on the host in FP64. The FP32
    # rounding of S (about 1e-7 relative, independent between y + h e_i and y - h e_i)
    # leaves a noise of about 3e-8 in each difference of E = 2e-2 against 2 h |g_i| of
    # about 6e-7 at h = 0.1 rms(y) (measured: 6e-3 relative L2 at h = 0.05 rms(y)). So this
    # is a check of the adjoint's structure at full size (a wrong sign or a missing term
    # is an O(1) error), to 1e-2 relative L2; the FP64 oracle's gradient is held to
    # central differences at this size to 1e-6, and this gradient to the oracle's to 1e-4.
    say("[parity] config 2 finite differences")
    x = ji.config2_signal(2)
    y = ji.white_noise_like(x, 3)
    plan = J.Plan(J.Params(*CFG2))
    ws = plan.workspace()
    S_x = host(plan.forward(dev(x), ws=ws))

    def E(v):
        d = host(plan.forward(v, ws=ws)) - S_x
        return float(np.dot(d, d)), d

    yd = dev(y)
    E0, d0 = E(yd)
    g = host(plan.backward(yd, dev(2.0 * d0), ws=ws, reuse_forward=True))
    idx = np.random.default_rng(4).choice(len(y), 64, replace=False)
    h = 0.1 * float(np.sqrt(np.mean(y * y)))
    fd = []
    for i in idx:
        vp = yd.clone()
        vp[int(i)] += h
        vm = yd.clone()
        vm[int(i)] -= h
        fd.append((E(vp)[0] - E(vm)[0]) / (2 * h))
    fd = np.asarray(fd)
    gs = g[idx]
    scale = np.max(np.abs(gs))
    err = np.abs(fd - gs)
    e_rel = np.linalg.norm(fd - gs) / np.linalg.norm(gs)
    say(f"[parity] config 2 FD: E={E0:.4e}, max |g| {scale:.3e}, max |fd - g| {err.max():.3e}, rel L2 {e_rel:.3e}")
    assert e_rel <= 1e-2
    assert np.all(err <= 2e-2 * scale)


def test_forward_is_deterministic():
    say("[parity] determinism cfg1")
    x = dev(ji.config1_signal(0))
    plan = J.Plan(J.Params(*CFG1))
    ws = plan.workspace()
    a = plan.forward(x, ws=ws).clone()
    b = plan.forward(x, ws=ws).clone()
    dS = torch.ones_like(a)
    g1 = plan.backward(x, dS, ws=ws).clone()
    g2 = plan.backward(x, dS, ws=ws).clone()
    assert torch.equal(a, b) and torch.equal(g1, g2)


def test_homogeneity_and_zero_input():
    say("[parity] homogeneity cfg1")
    x = ji.config1_signal(0)
    plan = J.Plan(J.Params(*CFG1))
    ws = plan.workspace()
    S = host(plan.forward(dev(x), ws=ws))
    S3 = host(plan.forward(dev(-3.0 * x), ws=ws))
    assert rel(S3, 3.0 * S) <= 1e-6
    S0 = host(plan.forward(dev(np.zeros_like(x)), ws=ws))
    assert np.all(S0 == 0.0)
    g0 = host(plan.backward(dev(np.zeros_like(x)), dev(np.ones(plan.n_coeff)), ws=ws))
    assert np.all(g0 == 0.0)


def test_euler_identity_config2():
    # <y, J^T dS> = <S(y), dS> for the degree-1 homogeneous transform, at full size.
    say("[parity] Euler identity cfg2")
    y = ji.config2_signal(3)
    plan = J.Plan(J.Params(*CFG2))
    ws = plan.workspace()
    yd = dev(y)
    S = host(plan.forward(yd, ws=ws))
    dS = np.random.default_rng(1).standard_normal(plan.n_coeff)
    g = host(plan.backward(yd, dev(dS), ws=ws, reuse_forward=True))
    lhs, rhs = float(np.dot(y, g)), float(np.dot(S, dS))
    say(f"[parity] Euler cfg2: {lhs:.8e} vs {rhs:.8e}")
    assert abs(lhs - rhs) <= 1e-5 * abs(rhs) + 1e-6 * np.linalg.norm(y) * np.linalg.norm(g)


def test_metamer_gd_trajectory_config1():
    # Config 1: 20 gradient-descent steps (step 0.1) from white noise, per-step losses.
    say("[parity] metamer GD trajectory cfg1")
    op = make_plan(*CFG1)
    x = ji.config1_signal(0)
    y0 = ji.white_noise_like(x, 1)
    S_x = fftroute.forward(op, x)
    _, losses_ref = descent.metamer(op, S_x, y0, descent.OptState("gd", lr=0.1), 20)
    plan = J.Plan(J.Params(*CFG1))
    ws = plan.workspace()
    opt = J.Optimizer(plan, "gd", lr=0.1)
    y = dev(y0)
    St = dev(S_x)
    loss = torch.zeros(1, device="cuda")
    got = []
    for _ in range(20):
        plan.metamer_step(y, St, opt, loss, ws)
        got.append(float(host(loss)[0]))
    err = max(abs(a - b) / abs(b) for a, b in zip(got, losses_ref))
    say(f"[parity] GD losses max rel err {err:.3e} (first {got[0]:.6e}, last {got[-1]:.6e})")
    assert err <= 1e-3


@pytest.mark.parametrize("kind", ["adam", "momentum"])
def test_metamer_optimisers_tiny(kind):
    say(f"[parity] metamer {kind} tiny")
    op = make_plan(*TINY)
    x = ji.config1_signal(0, n=op.N)
    y0 = ji.white_noise_like(x, 1)
    S_x = fftroute.forward(op, x)
    st = descent.OptState(kind, lr=0.1 if kind == "adam" else 2000.0)
    y_ref, losses_ref = descent.metamer(op, S_x, y0, st, 8)
    plan = J.Plan(J.Params(*TINY))
    ws = plan.workspace()
    opt = J.Optimizer(plan, kind, lr=0.1 if kind == "adam" else 2000.0)
    y = dev(y0)
    St = dev(S_x)
    loss = torch.zeros(1, device="cuda")
    got = []
    for _ in range(8):
        plan.metamer_step(y, St, opt, loss, ws)
        got.append(float(host(loss)[0]))
    err = max(abs(a - b) / abs(b) for a, b in zip(got, losses_ref))
    say(f"[parity] {kind} losses max rel err {err:.3e}; ref {losses_ref[0]:.4e} -> {losses_ref[-1]:.4e}")
    assert err <= 1e-3
    assert rel(host(y), y_ref) <= 1e-3


def test_nonfinite_loss_leaves_signal():
    say("[parity] non-finite step")
    plan = J.Plan(J.Params(*TINY))
    ws = plan.workspace()
    opt = J.Optimizer(plan, "momentum", lr=0.1)
    y = dev(np.random.default_rng(2).standard_normal(TINY[0]))
    y[7] = float("nan")
    before = y.clone()
    loss = torch.zeros(1, device="cuda")
    assert J.opt_status(plan, opt) == [0]
    plan.metamer_step(y, torch.zeros(plan.n_coeff, device="cuda"), opt, loss, ws)
    torch.cuda.synchronize()
    assert not math.isfinite(float(loss[0]))
    assert torch.equal(torch.isnan(y), torch.isnan(before))
    assert torch.equal(y[~torch.isnan(y)], before[~torch.isnan(before)])
    # the device flag reaches the host at synchronisation as JTFS_ERR_NONFINITE
    assert J.opt_status(plan, opt, raise_nonfinite=False) == [1]
    with pytest.raises(J.L.JTFSError) as err:
        J.opt_status(plan, opt)
    assert err.value.status == J.L.JTFS_ERR_NONFINITE


def test_batched_plan_matches_single():
    say("[parity] batch of two signals")
    a, b = TINY, TINY_B
    xa = ji.config1_signal(0, n=a[0])
    xb = ji.config1_signal(5, n=b[0])
    plan = J.Plan([J.Params(*a), J.Params(*b)])
    S = host(plan.forward(dev(np.concatenate([xa, xb])), ws=plan.workspace()))
    Sa = fftroute.forward(make_plan(*a), xa)
    Sb = fftroute.forward(make_plan(*b), xb)
    assert rel(S[: Sa.size], Sa) <= TOL_S
    assert rel(S[Sa.size:], Sb) <= TOL_S


@pytest.mark.parametrize("tuning", [(128, 16, 512, 1), (1024, 32, 128, -1),
                                    (256, 32, 256, 0, (16, 1024, 64, 512, 0), (1024, 16, 512, 64, 0))])
def test_tuned_plan_parity_cfg1(tuning):
    """Other tile schedules (row splits, time tiles, split points) compute the same transform."""
    say(f"[parity] tuned plan cfg1 {tuning}")
    op = make_plan(*CFG1)
    x = ji.config1_signal(0, n=op.N)
    y = ji.white_noise_like(x, 1)
    S_x = fftroute.forward(op, x)
    S_y, cache = fftroute.forward(op, y, return_cache=True)
    dS = 2.0 * (S_y - S_x)
    g_ref = fftroute.backward(op, y, dS, cache=cache)
    plan = J.Plan(J.Params(*CFG1), tuning=J.Tuning(*tuning))
    ws = plan.workspace()
    yd = dev(y)
    S = plan.forward(yd, ws=ws)
    err_s = rel(host(S), S_y)
    dx = plan.backward(yd, dev(dS), ws=ws, reuse_forward=True)
    err_g = rel(host(dx), g_ref)
    say(f"[parity] tuned {tuning}: S rel {err_s:.3e}, dx rel {err_g:.3e}")
    assert err_s <= TOL_S and err_g <= TOL_GRAD


def test_tuned_plan_config2_sampled():
    """A non-default tiling at full config-2 size against the oracle on sampled groups."""
    say("[parity] tuned plan config 2 sampled")
    op = make_plan(*CFG2)
    x = ji.config2_signal(2)
    # one group of each k-step bucket (K = 14, 26, 50, 98, 122: 4, 8, 16, 32 k-steps)
    n2s = sorted({next(g.n2 for g in op.groups if g.K >= k) for k in (14, 26, 50, 98, 122)})
    S_ref = fftroute.forward_partial(op, x, n2s)
    plan = J.Plan(J.Params(*CFG2), tuning=J.Tuning(512, 16, 1024, -1, (64, 1024, 128, 512, 0), (1024, 64, 512, 128, 0)))
    S = host(plan.forward(dev(x)))
    assert_blocks(op, S, S_ref, f"tuned config 2 groups {n2s}")


def test_autotune_returns_a_working_schedule():
    say("[autotune] cfg1")
    tuning, ms = J.autotune(J.Params(*CFG1))
    say(f"[autotune] {tuning} {ms:.3f} ms")
    assert ms > 0.0
    assert tuning.fwd_mt in (16, 32) and -2 <= tuning.split_bias <= 2
    op = make_plan(*CFG1)
    x = ji.config1_signal(0, n=op.N)
    S = host(J.Plan(J.Params(*CFG1), tuning=tuning).forward(dev(x)))
    assert rel(S, fftroute.forward(op, x)) <= TOL_S


WIDE = (8192, 7, 40, 2, 4, 2, 7, 16)


def test_wide_groups_parity():
    """Second-order groups of more than 128 stacked rows (the 64-k-step bucket: the
    register-W forward contraction and the widest backward, as at config 5) with 64
    frames: S and the gradient at full size against the oracle."""
    say("[parity] wide groups (K up to 145, 64 frames)")
    op = make_plan(*WIDE)
    assert max(g.K for g in op.groups) > 128
    x = ji.config1_signal(8, n=op.N)
    S_ref = fftroute.forward(op, x)
    say("[parity] wide groups: oracle forward done")
    plan, ws, S = run_forward(WIDE, x)
    assert_blocks(op, host(S), S_ref, "wide groups forward")
    dS = np.random.default_rng(6).standard_normal(op.n_coeff)
    dx = plan.backward(dev(x), dev(dS), ws=ws, reuse_forward=True)
    g_ref = fftroute.backward(op, x, dS)
    err_g = rel(host(dx), g_ref)
    say(f"[parity] wide groups backward: rel L2 {err_g:.3e}")
    assert err_g <= TOL_GRAD


CFG4 = (65536, 6, 8, 1, 3, 1, 9, 4)


def test_config4_many_frames_parity():
    """128 frames (T = 2^9 at N = 2^16): the forward pools each time chunk into a 32-frame
    window and the backward visits only the frames within the phi_T support."""
    say("[parity] config 4 (128 frames), full forward and backward")
    op = make_plan(*CFG4)
    x = ji.config4_signal(0)
    y = ji.white_noise_like(x, 1)
    S_x = fftroute.forward(op, x)
    S_y, cache = fftroute.forward(op, y, return_cache=True)
    plan = J.Plan(J.Params(*CFG4))
    ws = plan.workspace()
    yd = dev(y)
    S = plan.forward(yd, ws=ws)
    assert_blocks(op, host(S), S_y, "config 4 forward")
    dS = 2.0 * (S_y - S_x)
    g_ref = fftroute.backward(op, y, dS, cache=cache)
    dx = plan.backward(yd, dev(dS), ws=ws, reuse_forward=True)
    err = rel(host(dx), g_ref)
    say(f"[parity] config 4 backward: rel L2 {err:.3e}")
    assert err <= TOL_GRAD


@pytest.mark.parametrize("args", [(5000, 8, 8, 2, 3, 2, 8, 8.0), (3000, 7, 12, 2, 3, 2, 7, 6.0),
                                  (2048, 6, 8, 2, 3, 2, 6, 4.0), (2100, 6, 8, 2, 3, 2, 6, 4.0)])
def test_pooled_gradients_17_to_33_frames(args):
    """19, 23, 32 and 33 kept frames: up to 32 frames the backward stages each row tile's
    pooled gradients through LDS (32-frame instantiation, k-step buckets 4 to 16; the
    32-k-step bucket reads them in the loop), at 33 it reads them in the row loop."""
    say(f"[parity] frames test {args}")
    op = make_plan(*args)
    rng = np.random.default_rng(args[0])
    x = rng.standard_normal(args[0])
    y = rng.standard_normal(args[0])
    S_x = fftroute.forward(op, x)
    S_y, cache = fftroute.forward(op, y, return_cache=True)
    plan = J.Plan(J.Params(*args))
    ws = plan.workspace()
    yd = dev(y)
    S = plan.forward(yd, ws=ws)
    assert_blocks(op, host(S), S_y, f"{op.n_frames} frames forward")
    dS = 2.0 * (S_y - S_x)
    g_ref = fftroute.backward(op, y, dS, cache=cache)
    dx = plan.backward(yd, dev(dS), ws=ws, reuse_forward=True)
    err = rel(host(dx), g_ref)
    say(f"[parity] {op.n_frames} frames backward: rel L2 {err:.3e}")
    assert err <= TOL_GRAD
