"""The batched and long-signal workloads on the GPU: per-signal parity of the 64-signal
heterogeneous batch against the oracle, and self-consistency of the 8 x 2^20-sample batch
through the recompute autograd path (where the oracle is out of reach)."""
import sys

import numpy as np
import pytest
import torch

import jtfs_inputs as ji
from oracle import fftroute
from oracle.plan import make_plan

pytestmark = pytest.mark.gpu

J = pytest.importorskip("paper_2602_11896_amd.jtfs")

TOL_S = 1e-5
TOL_GRAD = 1e-4


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def test_config3_batch_signals_against_oracle():
    """The 64-signal batch of uneven lengths with its own (T, F) per signal, run as one
    batched plan: four signals (T = 2^11 with F = 12 and F = 48, T = 2^12 with F = 48,
    T = 2^13 with F = 24) are compared block by block with the oracle, and the gradient
    of two of them."""
    work = ji.batched_workload(64)
    params = [J.Params(len(sig), 12, 12, 2, 4, 2, lt, F) for sig, lt, F in work]
    picks = [17, 42, 59, 27]
    assert [(work[i][1], work[i][2]) for i in picks] == [(11, 12.0), (11, 48.0), (12, 48.0), (13, 24.0)]
    say("[configs] config 3 batch: plan and forward of 64 signals")
    plan = J.Plan(params)
    x = torch.as_tensor(np.concatenate([s for s, _, _ in work]).astype(np.float32), device="cuda")
    ws = plan.workspace()
    S = host(plan.forward(x, ws=ws))
    rng = np.random.default_rng(3)
    dS = np.zeros(plan.n_coeff)
    grads = {}
    for i in picks[:2]:
        a, b = plan.s_offsets[i], plan.s_offsets[i + 1]
        dS[a:b] = rng.standard_normal(b - a)
    dx = host(plan.backward(x, torch.as_tensor(dS.astype(np.float32), device="cuda"), ws=ws, reuse_forward=True))
    for i in picks:
        sig, lt, F = work[i]
        say(f"[configs] config 3 signal {i}: N={len(sig)} T=2^{lt} F={F}")
        op = make_plan(len(sig), 12, 12, 2, 4, 2, lt, F)
        S_ref, cache = fftroute.forward(op, sig, return_cache=True)
        Sg = S[plan.s_offsets[i]: plan.s_offsets[i + 1]]
        assert Sg.size == S_ref.size
        worst = 0.0
        for blk in op.blocks:
            sl = slice(blk.offset, blk.offset + blk.n_lambda * blk.n_frames)
            e = rel(Sg[sl], S_ref[sl])
            worst = max(worst, e)
            assert e <= 10 * TOL_S, f"signal {i} block order={blk.order} n2={blk.n2} n_fr={blk.n_fr}: {e:.3e}"
        err = rel(Sg, S_ref)
        say(f"[configs] signal {i}: S rel L2 {err:.3e} (worst block {worst:.3e})")
        assert err <= TOL_S
        if i in picks[:2]:
            g_ref = fftroute.backward(op, sig, dS[plan.s_offsets[i]: plan.s_offsets[i + 1]], cache=cache)
            eg = rel(dx[plan.x_offsets[i]: plan.x_offsets[i + 1]], g_ref)
            say(f"[configs] signal {i}: dx rel L2 {eg:.3e}")
            assert eg <= TOL_GRAD
            grads[i] = eg
    # signals outside the picks got dS = 0: their gradient is exactly zero
    others = np.ones(plan.n_samples, dtype=bool)
    for i in picks[:2]:
        others[plan.x_offsets[i]: plan.x_offsets[i + 1]] = False
    assert np.all(dx[others] == 0.0)


def test_config5_recompute_self_consistency():
    """8 signals of 2^20 samples (J = 14, Q1 = 16, T = 2^14, F = 32) through the autograd
    recompute path (signals in turn in one shared workspace, U1 recomputed in the
    backward): the Euler identity of the degree-1 homogeneous transform per signal,
    <y, J^T dS> = <S(y), dS>, homogeneity S(c y) = |c| S(y), and bitwise determinism."""
    from paper_2602_11896_amd.autograd import jtfs
    n_sig = 8
    p = J.Params(1 << 20, 14, 16, 2, 5, 2, 14, 32.0)
    say("[configs] config 5: plan")
    plan = J.Plan([p] * n_sig)
    y = torch.as_tensor(np.concatenate([ji.concatenated_signal(500 + i) for i in range(n_sig)]).astype(np.float32),
                        device="cuda")
    dS = torch.as_tensor(np.random.default_rng(5).standard_normal(plan.n_coeff).astype(np.float32), device="cuda")

    def run(v):
        v = v.clone().requires_grad_(True)
        S = jtfs(v, plan, "recompute")
        S.backward(dS)
        return S.detach(), v.grad.detach()

    say("[configs] config 5: forward + backward (recompute)")
    S1, g1 = run(y)
    S2, g2 = run(y)
    assert torch.equal(S1, S2) and torch.equal(g1, g2)
    Sh, gh, yh, dSh = host(S1), host(g1), host(y), host(dS)
    for i in range(n_sig):
        xs, xe = plan.x_offsets[i], plan.x_offsets[i + 1]
        ss, se = plan.s_offsets[i], plan.s_offsets[i + 1]
        lhs = float(np.dot(yh[xs:xe], gh[xs:xe]))
        rhs = float(np.dot(Sh[ss:se], dSh[ss:se]))
        say(f"[configs] config 5 signal {i}: Euler {lhs:.8e} vs {rhs:.8e}")
        assert abs(lhs - rhs) <= 1e-5 * abs(rhs) + 1e-6 * np.linalg.norm(yh[xs:xe]) * np.linalg.norm(gh[xs:xe])
    say("[configs] config 5: homogeneity")
    with torch.no_grad():
        S3 = host(jtfs(-2.5 * y, plan, "recompute"))
    assert rel(S3, 2.5 * Sh) <= 1e-6
