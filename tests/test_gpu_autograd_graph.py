"""GPU tests of the autograd wrapper (store / recompute) and of graph-captured steps."""
import numpy as np
import pytest
import torch

import jtfs_inputs as ji
from oracle import descent, fftroute
from oracle.plan import make_plan

pytestmark = pytest.mark.gpu

J = pytest.importorskip("paper_2602_11896_amd.jtfs")
A = pytest.importorskip("paper_2602_11896_amd.autograd")

TINY = (512, 4, 4, 1, 2, 1, 5, 2)
CFG1 = (8192, 6, 8, 1, 3, 1, 9, 4)


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def dev(x):
    return torch.as_tensor(np.asarray(x, dtype=np.float32), device="cuda").contiguous()


@pytest.mark.parametrize("mode", ["store", "recompute"])
def test_autograd_matches_oracle_gradient(mode):
    print(f"[autograd] {mode} cfg1", flush=True)
    op = make_plan(*CFG1)
    x = ji.config1_signal(0)
    y = ji.white_noise_like(x, 1)
    S_x = fftroute.forward(op, x)
    S_y, cache = fftroute.forward(op, y, return_cache=True)
    g_ref = fftroute.backward(op, y, 2 * (S_y - S_x), cache=cache)
    plan = J.Plan(J.Params(*CFG1))
    yd = dev(y).requires_grad_(True)
    loss = ((A.jtfs(yd, plan, mode) - dev(S_x)) ** 2).sum()
    loss.backward()
    g = yd.grad.double().cpu().numpy()
    assert np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref) <= 1e-4


def test_store_and_recompute_are_bitwise_equal():
    print("[autograd] store vs recompute", flush=True)
    plan = J.Plan(J.Params(*CFG1))
    x = dev(ji.config1_signal(3))
    grads = []
    for mode in ("store", "recompute"):
        xx = x.clone().requires_grad_(True)
        S = A.jtfs(xx, plan, mode)
        (S * torch.arange(S.numel(), device="cuda", dtype=torch.float32)).sum().backward()
        grads.append(xx.grad.clone())
    assert torch.equal(grads[0], grads[1])


def test_shared_workspace_batch_is_bitwise_equal():
    """A heterogeneous batch run in one shared workspace (signals one after another) gives
    the same S and gradient, bit for bit, as with a segment per signal; the batched
    store/recompute autograd modes agree bit for bit as well."""
    params = [J.Params(*CFG1), J.Params(*TINY), J.Params(384, 4, 3, 2, 2, 2, 4, 3)]
    print("[shared ws] batch cfg1 + tiny + 384", flush=True)
    plan = J.Plan(params)
    x = dev(np.concatenate([ji.config1_signal(7), ji.config1_signal(8, n=512), ji.config1_signal(9, n=384)]))
    dS = dev(np.random.default_rng(5).normal(size=plan.n_coeff))
    S_own = plan.forward(x)
    S_sh = plan.forward(x, ws=plan.workspace(x.device, backward=False, shared=True), shared=True)
    dx_own = plan.backward(x, dS)
    ws_sh = plan.workspace(x.device, shared=True)
    assert ws_sh.numel() < plan.ws_backward
    dx_sh = plan.backward(x, dS, ws=ws_sh, shared=True)
    torch.cuda.synchronize()
    assert torch.equal(S_own, S_sh)
    assert torch.equal(dx_own, dx_sh)
    with pytest.raises(Exception):
        plan.backward(x, dS, ws=ws_sh, shared=True, reuse_forward=True)
    grads = []
    for mode in ("store", "recompute"):
        xx = x.clone().requires_grad_(True)
        (A.jtfs(xx, plan, mode) * dS).sum().backward()
        grads.append(xx.grad.clone())
    assert torch.equal(grads[0], grads[1])
    assert torch.equal(grads[0], dx_own)
    # one signal: a shared forward can be reused by the backward
    one = J.Plan(J.Params(*CFG1))
    x1 = x[:8192]
    ws1 = one.workspace(x.device, shared=True)
    one.forward(x1, ws=ws1, shared=True)
    dx1 = one.backward(x1, dS[:one.n_coeff], ws=ws1, shared=True, reuse_forward=True)
    assert torch.equal(dx1, dx_own[:8192])


def test_module_and_batch_autograd():
    print("[autograd] module on a batch", flush=True)
    m = A.JTFS([J.Params(*TINY), J.Params(*TINY)], mode="recompute")
    x = dev(np.concatenate([ji.config1_signal(0, n=512), ji.config1_signal(1, n=512)])).requires_grad_(True)
    S = m(x)
    S.sum().backward()
    op = make_plan(*TINY)
    g0 = fftroute.backward(op, x[:512].detach().double().cpu().numpy(), np.ones(op.n_coeff))
    g = x.grad[:512].double().cpu().numpy()
    assert np.linalg.norm(g - g0) / np.linalg.norm(g0) <= 1e-4


@pytest.mark.parametrize("kind", ["gd", "adam", "momentum"])
def test_graph_replays_equal_eager_steps(kind):
    print(f"[graph] {kind}", flush=True)
    plan = J.Plan(J.Params(*CFG1))
    ws = plan.workspace()
    x = dev(ji.config1_signal(0))
    S_t = plan.forward(x, ws=ws).clone()
    y0 = dev(ji.white_noise_like(ji.config1_signal(0), 1))
    lr = {"gd": 0.1, "adam": 0.1, "momentum": 500.0}[kind]

    ye, oe, le = y0.clone(), J.Optimizer(plan, kind, lr=lr), torch.zeros(1, device="cuda")
    eager = []
    for _ in range(6):
        plan.metamer_step(ye, S_t, oe, le, ws)
        eager.append(le.clone())
    torch.cuda.synchronize()

    yg, og, lg = y0.clone(), J.Optimizer(plan, kind, lr=lr), torch.zeros(1, device="cuda")
    g = J.MetamerGraph(plan, yg, S_t, og, lg, ws)
    for i in range(6):
        g.step()
        torch.cuda.synchronize()
        # eager work and a synchronisation between replays
        _ = (yg * 2).sum().item()
        assert torch.equal(lg, eager[i]), f"replay {i}"
    assert torch.equal(yg, ye)
    assert torch.equal(og.state, oe.state)


def test_batched_graph_replays_equal_eager_steps():
    # Signals of a batch run on the plan's internal streams (event fork / join), which a
    # captured graph records as branches.
    print("[graph] batch of three signals", flush=True)
    params = [J.Params(*TINY), J.Params(*CFG1), J.Params(384, 4, 3, 2, 2, 2, 4, 3)]
    plan = J.Plan(params)
    ws = plan.workspace()
    xs = [ji.config1_signal(i, n=p.n) for i, p in enumerate(params)]
    S_t = plan.forward(dev(np.concatenate(xs)), ws=ws).clone()
    y0 = dev(np.concatenate([ji.white_noise_like(x, 10 + i) for i, x in enumerate(xs)]))
    ye, oe, le = y0.clone(), J.Optimizer(plan, "adam", lr=0.1), torch.zeros(3, device="cuda")
    eager = []
    for _ in range(4):
        plan.metamer_step(ye, S_t, oe, le, ws)
        eager.append(le.clone())
    torch.cuda.synchronize()
    yg, og, lg = y0.clone(), J.Optimizer(plan, "adam", lr=0.1), torch.zeros(3, device="cuda")
    g = J.MetamerGraph(plan, yg, S_t, og, lg, ws)
    for i in range(4):
        g.step()
        torch.cuda.synchronize()
        assert torch.equal(lg, eager[i]), f"replay {i}"
    assert torch.equal(yg, ye)
