"""Pins of the FP64 decoder oracle against library routines and finite differences."""
import numpy as np
import pytest
import torch

from jtfs_inputs import decoder_init
from oracle import decoder as D


def _torch_upconv(a, W, b, s):
    """PyTorch transposed convolution with the decoder's alignment ("same" after stuffing)."""
    K = W.shape[2]
    h = (K - 1) // 2
    wt = torch.as_tensor(W).flip(2).transpose(0, 1).contiguous()   # [C_in, C_out, K]
    return torch.nn.functional.conv_transpose1d(torch.as_tensor(a)[None], wt, torch.as_tensor(b),
                                                stride=s, padding=h, output_padding=s - 1)[0]


def _small_cfg(strides=(1, 4, 2, 1)):
    return D.DecoderConfig(c_in=6, n_frames=5, channels=4, kernel=9, strides=list(strides), leak=0.1, eps=1e-2)


def _theta(cfg, seed=3):
    layers = [(co, ci, s) for (co, ci, _, _), s in zip(cfg.shapes(), cfg.strides)]
    return decoder_init(layers, cfg.kernel, cfg.leak, seed)


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=4000) * 10.0 ** rng.integers(-6, 6, size=4000),
                        [0.0, -0.0, 1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -(1.0 + 2 ** -8)]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(D.bf16_round(x), ref)


@pytest.mark.parametrize("s", [1, 2, 4])
def test_upconv_is_transposed_convolution(s):
    rng = np.random.default_rng(s)
    a = rng.normal(size=(5, 7))
    W = rng.normal(size=(3, 5, 9))
    b = rng.normal(size=3)
    z = D.upconv(a, W, b, s)
    assert z.shape == (3, 7 * s)
    np.testing.assert_allclose(z, _torch_upconv(a, W, b, s).numpy(), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("s", [1, 2, 4])
def test_upconv_adjoint_matches_reverse_mode(s):
    rng = np.random.default_rng(10 + s)
    a = rng.normal(size=(4, 6))
    W = rng.normal(size=(3, 4, 9))
    b = rng.normal(size=3)
    dz = rng.normal(size=(3, 6 * s))
    ta = torch.tensor(a, requires_grad=True)
    tW = torch.tensor(W, requires_grad=True)
    tb = torch.tensor(b, requires_grad=True)
    wt = tW.flip(2).transpose(0, 1)
    z = torch.nn.functional.conv_transpose1d(ta[None], wt, tb, stride=s, padding=4, output_padding=s - 1)[0]
    (z * torch.tensor(dz)).sum().backward()
    dW, db, da = D.upconv_adjoint(dz, a, W, s)
    np.testing.assert_allclose(dW, tW.grad.numpy(), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(db, tb.grad.numpy(), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(da, ta.grad.numpy(), rtol=1e-12, atol=1e-12)


def test_decoder_gradient_matches_reverse_mode():
    cfg = _small_cfg()
    theta = _theta(cfg)
    rng = np.random.default_rng(4)
    S = rng.uniform(0.0, 0.1, size=cfg.c_in * cfg.n_frames)
    dy = rng.normal(size=cfg.out_len)
    y, cache = D.forward(cfg, theta, S, quantize=False)
    g = D.backward(cfg, theta, cache, dy, quantize=False)

    th = torch.tensor(theta, requires_grad=True)
    a = torch.log1p(torch.tensor(S).reshape(cfg.c_in, cfg.n_frames) / cfg.eps)
    o = 0
    for l, ((co, ci, _, _), s) in enumerate(zip(cfg.shapes(), cfg.strides)):
        W = th[o:o + co * ci * 9].reshape(co, ci, 9)
        o += co * ci * 9
        b = th[o:o + co]
        o += co
        z = torch.nn.functional.conv_transpose1d(a[None], W.flip(2).transpose(0, 1), b, stride=s,
                                                 padding=4, output_padding=s - 1)[0]
        a = torch.nn.functional.leaky_relu(z, cfg.leak) if l < cfg.n_layers - 1 else z
    np.testing.assert_allclose(y, a[0].detach().numpy(), rtol=1e-12, atol=1e-12)
    (a[0] * torch.tensor(dy)).sum().backward()
    np.testing.assert_allclose(g, th.grad.numpy(), rtol=1e-10, atol=1e-12)


def test_decoder_gradient_finite_differences():
    cfg = _small_cfg((2, 1, 4))
    theta = _theta(cfg, seed=7)
    rng = np.random.default_rng(5)
    S = rng.uniform(0.0, 0.1, size=cfg.c_in * cfg.n_frames)
    dy = rng.normal(size=cfg.out_len)
    _, cache = D.forward(cfg, theta, S, quantize=False)
    g = D.backward(cfg, theta, cache, dy, quantize=False)
    f = lambda th: float(np.dot(D.forward(cfg, th, S, quantize=False)[0], dy))
    h = 1e-6
    for idx in rng.choice(theta.size, size=40, replace=False):
        e = np.zeros_like(theta)
        e[idx] = h
        fd = (f(theta + e) - f(theta - e)) / (2 * h)
        assert abs(fd - g[idx]) <= 1e-6 * max(1.0, abs(g[idx])), (idx, fd, g[idx])


def test_quantized_forward_rounds_where_the_device_stores():
    cfg = _small_cfg()
    theta = _theta(cfg, seed=9)
    S = np.random.default_rng(6).uniform(0.0, 0.1, size=cfg.c_in * cfg.n_frames)
    y, (acts, Ws) = D.forward(cfg, theta, S, quantize=True)
    for a in acts:
        np.testing.assert_array_equal(a, D.bf16_round(a))
    for W in Ws:
        np.testing.assert_array_equal(W, D.bf16_round(W))
    # same pipeline through PyTorch's bfloat16 storage
    bf = lambda t: t.to(torch.float32).to(torch.bfloat16).to(torch.float64)
    a = bf(torch.log1p(torch.tensor(S).reshape(cfg.c_in, cfg.n_frames) / cfg.eps))
    for l, ((W, b), s) in enumerate(zip(D.unpack(cfg, theta), cfg.strides)):
        z = _torch_upconv(a.numpy(), bf(torch.tensor(W)).numpy(), b, s)
        a = bf(torch.nn.functional.leaky_relu(z, cfg.leak)) if l < cfg.n_layers - 1 else z
    np.testing.assert_allclose(y, a[0].numpy(), rtol=1e-12, atol=1e-12)


def test_adam_matches_torch():
    rng = np.random.default_rng(8)
    theta = rng.normal(size=50)
    m = np.zeros(50)
    v = np.zeros(50)
    p = torch.tensor(theta.copy(), requires_grad=True)
    opt = torch.optim.Adam([p], lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    for step in range(1, 6):
        g = rng.normal(size=50)
        theta, m, v = D.adam(theta, g, m, v, step, 3e-3)
        p.grad = torch.tensor(g)
        opt.step()
    np.testing.assert_allclose(theta, p.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_config4_decoder_shapes():
    cfg = D.DecoderConfig()
    assert cfg.out_len == 65536
    assert [t for _, _, t, _ in cfg.shapes()] == [128, 128, 512, 2048, 8192, 16384, 32768, 65536]
    assert 1.1e6 < D.n_params(cfg) < 1.3e6


def test_backward_branches_and_preactivation_gradients():
    """dz_out holds the gradient of every hidden pre-activation (PyTorch reverse mode);
    branches equal to the activations' signs change nothing; flipping one entry's branch
    scales that entry's dz by 1/leak (or leak) and leaves the rest of its layer alone."""
    cfg = _small_cfg()
    theta = _theta(cfg, seed=7)
    rng = np.random.default_rng(8)
    S = rng.uniform(0.0, 0.1, size=cfg.c_in * cfg.n_frames)
    dy = rng.normal(size=cfg.out_len)
    _, cache = D.forward(cfg, theta, S, quantize=False)
    dz = []
    g = D.backward(cfg, theta, cache, dy, quantize=False, dz_out=dz)
    acts = cache[0]
    same = D.backward(cfg, theta, cache, dy, quantize=False, branches=[a > 0 for a in acts[1:]])
    np.testing.assert_array_equal(same, g)

    th = torch.tensor(theta, requires_grad=True)
    a = torch.log1p(torch.tensor(S).reshape(cfg.c_in, cfg.n_frames) / cfg.eps)
    zs, o = [], 0
    for l, ((co, ci, _, _), s) in enumerate(zip(cfg.shapes(), cfg.strides)):
        W = th[o:o + co * ci * 9].reshape(co, ci, 9)
        o += co * ci * 9
        b = th[o:o + co]
        o += co
        z = torch.nn.functional.conv_transpose1d(a[None], W.flip(2).transpose(0, 1), b, stride=s,
                                                 padding=4, output_padding=s - 1)[0]
        if l < cfg.n_layers - 1:
            z.retain_grad()
            zs.append(z)
            a = torch.nn.functional.leaky_relu(z, cfg.leak)
        else:
            a = z
    (a[0] * torch.tensor(dy)).sum().backward()
    assert len(dz) == cfg.n_layers - 1
    for h, z in enumerate(zs):
        np.testing.assert_allclose(dz[h], z.grad.numpy(), rtol=1e-10, atol=1e-12)

    h = 1
    br = [a > 0 for a in acts[1:]]
    c, t = np.argwhere(~br[h])[0]
    br[h][c, t] = True
    dz2 = []
    D.backward(cfg, theta, cache, dy, quantize=False, branches=br, dz_out=dz2)
    np.testing.assert_allclose(dz2[h][c, t], dz[h][c, t] / cfg.leak, rtol=1e-12)
    keep = np.ones(dz[h].shape, dtype=bool)
    keep[c, t] = False
    np.testing.assert_array_equal(dz2[h][keep], dz[h][keep])
