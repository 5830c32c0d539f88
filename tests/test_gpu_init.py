"""GPU parity of the coloured-noise descent start (jtfs_colored_noise) with the FP64
oracle (oracle.init) on the same targets and the same standard normal draws.
Tolerance: relative L2 <= 1e-5 on y0 (FP32 transforms and sums against FP64)."""
import sys

import numpy as np
import pytest
import torch

import jtfs_inputs as ji
from oracle import init as OI
from oracle.plan import make_plan

pytestmark = pytest.mark.gpu

J = pytest.importorskip("paper_2602_11896_amd.jtfs")

TOL = 1e-5
CFG1 = (8192, 6, 8, 1, 3, 1, 9, 4)
CFG2 = (65536, 12, 12, 2, 4, 2, 13, 24)
TINY = (512, 4, 4, 1, 2, 1, 5, 2)


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def dev(x):
    return torch.as_tensor(np.asarray(x, dtype=np.float32), device="cuda").contiguous()


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


@pytest.mark.parametrize("name,cfg,periodic", [("cfg1", CFG1, False), ("cfg2", CFG2, False),
                                               ("cfg1 periodic", CFG1, True)])
def test_colored_noise_matches_oracle(name, cfg, periodic):
    say(f"[colored noise] {name}")
    n = cfg[0]
    x = ji.config2_signal(5, n=n) if n == 65536 else ji.config1_signal(4, n=n)
    w = ji.standard_normal(n, 17)
    plan = J.Plan(J.Params(*cfg, periodic=periodic))
    y0 = plan.colored_noise(dev(x), dev(w)).double().cpu().numpy()
    ref = OI.colored_noise(make_plan(*cfg, periodic=periodic), x.astype(np.float32).astype(np.float64),
                           w.astype(np.float32).astype(np.float64))
    err = rel(y0, ref)
    say(f"[colored noise] {name}: rel L2 {err:.3e}, rms y0 {np.sqrt(np.mean(ref ** 2)):.3e}")
    assert err <= TOL


def test_colored_noise_batch():
    """A heterogeneous batch in one call gives each signal its own start."""
    say("[colored noise] batch cfg1 + tiny")
    cfgs = [CFG1, TINY]
    xs = [ji.config1_signal(6, n=8192), ji.config1_signal(7, n=512)]
    ws = [ji.standard_normal(8192, 21), ji.standard_normal(512, 22)]
    plan = J.Plan([J.Params(*c) for c in cfgs])
    y0 = plan.colored_noise(dev(np.concatenate(xs)), dev(np.concatenate(ws))).double().cpu().numpy()
    o = 0
    for c, x, w in zip(cfgs, xs, ws):
        ref = OI.colored_noise(make_plan(*c), x.astype(np.float32).astype(np.float64),
                               w.astype(np.float32).astype(np.float64))
        err = rel(y0[o:o + c[0]], ref)
        say(f"  signal of {c[0]} samples: rel L2 {err:.3e}")
        assert err <= TOL
        o += c[0]
