"""Runners for the metamer workloads (synthetic inputs; see jtfs_inputs).

  python -m paper_2602_11896_amd.runs config1     # 20 GD steps, N = 2^13
  python -m paper_2602_11896_amd.runs config2     # Adam from noise at N = 2^16: time to rel. loss
  python -m paper_2602_11896_amd.runs config3     # 64 heterogeneous signals, batched + graph vs sequential
  python -m paper_2602_11896_amd.runs config5     # 8 x 2^20 samples: fwd+bwd, store vs recompute, peak HBM

Each prints one JSON line.
"""
from __future__ import annotations

import json
import sys
import time

import numpy as np
import torch

import jtfs_inputs as ji

from .autograd import jtfs
from .jtfs import MetamerGraph, Optimizer, Params, Plan

CFG1 = Params(8192, 6, 8, 1, 3, 1, 9, 4.0)
CFG2 = Params(65536, 12, 12, 2, 4, 2, 13, 24.0)


def _dev(x) -> torch.Tensor:
    return torch.as_tensor(np.asarray(x, dtype=np.float32), device="cuda").contiguous()


def config1(steps: int = 20) -> dict:
    plan = Plan(CFG1)
    x = ji.config1_signal(0)
    ws = plan.workspace()
    S_t = plan.forward(_dev(x), ws=ws).clone()
    y = _dev(ji.white_noise_like(x, 1))
    opt = Optimizer(plan, "gd", lr=0.1)
    loss = torch.zeros(1, device="cuda")
    norm = float(torch.dot(S_t, S_t))
    rel = []
    for _ in range(steps):
        plan.metamer_step(y, S_t, opt, loss, ws)
        rel.append(float(loss[0]) / norm)
    return {"workload": "config1", "steps": steps, "rel_loss_first": rel[0], "rel_loss_last": rel[-1]}


def descend_until(plan: Plan, S_t: torch.Tensor, y: torch.Tensor, opt: Optimizer, target_rel: float,
                  max_steps: int, check_every: int = 10, use_graph: bool = True) -> dict:
    """Descent until the relative loss (pre-update, per signal max) reaches target_rel."""
    ws = plan.workspace(y.device)
    loss = torch.zeros(plan.batch, device=y.device)
    norms = torch.stack([torch.dot(S_t[a:b], S_t[a:b]) for a, b in zip(plan.s_offsets[:-1], plan.s_offsets[1:])])
    g = MetamerGraph(plan, y, S_t, opt, loss, ws) if use_graph else None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps, rel = 0, float("inf")
    while steps < max_steps:
        for _ in range(check_every):
            g.step() if g else plan.metamer_step(y, S_t, opt, loss, ws)
            steps += 1
        rel = float((loss / norms).max())
        if rel <= target_rel:
            break
    torch.cuda.synchronize()
    return {"steps": steps, "seconds": time.perf_counter() - t0, "rel_loss": rel, "reached": rel <= target_rel}


def config2(max_steps: int = 500) -> dict:
    plan = Plan(CFG2)
    x = ji.config2_signal(2)
    S_t = plan.forward(_dev(x), ws=plan.workspace()).clone()
    y = _dev(ji.white_noise_like(x, 3))
    opt = Optimizer(plan, "adam", lr=0.1)
    out = descend_until(plan, S_t, y, opt, 1e-2, max_steps)
    out["workload"] = "config2 Adam lr 0.1 from white noise, target relative loss 1e-2"
    return out


def config3(n_signals: int = 64, iters: int = 10) -> dict:
    work = ji.batched_workload(n_signals)
    params = [Params(len(sig), 12, 12, 2, 4, 2, lt, F) for sig, lt, F in work]
    xs = [sig for sig, _, _ in work]
    # batched: one plan, one captured graph per iteration
    plan = Plan(params)
    ws = plan.workspace()
    x = _dev(np.concatenate(xs))
    S_t = plan.forward(x, ws=ws).clone()
    y = _dev(np.concatenate([ji.white_noise_like(s, 1000 + i) for i, s in enumerate(xs)]))
    opt = Optimizer(plan, "adam", lr=0.1)
    loss = torch.zeros(plan.batch, device="cuda")
    g = MetamerGraph(plan, y, S_t, opt, loss, ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(iters):
        g.step()
    torch.cuda.synchronize()
    t_batched = (time.perf_counter() - t0) / iters
    # sequential: one plan per signal, eager steps one after another
    plans = [Plan(p) for p in params]
    state = []
    for p, s in zip(plans, xs):
        w = p.workspace()
        st = p.forward(_dev(s), ws=w).clone()
        state.append((p, w, st, _dev(ji.white_noise_like(s, 7)), Optimizer(p, "adam", lr=0.1),
                      torch.zeros(1, device="cuda")))
    for p, w, st, yy, o, l in state:
        p.metamer_step(yy, st, o, l, w)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(iters):
        for p, w, st, yy, o, l in state:
            p.metamer_step(yy, st, o, l, w)
    torch.cuda.synchronize()
    t_seq = (time.perf_counter() - t0) / iters
    return {"workload": f"config3: {n_signals} signals, N in [2^14, 2^17], T in 2^11..2^13, F in 12/24/48",
            "batched_graph_ms_per_iter": t_batched * 1e3, "sequential_ms_per_iter": t_seq * 1e3,
            "speedup": t_seq / t_batched, "signals_per_s_batched": n_signals / t_batched}


def config5(n_signals: int = 8, iters: int = 2) -> dict:
    p = Params(1 << 20, 14, 16, 2, 5, 2, 14, 32.0)
    out = {"workload": f"config5: {n_signals} x 2^20 samples, J=14 Q1=16 Q2=2 J_fr=5 Q_fr=2 T=2^14 F=32"}
    plan = Plan([p] * n_signals)
    x = _dev(np.concatenate([ji.concatenated_signal(500 + i) for i in range(n_signals)]))
    for mode in ("recompute", "store"):
        torch.cuda.synchronize()
        torch.cuda.reset_peak_memory_stats()
        base = torch.cuda.memory_allocated()
        xx = x.clone().requires_grad_(True)
        t0 = time.perf_counter()
        for _ in range(iters):
            S = jtfs(xx, plan, mode)
            (S * S).sum().backward()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / iters
        out[mode] = {"iters_per_s": 1.0 / dt, "peak_hbm_GB": (torch.cuda.max_memory_allocated() - base) / 1e9}
        del xx, S
    return out


def main(argv) -> int:
    which = argv[1] if len(argv) > 1 else "config1"
    fn = {"config1": config1, "config2": config2, "config3": config3, "config5": config5}[which]
    print(json.dumps(fn()), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv))
