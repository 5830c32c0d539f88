"""Runners for the metamer workloads (synthetic inputs; see jtfs_inputs).

  python -m paper_2602_11896_amd.runs config1     # 20 GD steps, N = 2^13
  python -m paper_2602_11896_amd.runs config2     # Adam from noise at N = 2^16: time to rel. loss
  python -m paper_2602_11896_amd.runs config3     # 64 heterogeneous signals, batched + graph vs sequential
  python -m paper_2602_11896_amd.runs config3_graph   # only the batched graph replays (for kernel traces)
  python -m paper_2602_11896_amd.runs config4     # learned warm start vs noise: time to rel. loss 1e-2
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
                  max_steps: int, check_every: int = 10, use_graph: bool = True, extra_targets=()) -> dict:
    """Descent until the relative loss (pre-update, per signal max) reaches target_rel.

    The loss of every step is kept on the device, so the first iterate below each target is
    found exactly even though the host checks only every ``check_every`` steps; the time to
    reach it is the measured wall time scaled to that step count (steps take equal time)."""
    ws = plan.workspace(y.device)
    loss = torch.zeros(plan.batch, device=y.device)
    norms = torch.stack([torch.dot(S_t[a:b], S_t[a:b]) for a, b in zip(plan.s_offsets[:-1], plan.s_offsets[1:])])
    hist = torch.zeros(max_steps, plan.batch, device=y.device)
    g = MetamerGraph(plan, y, S_t, opt, loss, ws) if use_graph else None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps, rel = 0, float("inf")
    while steps < max_steps:
        for _ in range(min(check_every, max_steps - steps)):
            g.step() if g else plan.metamer_step(y, S_t, opt, loss, ws)
            hist[steps].copy_(loss)
            steps += 1
        rel = float((loss / norms).max())
        if rel <= target_rel:
            break
    torch.cuda.synchronize()
    seconds = time.perf_counter() - t0
    rel_hist = (hist[:steps] / norms).max(dim=1).values.cpu().numpy()
    out = {"steps_run": steps, "seconds_run": seconds, "rel_loss": rel}
    for name, tgt in [("", target_rel)] + [(f"_{t:g}", t) for t in extra_targets]:
        below = np.nonzero(rel_hist <= tgt)[0]
        k = int(below[0]) if below.size else None   # iterate y_k (after k updates) is below tgt
        out["reached" + name] = k is not None
        out["steps" + name] = k
        out["seconds" + name] = seconds * k / steps if k is not None else None
    return out


def config2(max_steps: int = 500) -> dict:
    plan = Plan(CFG2)
    x = ji.config2_signal(2)
    S_t = plan.forward(_dev(x), ws=plan.workspace()).clone()
    y = _dev(ji.white_noise_like(x, 3))
    opt = Optimizer(plan, "adam", lr=0.1)
    out = descend_until(plan, S_t, y, opt, 1e-2, max_steps)
    out["workload"] = "config2 Adam lr 0.1 from white noise, target relative loss 1e-2"
    return out


def config4(n_signals: int = 32, learned_steps: int = 100, plain_max_steps: int = 5000, weights: str = None,
            target: float = 1e-2, extra_target: float = 1e-3, extra_cap: int = 1000,
            colored_max_steps: int = None) -> dict:
    """Time to relative loss 1e-2 from the learned start (decoder, then at most ``learned_steps``
    Adam steps), from white noise (Adam, at most ``plain_max_steps`` steps) and from the
    paper's coloured-noise start (Adam, and the paper's momentum + bold-driver update with
    mu0 = 0.1; at most ``colored_max_steps`` steps, default ``plain_max_steps``), on held-out
    seeds 0 .. n_signals-1 of the config-1 generator at N = 2^16, 8 kHz; Adam lr 0.1. The
    learned time counts the decoder and the evaluation of S at its output, the coloured
    time the construction of the start. The time to ``extra_target`` is reported too where
    it is reached within ``learned_steps`` (learned) or ``extra_cap`` steps (the others)."""
    from .decoder import Decoder, DecoderConfig
    from .train_decoder import CFG4, WEIGHTS, load_params
    cfg = DecoderConfig()
    theta = _dev(load_params(weights or WEIGHTS, cfg))
    dec = Decoder(cfg, 1)
    ws_d = dec.workspace()
    plan = Plan(CFG4)
    ws = plan.workspace()
    S_y = torch.empty(plan.n_coeff, device="cuda")
    rows = []
    for seed in range(-1, n_signals):       # seed -1: untimed warm-up of every code path
        x = ji.config4_signal(max(seed, 0))
        S_t = plan.forward(_dev(x), ws=ws).clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        y = dec.forward(theta, S_t, 1, ws=ws_d)
        loss0, _ = plan.loss(plan.forward(y, S_y, ws=ws), S_t, relative=True)
        rel0 = float(loss0[0])
        t_dec = time.perf_counter() - t0
        learned = descend_until(plan, S_t, y, Optimizer(plan, "adam", lr=0.1), extra_target, learned_steps,
                                check_every=5, extra_targets=(target,))
        lr_ = {"rel_loss_decoder": rel0, "decoder_and_check_seconds": t_dec}
        for tag, tgt in (("target", target), ("extra", extra_target)):
            name = "" if tgt == extra_target else f"_{tgt:g}"
            if rel0 <= tgt:
                lr_[tag] = {"reached": True, "steps": 0, "seconds": t_dec}
            elif learned["reached" + name]:
                lr_[tag] = {"reached": True, "steps": learned["steps" + name],
                            "seconds": t_dec + learned["seconds" + name]}
            else:
                lr_[tag] = {"reached": False, "steps": None, "seconds": None}
        y = _dev(ji.white_noise_like(x, 10 ** 5 + max(seed, 0)))
        plain = _two_targets(plan, S_t, y, Optimizer(plan, "adam", lr=0.1), target, extra_target, extra_cap,
                             plain_max_steps)
        # the paper's start (Sec. 2.3): noise coloured to S1 x, with Adam and with the
        # paper's momentum + bold-driver update; its time counts the start's construction
        xd, wd = _dev(x), _dev(ji.standard_normal(len(x), 2 * 10 ** 5 + max(seed, 0)))
        col = {}
        for name, kind in (("colored", "adam"), ("colored_bold", "momentum")):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            y = plan.colored_noise(xd, wd, ws=ws)
            torch.cuda.synchronize()
            t_init = time.perf_counter() - t0
            col[name] = _two_targets(plan, S_t, y, Optimizer(plan, kind, lr=0.1), target, extra_target, extra_cap,
                                     colored_max_steps or plain_max_steps, t_init)
        if seed < 0:
            continue
        rows.append({"seed": seed, "learned": lr_, "plain": plain, **col})
        print(json.dumps(rows[-1]), flush=True)

    def med(which, tag, key):
        v = [r[which][tag][key] for r in rows if r[which][tag]["reached"]]
        return float(np.median(v)) if v else None

    out = {"workload": f"config4: held-out seeds 0-{n_signals - 1}, learned start vs white noise vs the "
                       f"coloured-noise start (Adam lr 0.1; coloured also with momentum + bold driver, mu0 0.1)",
           "n_signals": n_signals, "median_rel_loss_decoder": float(np.median([r["learned"]["rel_loss_decoder"]
                                                                               for r in rows]))}
    for tag, tgt in (("target", target), ("extra", extra_target)):
        k = f"{tgt:g}"
        out[f"learned_reached_{k}"] = sum(r["learned"][tag]["reached"] for r in rows)
        out[f"plain_reached_{k}"] = sum(r["plain"][tag]["reached"] for r in rows)
        out[f"learned_median_seconds_{k}"] = med("learned", tag, "seconds")
        out[f"plain_median_seconds_{k}"] = med("plain", tag, "seconds")
        out[f"learned_median_steps_{k}"] = med("learned", tag, "steps")
        out[f"plain_median_steps_{k}"] = med("plain", tag, "steps")
        for name in ("colored", "colored_bold"):
            out[f"{name}_reached_{k}"] = sum(r[name][tag]["reached"] for r in rows)
            out[f"{name}_median_seconds_{k}"] = med(name, tag, "seconds")
            out[f"{name}_median_steps_{k}"] = med(name, tag, "steps")
    out["plain_seconds_per_step"] = float(np.median([r["plain"]["seconds_per_step"] for r in rows]))
    return out


def _two_targets(plan: Plan, S_t: torch.Tensor, y: torch.Tensor, opt: Optimizer, target: float, extra_target: float,
                 extra_cap: int, max_steps: int, t_init: float = 0.0) -> dict:
    """Descent from y to ``extra_target`` (at most ``extra_cap`` steps), continued to
    ``target`` alone up to ``max_steps``; per target: reached, steps, seconds (plus t_init)."""
    pl = descend_until(plan, S_t, y, opt, extra_target, min(extra_cap, max_steps), check_every=10,
                       extra_targets=(target,))
    if not pl[f"reached_{target:g}"] and max_steps > extra_cap:
        # continue the same descent up to the cap for the main target only
        more = descend_until(plan, S_t, y, opt, target, max_steps - extra_cap, check_every=10)
        pl[f"reached_{target:g}"] = more["reached"]
        pl[f"steps_{target:g}"] = extra_cap + more["steps"] if more["reached"] else None
        pl[f"seconds_{target:g}"] = pl["seconds_run"] + more["seconds"] if more["reached"] else None
        pl["steps_run"] += more["steps_run"]
        pl["seconds_run"] += more["seconds_run"]
    res = {}
    for tag, tgt in (("target", target), ("extra", extra_target)):
        name = "" if tgt == extra_target else f"_{tgt:g}"
        sec = pl["seconds" + name]
        res[tag] = {"reached": pl["reached" + name], "steps": pl["steps" + name],
                    "seconds": None if sec is None else t_init + sec}
    res["seconds_per_step"] = pl["seconds_run"] / pl["steps_run"]
    return res


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
    g.step()   # untimed first replay
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


def config3_graph(n_signals: int = 64, replays: int = 3) -> dict:
    """Only the batched half of config 3: the captured descent step, one untimed replay,
    then `replays` timed ones. Under a kernel trace the replays are the kernels after the
    last PyTorch kernel, in 1 + replays equal runs."""
    work = ji.batched_workload(n_signals)
    params = [Params(len(sig), 12, 12, 2, 4, 2, lt, F) for sig, lt, F in work]
    xs = [sig for sig, _, _ in work]
    plan = Plan(params)
    ws = plan.workspace()
    S_t = plan.forward(_dev(np.concatenate(xs)), ws=ws).clone()
    y = _dev(np.concatenate([ji.white_noise_like(s, 1000 + i) for i, s in enumerate(xs)]))
    opt = Optimizer(plan, "adam", lr=0.1)
    loss = torch.zeros(plan.batch, device="cuda")
    g = MetamerGraph(plan, y, S_t, opt, loss, ws)
    g.step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(replays):
        g.step()
    torch.cuda.synchronize()
    return {"workload": f"config3 batched graph: {n_signals} signals", "replays": replays,
            "ms_per_replay": (time.perf_counter() - t0) / replays * 1e3}


def config5(n_signals: int = 8, iters: int = 2) -> dict:
    p = Params(1 << 20, 14, 16, 2, 5, 2, 14, 32.0)
    out = {"workload": f"config5: {n_signals} x 2^20 samples, J=14 Q1=16 Q2=2 J_fr=5 Q_fr=2 T=2^14 F=32"}
    plan = Plan([p] * n_signals)
    # planned backward workspaces: one segment per signal (store) or one shared segment (recompute)
    out["ws_backward_GB"] = {"store": plan.ws_backward / 1e9, "recompute": plan.ws_shared_backward / 1e9}
    x = _dev(np.concatenate([ji.concatenated_signal(500 + i) for i in range(n_signals)]))
    for mode in ("recompute", "store"):
        torch.cuda.synchronize()
        torch.cuda.reset_peak_memory_stats()
        base = torch.cuda.memory_allocated()
        xx = x.clone().requires_grad_(True)
        (jtfs(xx, plan, mode) ** 2).sum().backward()   # untimed: first use uploads the plan's tables
        torch.cuda.synchronize()
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
    fn = {"config1": config1, "config2": config2, "config3": config3, "config3_graph": config3_graph,
          "config4": config4, "config5": config5}[which]
    print(json.dumps(fn()), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv))
