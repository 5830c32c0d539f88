"""Training of the warm-start decoder on (signal, S(signal)) pairs the transform generates.

Signals come from the config-1 generator at N = 2^16, 8 kHz (``jtfs_inputs.config4_signal``,
training seeds from 10^6 upwards), drawn on host worker processes while the GPU trains.
Per step, for a batch of B signals x:
    S_x = jtfs_forward(x)                       (targets, J = 6, Q1 = 8, T = 2^9, F = 4)
    y   = decoder(S_x)
    L   = (1 / B) sum_b ||S(y_b) - S_x,b||^2 / ||S_x,b||^2   (jtfs_forward + jtfs_loss)
    dy  = jtfs_backward(y, dL/dS)               (exact adjoint of the transform)
    grad = decoder backward(dy); Adam on the FP32 master parameters.
Every step runs in the library's kernels; Python orders the calls.

  python -m paper_2602_11896_amd.train_decoder --seconds 480 --batch 16 --out weights.npz
"""
from __future__ import annotations

import argparse
import json
import math
import multiprocessing as mp
import os
import queue
import sys
import time

import numpy as np
import torch

import jtfs_inputs as ji

from .decoder import Decoder, DecoderConfig
from .jtfs import Params, Plan

CFG4 = Params(65536, 6, 8, 1, 3, 1, 9, 4.0)
TRAIN_SEED0 = 10 ** 6
WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "decoder_config4.npz")


def _batch_signals(args):
    first, batch = args
    return np.stack([ji.config4_signal(first + i) for i in range(batch)]).astype(np.float32)


def _producer(q, stop, worker: int, n_workers: int, batch: int) -> None:
    """Batches worker, worker + n_workers, ... of the training stream, in order, into q,
    until `stop` is set."""
    q.cancel_join_thread()   # exit without waiting for unread batches to be flushed
    i = worker
    while not stop.is_set():
        x = _batch_signals((TRAIN_SEED0 + i * batch, batch))
        while not stop.is_set():
            try:
                q.put(x, timeout=0.2)
                break
            except queue.Full:
                pass
        i += n_workers


class _Batches:
    """Training batches from daemon worker processes, each with its own bounded queue, read
    round-robin so that batch i always holds seeds TRAIN_SEED0 + i B .. + B - 1."""

    def __init__(self, batch: int, workers: int):
        ctx = mp.get_context("fork")
        self.stop_event = ctx.Event()
        self.qs = [ctx.Queue(maxsize=2) for _ in range(workers)]
        self.ps = [ctx.Process(target=_producer, args=(q, self.stop_event, w, workers, batch), daemon=True)
                   for w, q in enumerate(self.qs)]
        for p in self.ps:
            p.start()
        self.i = 0

    def next(self) -> np.ndarray:
        x = self.qs[self.i % len(self.qs)].get()
        self.i += 1
        return x

    def stop(self) -> None:
        """Asks the workers to finish their current batch and exit; ends any that do not
        within a few seconds."""
        self.stop_event.set()
        deadline = time.monotonic() + 10.0
        for p in self.ps:
            p.join(timeout=max(0.0, deadline - time.monotonic()))
        for p in self.ps:
            if p.is_alive():
                p.terminate()
                p.join(timeout=1.0)
        for q in self.qs:
            q.cancel_join_thread()
            q.close()


def save_params(path: str, theta: np.ndarray, cfg: DecoderConfig, meta: dict) -> None:
    """Weights as bfloat16 bit patterns (the kernels use them rounded to bfloat16 anyway),
    biases as FP32."""
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    is_bias = np.zeros(theta.size, dtype=bool)
    o = 0
    for co, ci, _ in cfg.layer_shapes():
        o += co * ci * cfg.kernel
        is_bias[o:o + co] = True
        o += co
    f = theta.astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    bf = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)
    np.savez_compressed(path, weights_bf16=bf[~is_bias], biases=f[is_bias],
                        meta=np.frombuffer(json.dumps(meta).encode(), dtype=np.uint8))


def load_params(path: str, cfg: DecoderConfig) -> np.ndarray:
    z = np.load(path, allow_pickle=False)
    is_bias = []
    for co, ci, _ in cfg.layer_shapes():
        is_bias += [False] * (co * ci * cfg.kernel) + [True] * co
    is_bias = np.asarray(is_bias)
    theta = np.zeros(is_bias.size, dtype=np.float32)
    theta[~is_bias] = (z["weights_bf16"].astype(np.uint32) << 16).view(np.float32)
    theta[is_bias] = z["biases"]
    return theta


def train(seconds: float = 300.0, batch: int = 16, lr: float = 1e-3, init_seed: int = 0, workers: int = 12,
          log_every: int = 50, out: str = WEIGHTS, max_steps: int = 10 ** 9, resume: str = None) -> dict:
    # the generator processes are forked before this process touches the GPU
    batches = _Batches(batch, workers)
    cfg = DecoderConfig()
    plan = Plan([CFG4] * batch)
    dec = Decoder(cfg, max_batch=batch)
    if resume:
        theta0 = load_params(resume, cfg)
    else:
        theta0 = ji.decoder_init(cfg.layer_shapes(), cfg.kernel, cfg.leak, init_seed)
    theta = torch.as_tensor(np.asarray(theta0, dtype=np.float32), device="cuda").contiguous()
    m = torch.zeros_like(theta)
    v = torch.zeros_like(theta)
    ws_j = plan.workspace()
    ws_d = dec.workspace()
    x = torch.empty(plan.n_samples, dtype=torch.float32, device="cuda")
    S_t = torch.empty(plan.n_coeff, dtype=torch.float32, device="cuda")
    S_y = torch.empty(plan.n_coeff, dtype=torch.float32, device="cuda")
    dS = torch.empty(plan.n_coeff, dtype=torch.float32, device="cuda")
    loss = torch.empty(batch, dtype=torch.float32, device="cuda")
    y = torch.empty(plan.n_samples, dtype=torch.float32, device="cuda")
    dy = torch.empty(plan.n_samples, dtype=torch.float32, device="cuda")
    grad = torch.empty_like(theta)
    # two pinned staging buffers: one is refilled while the copy from the other may be in flight
    pins = [torch.empty(plan.n_samples, dtype=torch.float32).pin_memory() for _ in range(2)]
    copied = [None, None]

    history = []
    t_start = time.perf_counter()
    step = 0
    warm = 100
    try:
        while step < max_steps:
            sig = batches.next()
            k = step % 2
            if copied[k] is not None:
                copied[k].synchronize()
            pins[k].copy_(torch.from_numpy(sig.reshape(-1)))
            x.copy_(pins[k], non_blocking=True)
            copied[k] = torch.cuda.Event()
            copied[k].record()
            step += 1
            elapsed = time.perf_counter() - t_start
            frac = min(1.0, elapsed / seconds)
            lr_t = lr * min(1.0, step / warm) * (0.5 * (1.0 + math.cos(math.pi * frac)) * 0.9 + 0.1)
            plan.forward(x, S_t, ws=ws_j)
            dec.forward(theta, S_t, batch, y=y, ws=ws_d)
            plan.forward(y, S_y, ws=ws_j)
            plan.loss(S_y, S_t, dS, loss, relative=True, scale=1.0 / batch)
            plan.backward(y, dS, dy, ws=ws_j, reuse_forward=True)
            dec.backward(theta, dy, batch, ws_d, grad=grad)
            dec.adam_step(theta, grad, m, v, step, lr_t)
            if step % log_every == 0 or step == 1:
                mean_rel = float(loss.cpu().numpy().astype(np.float64).sum())   # scaled by 1/B: the mean
                history.append((step, round(elapsed, 2), mean_rel))
                print(json.dumps({"step": step, "seconds": round(elapsed, 1), "samples": step * batch,
                                  "mean_rel_loss": mean_rel, "lr": lr_t}), flush=True)
                if not math.isfinite(mean_rel):
                    raise RuntimeError("training diverged")
            if elapsed >= seconds:
                break
        torch.cuda.synchronize()
        wall = time.perf_counter() - t_start
        meta = {"steps": step, "batch": batch, "samples": step * batch, "seconds": round(wall, 1), "lr": lr,
                "init_seed": init_seed, "train_seeds": [TRAIN_SEED0, TRAIN_SEED0 + step * batch - 1],
                "final_mean_rel_loss": history[-1][2] if history else None}
        if out:
            save_params(out, theta.cpu().numpy(), cfg, meta)
            print(json.dumps({"saved": out}), flush=True)
    finally:
        batches.stop()
    meta["history"] = history
    return meta


def main(argv=None) -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--seconds", type=float, default=300.0)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--workers", type=int, default=12)
    ap.add_argument("--init-seed", type=int, default=0)
    ap.add_argument("--max-steps", type=int, default=10 ** 9)
    ap.add_argument("--resume", default=None)
    ap.add_argument("--out", default=WEIGHTS)
    a = ap.parse_args(argv)
    r = train(a.seconds, a.batch, a.lr, a.init_seed, a.workers, out=a.out, max_steps=a.max_steps, resume=a.resume)
    r.pop("history")
    print(json.dumps(r), flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
