"""Python face of the JTFS library: plans, forward, backward and metamer steps.

Every computation runs in the HIP kernels behind the C ABI (include/jtfs.h); this
module only marshals arguments. PyTorch supplies device memory and the current stream.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Iterable, List, Sequence, Tuple, Union

import torch

from . import _lib as L


@dataclass(frozen=True)
class Params:
    """Parameters of one signal (jtfs_params): sample count and filterbank settings."""
    n: int
    J: int
    Q1: int
    Q2: int
    J_fr: int
    Q_fr: int
    log2_T: int
    F: float
    periodic: bool = False
    zeroth: bool = False          # output the zeroth-order block first (JTFS_ZEROTH)
    zeroth_weight: float = 0.0    # its weight in the metamer loss
    average_local: bool = True    # False: JTFS_NO_AVERAGE_LOCAL (U0, no phi_T on order 2)
    average_local_fr: bool = True  # False: JTFS_NO_AVERAGE_LOCAL_FR (k_fr = j_fr, no phi_F)

    def c(self) -> L.jtfs_params:
        flags = ((L.JTFS_ZEROTH if self.zeroth else 0) | (0 if self.average_local else L.JTFS_NO_AVERAGE_LOCAL) |
                 (0 if self.average_local_fr else L.JTFS_NO_AVERAGE_LOCAL_FR))
        return L.jtfs_params(self.n, self.J, self.Q1, self.Q2, self.J_fr, self.Q_fr, self.log2_T, float(self.F),
                             1 if self.periodic else 0, flags, float(self.zeroth_weight))


def _stream(device: torch.device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t: torch.Tensor) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def _require(t: torch.Tensor, numel: int, name: str, dtype=torch.float32) -> None:
    if not isinstance(t, torch.Tensor) or t.dtype != dtype or not t.is_cuda or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous {dtype} CUDA/HIP tensor")
    if t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")


@dataclass
class Tuning:
    """Tile schedules of a plan (jtfs_tuning); 0 selects a field's default. fwd_rows_k and
    bwd_rows_k hold per-bucket row targets for k-step buckets S = 4, 8, 16, 32, 64 (0: the
    global field)."""
    fwd_rows: int = 0
    fwd_mt: int = 0
    bwd_rows: int = 0
    split_bias: int = 0
    fwd_rows_k: Tuple[int, ...] = (0,) * L.JTFS_N_BUCKETS
    bwd_rows_k: Tuple[int, ...] = (0,) * L.JTFS_N_BUCKETS

    def c(self) -> L.jtfs_tuning:
        if len(self.fwd_rows_k) != L.JTFS_N_BUCKETS or len(self.bwd_rows_k) != L.JTFS_N_BUCKETS:
            raise ValueError(f"per-bucket targets need {L.JTFS_N_BUCKETS} entries")
        arr = ctypes.c_int32 * L.JTFS_N_BUCKETS
        return L.jtfs_tuning(self.fwd_rows, self.fwd_mt, self.bwd_rows, self.split_bias,
                             arr(*self.fwd_rows_k), arr(*self.bwd_rows_k))

    @staticmethod
    def from_c(t: L.jtfs_tuning) -> "Tuning":
        return Tuning(t.fwd_rows, t.fwd_mt, t.bwd_rows, t.split_bias, tuple(t.fwd_rows_k), tuple(t.bwd_rows_k))


def autotune(params: Union[Params, Sequence[Params]], device="cuda"):
    """Tile schedules measured fastest on this device (jtfs_autotune); returns (Tuning, ms)."""
    plist = [params] if isinstance(params, Params) else list(params)
    arr = (L.jtfs_params * len(plist))(*[p.c() for p in plist])
    t = L.jtfs_tuning()
    ms = ctypes.c_double()
    L.check(L.lib().jtfs_autotune(arr, len(plist), _stream(torch.device(device)), ctypes.byref(t), ctypes.byref(ms)),
            "jtfs_autotune")
    return Tuning.from_c(t), ms.value


class Plan:
    """A JTFS plan for one or more signals (jtfs_plan / jtfs_plan_tuned)."""

    def __init__(self, params: Union[Params, Sequence[Params]], tuning: "Tuning" = None):
        plist = [params] if isinstance(params, Params) else list(params)
        arr = (L.jtfs_params * len(plist))(*[p.c() for p in plist])
        handle = ctypes.c_void_p()
        if tuning is None:
            L.check(L.lib().jtfs_plan(arr, len(plist), ctypes.byref(handle)), "jtfs_plan")
        else:
            tc = tuning.c()
            L.check(L.lib().jtfs_plan_tuned(arr, len(plist), ctypes.byref(tc), ctypes.byref(handle)),
                    "jtfs_plan_tuned")
        self.tuning = tuning
        self._h = handle
        self._destroy = L.lib().jtfs_plan_destroy
        self.params = plist
        info = L.jtfs_plan_info()
        L.check(L.lib().jtfs_plan_query(self._h, ctypes.byref(info)), "jtfs_plan_query")
        self.batch = info.batch
        self.n_samples = info.n_samples_total
        self.n_coeff = info.n_coeff_total
        self.ws_forward = info.ws_forward
        self.ws_backward = info.ws_backward
        self.ws_shared_forward = info.ws_shared_forward
        self.ws_shared_backward = info.ws_shared_backward
        xo = (ctypes.c_int64 * (self.batch + 1))()
        so = (ctypes.c_int64 * (self.batch + 1))()
        L.check(L.lib().jtfs_plan_offsets(self._h, xo, so), "jtfs_plan_offsets")
        self.x_offsets = list(xo)
        self.s_offsets = list(so)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._destroy(h)
            self._h = None

    # ---------------------------------------------------------------- introspection
    def meta(self, signal: int = 0) -> List[dict]:
        n = ctypes.c_int64()
        L.check(L.lib().jtfs_plan_meta(self._h, signal, None, 0, ctypes.byref(n)), "jtfs_plan_meta")
        rows = (L.jtfs_path * n.value)()
        L.check(L.lib().jtfs_plan_meta(self._h, signal, rows, n.value, ctypes.byref(n)), "jtfs_plan_meta")
        keys = [f[0] for f in L.jtfs_path._fields_]
        return [{k: getattr(r, k) for k in keys} for r in rows]

    def filters(self, signal: int, bank: int):
        n = ctypes.c_int32()
        L.check(L.lib().jtfs_plan_filters(self._h, signal, bank, None, None, None, None, 0, ctypes.byref(n)),
                "jtfs_plan_filters")
        m = n.value
        xi, sg = (ctypes.c_double * m)(), (ctypes.c_double * m)()
        j, k = (ctypes.c_int32 * m)(), (ctypes.c_int32 * m)()
        L.check(L.lib().jtfs_plan_filters(self._h, signal, bank, xi, sg, j, k, m, ctypes.byref(n)),
                "jtfs_plan_filters")
        return list(xi), list(sg), list(j), list(k)

    def sizes(self, signal: int = 0) -> dict:
        out = (ctypes.c_int64 * 8)()
        L.check(L.lib().jtfs_plan_sizes(self._h, signal, out), "jtfs_plan_sizes")
        keys = ["N_pad", "pad_left", "N_fr", "s_F", "nf_pad", "f_lo", "n_frames", "n_coeff"]
        return dict(zip(keys, list(out)))

    def ws_region(self, ws: torch.Tensor, signal: int, which: int, dtype=torch.complex64) -> torch.Tensor:
        """View of an intermediate left in the workspace by forward (see jtfs_plan_ws_region)."""
        off, cnt = ctypes.c_int64(), ctypes.c_int64()
        L.check(L.lib().jtfs_plan_ws_region(self._h, signal, which, ctypes.byref(off), ctypes.byref(cnt)),
                "jtfs_plan_ws_region")
        item = torch.empty((), dtype=dtype).element_size()
        return ws[off.value: off.value + cnt.value * item].view(dtype)

    def cost(self, signal: int = 0) -> dict:
        """Forward frequential work (see jtfs_plan_cost), in multiply-adds."""
        out = (ctypes.c_double * 4)()
        L.check(L.lib().jtfs_plan_cost(self._h, signal, out), "jtfs_plan_cost")
        return dict(zip(["mac_dense", "mac_banded", "mac_exec", "mac_pool"], list(out)))

    def timing(self, on: bool, stages: Sequence[str] = None) -> None:
        """Bracket every kernel stage (or only the named ones) with HIP events on the
        caller's stream (see jtfs.h)."""
        if stages is None:
            L.check(L.lib().jtfs_timing_enable(self._h, 1 if on else 0), "jtfs_timing_enable")
            return
        mask = 0
        for name in stages:
            mask |= 1 << L.STAGE_NAMES.index(name)
        L.check(L.lib().jtfs_timing_stages(self._h, mask if on else 0), "jtfs_timing_stages")

    def timing_read(self) -> dict:
        """{stage name: (total ms, launches)} since the previous read (waits for the events)."""
        ms = (ctypes.c_double * L.JTFS_N_STAGES)()
        cnt = (ctypes.c_int64 * L.JTFS_N_STAGES)()
        L.check(L.lib().jtfs_timing_read(self._h, ms, cnt, L.JTFS_N_STAGES), "jtfs_timing_read")
        return {L.STAGE_NAMES[i]: (ms[i], cnt[i]) for i in range(L.JTFS_N_STAGES) if cnt[i]}

    def opt_state_floats(self, kind: int) -> int:
        return int(L.lib().jtfs_opt_state_floats(self._h, kind))

    # ---------------------------------------------------------------- buffers
    def workspace(self, device="cuda", backward: bool = True, shared: bool = False) -> torch.Tensor:
        """Workspace for forward (backward=False) or backward calls; `shared`: the size for
        calls with shared=True, where the signals take turns in one segment."""
        if shared:
            n = self.ws_shared_backward if backward else self.ws_shared_forward
        else:
            n = self.ws_backward if backward else self.ws_forward
        return torch.empty(max(n, 1), dtype=torch.uint8, device=device)

    # ---------------------------------------------------------------- compute
    def forward(self, x: torch.Tensor, S: torch.Tensor = None, ws: torch.Tensor = None,
                shared: bool = False) -> torch.Tensor:
        """S(x). shared=True: the signals run one after another in a workspace of
        ws_shared_forward bytes (JTFS_SHARED_WORKSPACE)."""
        _require(x, self.n_samples, "x")
        if S is None:
            S = torch.empty(self.n_coeff, dtype=torch.float32, device=x.device)
        _require(S, self.n_coeff, "S")
        if ws is None:
            ws = self.workspace(x.device, backward=False, shared=shared)
        flags = L.JTFS_SHARED_WORKSPACE if shared else 0
        L.check(L.lib().jtfs_forward_ex(self._h, _ptr(x), _ptr(S), _ptr(ws), ws.numel(), flags,
                                        _stream(x.device)), "jtfs_forward_ex")
        return S

    def joint_wavelet(self, n2: int, n_fr: int, n_t: int, signal: int = 0, device="cuda") -> torch.Tensor:
        """Re(psi_alpha(t) psi_beta(log2 lambda)) of path (n2, n_fr) on N_fr x n_t centred
        samples (jtfs_joint_wavelet; the interference pattern of Sec. 2.1, Fig. 1)."""
        n_fr_bins = self.sizes(signal)["N_fr"]
        out = torch.empty((n_fr_bins, n_t), dtype=torch.float32, device=device)
        L.check(L.lib().jtfs_joint_wavelet(self._h, signal, n2, n_fr, n_t, _ptr(out), _stream(out.device)),
                "jtfs_joint_wavelet")
        return out

    def prepare(self, device="cuda") -> None:
        """Set-up for forward_noalloc on `device` (jtfs_plan_prepare; allocates)."""
        with torch.cuda.device(torch.device(device)):
            L.check(L.lib().jtfs_plan_prepare(self._h), "jtfs_plan_prepare")

    def forward_noalloc(self, x: torch.Tensor, S: torch.Tensor) -> torch.Tensor:
        """S(x) with the library's static scratch as workspace (jtfs_forward_noalloc): the
        caller passes the output; the call allocates nothing. Needs prepare() first."""
        _require(x, self.n_samples, "x")
        _require(S, self.n_coeff, "S")
        L.check(L.lib().jtfs_forward_noalloc(self._h, _ptr(x), _ptr(S), _stream(x.device)), "jtfs_forward_noalloc")
        return S

    def backward(self, x: torch.Tensor, dS: torch.Tensor, dx: torch.Tensor = None, ws: torch.Tensor = None,
                 reuse_forward: bool = False, shared: bool = False) -> torch.Tensor:
        """dx = J_S(x)^T dS. shared=True: the signals run one after another in a workspace
        of ws_shared_backward bytes (JTFS_SHARED_WORKSPACE; with a batch of several signals
        it cannot be combined with reuse_forward)."""
        _require(x, self.n_samples, "x")
        _require(dS, self.n_coeff, "dS")
        if dx is None:
            dx = torch.empty(self.n_samples, dtype=torch.float32, device=x.device)
        _require(dx, self.n_samples, "dx")
        if ws is None:
            if reuse_forward:
                raise ValueError("reuse_forward needs the workspace of the preceding forward")
            ws = self.workspace(x.device, shared=shared)
        flags = (L.JTFS_REUSE_FORWARD if reuse_forward else 0) | (L.JTFS_SHARED_WORKSPACE if shared else 0)
        L.check(L.lib().jtfs_backward(self._h, _ptr(x), _ptr(dS), _ptr(dx), _ptr(ws), ws.numel(), flags,
                                      _stream(x.device)), "jtfs_backward")
        return dx

    def colored_noise(self, x: torch.Tensor, w: torch.Tensor, y0: torch.Tensor = None,
                      ws: torch.Tensor = None) -> torch.Tensor:
        """The descent start of Sec. 2.3 (jtfs_colored_noise): the standard normal draws w
        shaped to the power spectral density that S1 x describes."""
        _require(x, self.n_samples, "x")
        _require(w, self.n_samples, "w")
        if y0 is None:
            y0 = torch.empty(self.n_samples, dtype=torch.float32, device=x.device)
        _require(y0, self.n_samples, "y0")
        if ws is None:
            ws = self.workspace(x.device)
        L.check(L.lib().jtfs_colored_noise(self._h, _ptr(x), _ptr(w), _ptr(y0), _ptr(ws), ws.numel(),
                                           _stream(x.device)), "jtfs_colored_noise")
        return y0

    def metamer_step(self, y: torch.Tensor, S_target: torch.Tensor, opt: "Optimizer", loss: torch.Tensor,
                     ws: torch.Tensor) -> None:
        _require(y, self.n_samples, "y")
        _require(S_target, self.n_coeff, "S_target")
        _require(loss, self.batch, "loss")
        c = opt.c()
        L.check(L.lib().jtfs_metamer_step(self._h, _ptr(y), _ptr(S_target), ctypes.byref(c), _ptr(loss), _ptr(ws),
                                          ws.numel(), _stream(y.device)), "jtfs_metamer_step")


    def loss(self, S: torch.Tensor, S_target: torch.Tensor, dS: torch.Tensor = None, loss: torch.Tensor = None,
             relative: bool = True, scale: float = 1.0):
        """Per-signal (relative) loss and its gradient with respect to S (jtfs_loss); returns (loss, dS)."""
        _require(S, self.n_coeff, "S")
        _require(S_target, self.n_coeff, "S_target")
        if dS is None:
            dS = torch.empty(self.n_coeff, dtype=torch.float32, device=S.device)
        if loss is None:
            loss = torch.empty(self.batch, dtype=torch.float32, device=S.device)
        _require(dS, self.n_coeff, "dS")
        _require(loss, self.batch, "loss")
        L.check(L.lib().jtfs_loss(self._h, _ptr(S), _ptr(S_target), _ptr(dS), _ptr(loss), int(bool(relative)),
                                  float(scale), _stream(S.device)), "jtfs_loss")
        return loss, dS


class Optimizer:
    """Descent settings plus the device state buffer of jtfs_opt."""

    def __init__(self, plan: Plan, kind: str = "gd", lr: float = 0.1, momentum: float = 0.9, beta1: float = 0.9,
                 beta2: float = 0.999, eps: float = 1e-8, bold_up: float = 1.1, bold_down: float = 0.5,
                 device="cuda"):
        self.kind = {"gd": L.JTFS_OPT_GD, "momentum": L.JTFS_OPT_MOMENTUM_BOLD, "adam": L.JTFS_OPT_ADAM}[kind]
        self.lr, self.momentum = lr, momentum
        self.beta1, self.beta2, self.eps = beta1, beta2, eps
        self.bold_up, self.bold_down = bold_up, bold_down
        self.state = torch.zeros(max(plan.opt_state_floats(self.kind), 1), dtype=torch.float32, device=device)

    def c(self) -> L.jtfs_opt:
        return L.jtfs_opt(self.kind, self.lr, self.momentum, self.beta1, self.beta2, self.eps, self.bold_up,
                          self.bold_down, ctypes.c_void_p(self.state.data_ptr()))

    def reset(self) -> None:
        self.state.zero_()


def opt_status(plan: Plan, opt: Optimizer, raise_nonfinite: bool = True) -> List[int]:
    """Per-signal counts of metamer steps whose loss was not finite (jtfs_opt_status; waits
    for the current stream). Raises JTFSError with JTFS_ERR_NONFINITE if any is nonzero and
    raise_nonfinite is set."""
    counts = (ctypes.c_int32 * plan.batch)()
    c = opt.c()
    st = L.lib().jtfs_opt_status(plan._h, ctypes.byref(c), counts, _stream(opt.state.device))
    if st not in (L.JTFS_OK, L.JTFS_ERR_NONFINITE) or (st == L.JTFS_ERR_NONFINITE and raise_nonfinite):
        L.check(st, "jtfs_opt_status")
    return list(counts)


# Names of the C ABI, for callers that prefer them.
jtfs_plan = Plan


def jtfs_forward(plan: Plan, x, S=None, ws=None):
    return plan.forward(x, S, ws)


def jtfs_backward(plan: Plan, x, dS, dx=None, ws=None, reuse_forward=False):
    return plan.backward(x, dS, dx, ws, reuse_forward)


def jtfs_metamer_step(plan: Plan, y, S_target, opt: Optimizer, loss, ws):
    return plan.metamer_step(y, S_target, opt, loss, ws)


def jtfs_loss(plan: Plan, S, S_target, dS=None, loss=None, relative=True, scale=1.0):
    return plan.loss(S, S_target, dS, loss, relative, scale)


class MetamerGraph:
    """One metamer step of a plan captured as a HIP graph, replayed once per iteration.

    Capture needs the plan's device tables uploaded and every buffer allocated, so one
    step is first run eagerly and its effect on y, the optimiser state and the loss is
    undone before capturing. Replays are bitwise identical to eager steps (all kernels
    are deterministic and the graph holds no memset node).
    """

    def __init__(self, plan: Plan, y: torch.Tensor, S_target: torch.Tensor, opt: Optimizer, loss: torch.Tensor,
                 ws: torch.Tensor):
        self.plan, self.y, self.S_target, self.opt, self.loss, self.ws = plan, y, S_target, opt, loss, ws
        y0, st0, l0 = y.clone(), opt.state.clone(), loss.clone()
        plan.metamer_step(y, S_target, opt, loss, ws)
        torch.cuda.synchronize(y.device)
        y.copy_(y0)
        opt.state.copy_(st0)
        loss.copy_(l0)
        torch.cuda.synchronize(y.device)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            plan.metamer_step(y, S_target, opt, loss, ws)
        torch.cuda.synchronize(y.device)

    def step(self) -> None:
        self.graph.replay()
