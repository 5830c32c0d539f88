"""CPU tests of the native library: exports, plan parity with the oracle, error paths,
and a host emulation of the FFT kernels' index logic. No device work is launched."""
import ctypes
import os
import re
import shutil
import subprocess

import numpy as np
import pytest

from oracle.plan import make_plan

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "jtfs.h")

J = pytest.importorskip("paper_2602_11896_amd.jtfs")
from paper_2602_11896_amd import _lib as L  # noqa: E402

CONFIGS = {
    "tiny": (512, 4, 4, 1, 2, 1, 5, 2, False),
    "tiny_b": (384, 4, 3, 2, 2, 2, 4, 3, False),
    "periodic": (1024, 4, 4, 2, 2, 2, 5, 2, True),
    "cfg1": (8192, 6, 8, 1, 3, 1, 9, 4, False),
    "cfg2": (65536, 12, 12, 2, 4, 2, 13, 24, False),
    "cfg4": (65536, 6, 8, 1, 3, 1, 9, 4, False),
    "cfg5": (1 << 20, 14, 16, 2, 5, 2, 14, 32, False),
}


def test_library_exports_every_declared_function():
    text = open(HEADER).read()
    declared = set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\*?\s+\**(jtfs_[a-z_]+)\s*\(", text, re.M))
    assert {"jtfs_plan", "jtfs_forward", "jtfs_backward", "jtfs_metamer_step"} <= declared
    lib = ctypes.CDLL(L.LIB_PATH)
    for name in declared:
        assert hasattr(lib, name), name
    assert {s[0] for s in L.SIGNATURES} == declared


@pytest.mark.parametrize("name", list(CONFIGS))
def test_plan_matches_oracle_plan(name):
    args = CONFIGS[name]
    op = make_plan(*args[:8], periodic=args[8])
    p = J.Plan(J.Params(*args))
    for bank, ref in ((0, op.psi1), (1, op.psi2), (2, op.fr)):
        xi, sg, j, k = p.filters(0, bank)
        assert len(xi) == len(ref)
        assert np.allclose(xi, [b.xi for b in ref], rtol=1e-15, atol=0)
        assert np.allclose(sg, [b.sigma for b in ref], rtol=1e-15, atol=0)
        assert j == [b.j for b in ref]
        if bank != 1:
            assert k == [b.k for b in ref]
    sz = p.sizes()
    assert (sz["N_pad"], sz["pad_left"], sz["N_fr"], sz["s_F"]) == (op.N_pad, op.pad_left, op.N_fr, op.s_F)
    assert (sz["nf_pad"], sz["f_lo"], sz["n_frames"], sz["n_coeff"]) == (op.nf_pad, op.f_lo, op.n_frames, op.n_coeff)
    rows = p.meta()
    assert len(rows) == len(op.blocks)
    for r, b in zip(rows, op.blocks):
        assert (r["order"], r["n2"], r["n_fr"], r["spin"], r["j2"], r["j_fr"], r["n_lambda"], r["n_frames"],
                r["offset"]) == (b.order, b.n2, b.n_fr, b.spin, b.j2, b.j_fr, b.n_lambda, b.n_frames, b.offset)


@pytest.mark.parametrize("name", ["tiny", "cfg1"])
def test_zeroth_order_layout_matches_oracle(name):
    # JTFS_ZEROTH: the S0 block first, every other block shifted by the kept frames
    args = CONFIGS[name]
    op = make_plan(*args[:8], periodic=args[8], zeroth=True)
    p = J.Plan(J.Params(*args, zeroth=True, zeroth_weight=0.5))
    assert p.n_coeff == op.n_coeff
    rows = p.meta()
    assert len(rows) == len(op.blocks)
    for r, b in zip(rows, op.blocks):
        assert (r["order"], r["n2"], r["n_fr"], r["n_lambda"], r["n_frames"], r["offset"]) == \
            (b.order, b.n2, b.n_fr, b.n_lambda, b.n_frames, b.offset)


@pytest.mark.parametrize("flags", [dict(average_local=False), dict(average_local_fr=False),
                                   dict(zeroth=True, average_local=False, average_local_fr=False)])
def test_unaveraged_layout_matches_oracle(flags):
    args = CONFIGS["tiny"]
    op = make_plan(*args[:8], periodic=args[8], **flags)
    p = J.Plan(J.Params(*args, **flags))
    assert p.n_coeff == op.n_coeff
    for r, b in zip(p.meta(), op.blocks):
        assert (r["order"], r["n2"], r["n_fr"], r["n_lambda"], r["n_frames"], r["offset"]) == \
            (b.order, b.n2, b.n_fr, b.n_lambda, b.n_frames, b.offset)
    _, _, j, k = p.filters(0, 2)
    assert k == [b.k for b in op.fr]


def test_bad_flags_and_weights_are_rejected():
    lib = L.lib()
    prm = J.Params(*CONFIGS["tiny"]).c()
    prm.flags = 8
    h = ctypes.c_void_p()
    assert lib.jtfs_plan(ctypes.byref(prm), 1, ctypes.byref(h)) == L.JTFS_ERR_ARG
    for w in (-1.0, float("nan"), float("inf")):
        prm = J.Params(*CONFIGS["tiny"], zeroth=True, zeroth_weight=w).c()
        assert lib.jtfs_plan(ctypes.byref(prm), 1, ctypes.byref(h)) == L.JTFS_ERR_ARG


def test_batch_offsets():
    a, b = CONFIGS["tiny"], CONFIGS["cfg1"]
    p = J.Plan([J.Params(*a), J.Params(*b), J.Params(*a)])
    na, nb = a[0], b[0]
    ca, cb = make_plan(*a[:8]).n_coeff, make_plan(*b[:8]).n_coeff
    assert p.x_offsets == [0, na, na + nb, 2 * na + nb]
    assert p.s_offsets == [0, ca, ca + cb, 2 * ca + cb]
    assert p.ws_forward < p.ws_backward


@pytest.mark.parametrize("bad,status", [
    ((1, 4, 4, 1, 2, 1, 5, 2, False), L.JTFS_ERR_ARG),            # n < 2
    ((512, 4, 0, 1, 2, 1, 5, 2, False), L.JTFS_ERR_ARG),          # Q1 = 0
    ((512, 4, 4, 1, 2, 1, 5, 0.5, False), L.JTFS_ERR_ARG),        # F < 1
    ((500, 4, 4, 1, 2, 1, 5, 2, True), L.JTFS_ERR_ARG),           # periodic, not a power of two
    ((512, 4, 4, 1, 2, 1, 12, 2, False), L.JTFS_ERR_ARG),         # T beyond the padded length
    ((512, 8, 4, 1, 2, 1, 2, 2, False), L.JTFS_ERR_UNSUPPORTED),  # second order coarser than T
])
def test_plan_rejects(bad, status):
    with pytest.raises(L.JTFSError) as e:
        J.Plan(J.Params(*bad))
    assert e.value.status == status


def test_host_side_argument_errors():
    lib = L.lib()
    p = J.Plan(J.Params(*CONFIGS["tiny"]))
    fake = ctypes.c_void_p(0x1000)
    assert lib.jtfs_forward(p._h, fake, fake, fake, 16, None) == L.JTFS_ERR_WORKSPACE
    assert lib.jtfs_forward(p._h, None, fake, fake, p.ws_forward, None) == L.JTFS_ERR_ARG
    assert lib.jtfs_backward(p._h, fake, fake, fake, fake, p.ws_forward, 0, None) == L.JTFS_ERR_WORKSPACE
    assert lib.jtfs_backward(p._h, fake, fake, fake, fake, p.ws_backward, 8, None) == L.JTFS_ERR_ARG
    opt = L.jtfs_opt(7, 0.1, 0.9, 0.9, 0.999, 1e-8, 1.1, 0.5, fake)
    assert lib.jtfs_metamer_step(p._h, fake, fake, ctypes.byref(opt), fake, fake, p.ws_backward, None) == L.JTFS_ERR_ARG
    assert lib.jtfs_opt_state_floats(p._h, 2) == 2 * 512 + 4
    assert b"workspace" in lib.jtfs_status_str(L.JTFS_ERR_WORKSPACE)


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_timing_stage_mask():
    lib = L.lib()
    p = J.Plan(J.Params(*CONFIGS["tiny"]))
    assert lib.jtfs_timing_stages(p._h, (1 << 6) | (1 << 9)) == L.JTFS_OK
    assert lib.jtfs_timing_stages(p._h, 1 << L.JTFS_N_STAGES) == L.JTFS_ERR_ARG
    assert lib.jtfs_timing_stages(None, 1) == L.JTFS_ERR_ARG
    p.timing(True, stages=("freq_fwd", "freq_bwd"))
    p.timing(False)
    assert p.timing_read() == {}


def test_colored_noise_host_argument_errors():
    lib = L.lib()
    p = J.Plan(J.Params(*CONFIGS["tiny"]))
    a, b, c = ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000), ctypes.c_void_p(0x3000)
    assert lib.jtfs_colored_noise(p._h, None, b, c, a, p.ws_backward, None) == L.JTFS_ERR_ARG
    assert lib.jtfs_colored_noise(p._h, a, b, a, c, p.ws_backward, None) == L.JTFS_ERR_ARG     # y0 aliases x
    assert lib.jtfs_colored_noise(p._h, a, b, b, c, p.ws_backward, None) == L.JTFS_ERR_ARG     # y0 aliases w
    assert lib.jtfs_colored_noise(p._h, a, b, c, a, p.ws_backward - 1, None) == L.JTFS_ERR_WORKSPACE


def test_shared_workspace_sizes_and_flags():
    """JTFS_SHARED_WORKSPACE: the batch needs the largest signal's segment, not the sum,
    and a shared forward cannot be reused by a batched backward."""
    a, b = J.Params(*CONFIGS["tiny"]), J.Params(*CONFIGS["cfg1"])
    batch = J.Plan([a, b, a])
    single = [J.Plan(q) for q in (a, b)]
    assert batch.ws_shared_forward == max(q.ws_forward for q in single)
    assert batch.ws_shared_backward == max(q.ws_backward for q in single)
    assert batch.ws_shared_backward < batch.ws_backward
    for q in single:   # one signal: the shared segment is the signal's own
        assert (q.ws_shared_forward, q.ws_shared_backward) == (q.ws_forward, q.ws_backward)
    lib = L.lib()
    fake = ctypes.c_void_p(0x1000)
    SH, RE = L.JTFS_SHARED_WORKSPACE, L.JTFS_REUSE_FORWARD
    h = batch._h
    assert lib.jtfs_forward_ex(h, fake, fake, fake, batch.ws_shared_forward - 1, SH, None) == L.JTFS_ERR_WORKSPACE
    assert lib.jtfs_forward_ex(h, fake, fake, fake, batch.ws_forward, RE, None) == L.JTFS_ERR_ARG
    assert lib.jtfs_forward_ex(h, fake, fake, fake, batch.ws_forward, 4, None) == L.JTFS_ERR_ARG
    assert lib.jtfs_backward(h, fake, fake, fake, fake, batch.ws_shared_backward - 1, SH, None) == L.JTFS_ERR_WORKSPACE
    assert lib.jtfs_backward(h, fake, fake, fake, fake, batch.ws_backward, SH | RE, None) == L.JTFS_ERR_ARG
    assert b"batch of one" in lib.jtfs_last_error()
    assert lib.jtfs_backward(h, fake, fake, fake, fake, batch.ws_backward, 4, None) == L.JTFS_ERR_ARG


def test_fft_tile_index_logic_host_emulation(tmp_path):
    exe = tmp_path / "fft_emul"
    subprocess.run(["g++", "-std=c++17", "-O2", "-o", str(exe), os.path.join(ROOT, "tests", "native", "fft_emul.cpp")],
                   check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.strip().endswith("OK")
    assert "tile_slot permutation ok" in out.stdout and "tile bank spread ok" in out.stdout


def _dec(cfg, max_batch=2):
    from paper_2602_11896_amd.decoder import Decoder
    return Decoder(cfg, max_batch)


def test_decoder_sizes_match_oracle():
    from oracle import decoder as OD
    from paper_2602_11896_amd.decoder import DecoderConfig
    for strides, c_in, F in (([1, 4, 4, 4, 2, 2, 2, 1], 266, 128), ([2, 1], 3, 8), ([4, 1, 2, 1], 20, 16)):
        cfg = DecoderConfig(c_in=c_in, n_frames=F, strides=strides)
        ocfg = OD.DecoderConfig(c_in=c_in, n_frames=F, strides=strides)
        d = _dec(cfg, 4)
        assert d.n_params == OD.n_params(ocfg)
        assert d.out_len == ocfg.out_len
        assert d.ws_bytes > 0


@pytest.mark.parametrize("field,value", [("channels", 64), ("kernel", 7), ("n_frames", 12), ("c_in", 0),
                                         ("strides", [1]), ("strides", [3, 1]), ("strides", [1, 2]),
                                         ("leak", 0.0), ("eps", -1.0)])
def test_decoder_rejects(field, value):
    from paper_2602_11896_amd.decoder import DecoderConfig
    cfg = DecoderConfig(c_in=10, n_frames=16, strides=[2, 1])
    setattr(cfg, field, value)
    with pytest.raises(L.JTFSError) as e:
        _dec(cfg)
    assert e.value.status in (L.JTFS_ERR_ARG, L.JTFS_ERR_UNSUPPORTED)


def test_decoder_host_argument_errors():
    from paper_2602_11896_amd.decoder import DecoderConfig
    d = _dec(DecoderConfig(c_in=10, n_frames=16, strides=[2, 1]), 2)
    lib = L.lib()
    buf = ctypes.create_string_buffer(16)
    p = ctypes.cast(buf, ctypes.c_void_p)
    assert lib.jtfs_dec_forward(d._h, p, p, 3, p, p, d.ws_bytes, None) == L.JTFS_ERR_ARG        # batch > max
    assert lib.jtfs_dec_forward(d._h, p, p, 1, p, p, d.ws_bytes - 1, None) == L.JTFS_ERR_WORKSPACE
    assert lib.jtfs_dec_forward(d._h, None, p, 1, p, p, d.ws_bytes, None) == L.JTFS_ERR_ARG
    assert lib.jtfs_dec_backward(d._h, p, 0, p, p, p, d.ws_bytes, None) == L.JTFS_ERR_ARG
    assert lib.jtfs_dec_adam_step(d._h, p, p, p, p, 0, 1e-3, 0.9, 0.999, 1e-8, None) == L.JTFS_ERR_ARG
    assert lib.jtfs_dec_adam_step(d._h, p, p, p, p, 1, 1e-3, 1.0, 0.999, 1e-8, None) == L.JTFS_ERR_ARG
    lib.jtfs_dec_destroy(None)
    plan = J.Plan(J.Params(*CONFIGS["tiny"][:8], periodic=CONFIGS["tiny"][8]))
    assert lib.jtfs_loss(plan._h, p, p, p, p, 1, 1.0, None) == L.JTFS_ERR_ARG               # dS aliases S
    assert lib.jtfs_loss(plan._h, None, p, p, p, 1, 1.0, None) == L.JTFS_ERR_ARG


@pytest.mark.parametrize("tuning", [(128, 16, 512, 1), (1024, 32, 128, -1), (0, 0, 0, 2), (16, 16, 8192, -2),
                                    (256, 32, 256, 0, (64, 1024, 16, 8192, 0), (8192, 16, 64, 1024, 512))])
def test_tuned_plans_keep_the_layout(tuning):
    """Tile schedules change neither the output layout nor the offsets of a plan."""
    args = CONFIGS["cfg2"]
    p0 = J.Plan(J.Params(*args[:8], periodic=args[8]))
    p1 = J.Plan(J.Params(*args[:8], periodic=args[8]), tuning=J.Tuning(*tuning))
    assert p1.n_coeff == p0.n_coeff and p1.n_samples == p0.n_samples
    assert p1.s_offsets == p0.s_offsets and p1.x_offsets == p0.x_offsets
    assert p1.meta() == p0.meta()


@pytest.mark.parametrize("tuning", [(8, 0, 0, 0), (0, 24, 0, 0), (0, 0, 20000, 0), (0, 0, 0, 3), (0, 0, 0, -3),
                                    (0, 0, 0, 0, (8, 0, 0, 0, 0), (0,) * 5), (0, 0, 0, 0, (0,) * 5, (0, 0, 0, 0, 9000))])
def test_tuning_out_of_range_is_rejected(tuning):
    args = CONFIGS["tiny"]
    with pytest.raises(L.JTFSError) as e:
        J.Plan(J.Params(*args[:8], periodic=args[8]), tuning=J.Tuning(*tuning))
    assert e.value.status == L.JTFS_ERR_ARG
