"""The no-allocation forward (jtfs_forward_noalloc) against jtfs_forward, through the C ABI."""
import ctypes

import numpy as np
import pytest
import torch

import jtfs_inputs as ji

pytestmark = pytest.mark.gpu


def _run(args, seed):
    from paper_2602_11896_amd import _lib as L
    import paper_2602_11896_amd as J
    dev = torch.device("cuda:0")
    plan = J.Plan(J.Params(*args))
    assert plan.ws_shared_forward <= L.JTFS_NOALLOC_SCRATCH_BYTES
    x = torch.as_tensor(ji.config1_signal(seed, n=args[0]), dtype=torch.float32, device=dev)
    ws = plan.workspace(dev, backward=False)
    ref = plan.forward(x, ws=ws)
    plan.prepare(dev)
    S = torch.full((plan.n_coeff,), float("nan"), dtype=torch.float32, device=dev)
    st = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    rc = L.lib().jtfs_forward_noalloc(plan._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(S.data_ptr()), st)
    assert rc == L.JTFS_OK, L.lib().jtfs_last_error()
    torch.cuda.synchronize()
    return plan, ref.cpu().numpy(), S.cpu().numpy()


def test_noalloc_forward_matches_forward_twice_smaller_second():
    # first call on config 1's transform (N = 2^13), then a smaller plan (N = 512) that
    # finds the first call's contents in the scratch
    for args, seed in [((8192, 6, 8, 1, 3, 1, 9, 4.0), 0), ((512, 4, 4, 1, 2, 1, 5, 2), 1)]:
        print(f"noalloc forward: N={args[0]} seed={seed}", flush=True)
        _, ref, got = _run(args, seed)
        assert np.all(np.isfinite(got))
        # same kernels, same launch shapes, same order: bitwise equal
        assert np.array_equal(got, ref), float(np.max(np.abs(got - ref)))


def test_noalloc_forward_rejects_too_large_plan_and_unprepared():
    from paper_2602_11896_amd import _lib as L
    import paper_2602_11896_amd as J
    dev = torch.device("cuda:0")
    big = J.Plan(J.Params(65536, 12, 12, 2, 4, 2, 13, 24.0))
    assert big.ws_shared_forward > L.JTFS_NOALLOC_SCRATCH_BYTES
    x = torch.zeros(big.n_samples, device=dev)
    S = torch.zeros(big.n_coeff, device=dev)
    st = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    rc = L.lib().jtfs_forward_noalloc(big._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(S.data_ptr()), st)
    assert rc == L.JTFS_ERR_WORKSPACE
    small = J.Plan(J.Params(1024, 4, 4, 1, 2, 1, 5, 2))     # never prepared
    x = torch.zeros(small.n_samples, device=dev)
    S = torch.zeros(small.n_coeff, device=dev)
    rc = L.lib().jtfs_forward_noalloc(small._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(S.data_ptr()), st)
    assert rc == L.JTFS_ERR_ARG
