"""lbfz_nn_mse_noalloc (the loss of the surrogate's training step without a
caller-provided partial-sum buffer) against lbfz_nn_mse through the C ABI:
two calls in a row, the second on a smaller input, each compared with the
workspace form on the same inputs.  Both forms run the same kernels with
the same number of partial sums, so loss and gradient agree bit for bit."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _mse_pair(torch, sg, P, C, cs, nblocks, seed):
    L = sg.nnlib()
    L.lbfz_nn_mse_noalloc.restype = ctypes.c_int
    L.lbfz_nn_mse_noalloc.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                      ctypes.c_long, ctypes.c_int32, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                      ctypes.c_void_p]
    g = torch.Generator().manual_seed(seed)
    out = torch.randn(P, cs, generator=g).to("cuda")
    tgt = torch.randn(P, C, generator=g).to("cuda")
    wch = torch.rand(C, generator=g).to("cuda")
    d_a = torch.full((P, cs), 7.0, dtype=torch.bfloat16, device="cuda")
    d_b = torch.full((P, cs), -3.0, dtype=torch.bfloat16, device="cuda")
    part = torch.empty(nblocks, dtype=torch.float64, device="cuda")
    loss_a = torch.empty(1, dtype=torch.float64, device="cuda")
    loss_b = torch.full((1,), 123.0, dtype=torch.float64, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    rc = L.lbfz_nn_mse(out.data_ptr(), cs, tgt.data_ptr(), P, C, wch.data_ptr(), d_a.data_ptr(),
                       part.data_ptr(), nblocks, loss_a.data_ptr(), st)
    assert rc == 0
    rc = L.lbfz_nn_mse_noalloc(out.data_ptr(), cs, tgt.data_ptr(), P, C, wch.data_ptr(),
                               d_b.data_ptr(), nblocks, loss_b.data_ptr(), st)
    assert rc == 0
    torch.cuda.synchronize()
    # the loss also against a float64 evaluation of its definition
    o64 = out[:, :C].double().cpu().numpy()
    t64 = tgt.double().cpu().numpy()
    w64 = wch.double().cpu().numpy()
    ref = float((w64 * (o64 - t64) ** 2).sum() / (P * C))
    return loss_a.item(), loss_b.item(), d_a.float().cpu().numpy(), d_b.float().cpu().numpy(), ref


def test_mse_noalloc_matches_workspace_form_twice():
    torch = pytest.importorskip("torch")
    from paper_2511_09422_amd import surrogate as sg
    for (P, C, cs, nblocks, seed) in ((256 * 256 * 2, 6, 8, 1024, 1), (64 * 64, 6, 8, 96, 2)):
        print(f"[noalloc] mse P={P} C={C} nblocks={nblocks}", flush=True)
        la, lb, da, db, ref = _mse_pair(torch, sg, P, C, cs, nblocks, seed)
        assert la == lb, (P, la, lb)
        assert np.array_equal(da, db), P
        assert abs(la - ref) <= 1e-6 * abs(ref), (la, ref)   # FP32 differences inside


def test_mse_noalloc_rejects_blocks_beyond_its_array():
    from paper_2511_09422_amd import surrogate as sg
    L = sg.nnlib()
    fake = 1 << 20   # never dereferenced: the size check fails first
    f = L.lbfz_nn_mse_noalloc
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_long, ctypes.c_int32,
                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                  ctypes.c_void_p]
    assert f(fake, 8, fake, 100, 6, None, None, 4097, fake, None) == sg.LBFZ_NN_EINVAL
    assert f(fake, 8, fake, 100, 6, None, None, 0, fake, None) == sg.LBFZ_NN_EINVAL
