"""rsg_dot_noalloc (partial sums in the library's static device array, for
callers that cannot allocate) against rsg_dot (caller workspace): the same
kernels, so the results are equal bit for bit; two calls in a row, the
second on a smaller input, so the second call runs over partials the first
left behind.  Called through the C ABI."""
import ctypes as C

import numpy as np
import pytest
import torch

import synth
from tests.gpu_common import rsg

pytestmark = pytest.mark.gpu


def _call(R, g, a, b, nst, noalloc):
    out = torch.full((2 * nst,), np.nan, dtype=torch.float64, device="cuda")
    if noalloc:
        rc = R._lib.rsg_dot_noalloc(g._h, a.data_ptr(), b.data_ptr(), nst, a.shape[1], out.data_ptr(), None)
    else:
        nbytes = int(R._lib.rsg_reduce_workspace_bytes(g._h, nst))
        ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        rc = R._lib.rsg_dot(g._h, a.data_ptr(), b.data_ptr(), nst, a.shape[1], out.data_ptr(), ws.data_ptr(),
                            nbytes, None)
    assert rc == 0, R._lib.rsg_last_error()
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _pair(g, nst, seed):
    a = torch.from_numpy(synth.white_noise(seed, g.np, nst, g.h).T.copy()).cuda()
    b = torch.from_numpy(synth.white_noise(seed + 1, g.np, nst, g.h).T.copy()).cuda()
    return a, b


def test_dot_noalloc_equals_dot_on_two_calls():
    R = rsg()
    assert int(R._lib.rsg_dot_noalloc_max_bytes()) == 1 << 20
    big = R.Grid(0.2, R=9.0)      # many partial sums per orbital
    small = R.Grid(0.3, R=2.5)
    for g, nst, seed in ((big, 16, 5), (small, 3, 6)):
        a, b = _pair(g, nst, seed)
        ref = _call(R, g, a, b, nst, noalloc=False)
        got = _call(R, g, a, b, nst, noalloc=True)
        np.testing.assert_array_equal(got, ref)
        assert np.all(np.isfinite(got))


def test_dot_noalloc_rejects_oversize_before_enqueueing():
    R = rsg()
    g = R.Grid(0.2, R=9.0)
    nst = 200  # 200 orbitals x 1024 partials x 16 B > 1 MiB
    assert int(R._lib.rsg_reduce_workspace_bytes(g._h, nst)) > (1 << 20)
    a = torch.zeros((nst, g.np), dtype=torch.complex128, device="cuda")
    out = torch.full((2 * nst,), 3.0, dtype=torch.float64, device="cuda")
    rc = R._lib.rsg_dot_noalloc(g._h, a.data_ptr(), a.data_ptr(), nst, g.np, out.data_ptr(), None)
    assert rc == -6 and b"scratch" in R._lib.rsg_last_error()
    torch.cuda.synchronize()
    assert torch.all(out == 3.0)
