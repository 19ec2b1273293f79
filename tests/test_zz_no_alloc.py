"""The allocation-free residual check (mrhs_residual_norms_noalloc) against the entry point
with a caller's workspace (mrhs_residual_norms), through the C-ABI: two calls in a row on
the library's static scratch, the second with a smaller input, each equal bit for bit to
the workspace call (the same kernels and summation order); requests beyond the scratch
are refused before anything is enqueued."""
import numpy as np
import pytest
import torch

from gpu_helpers import Case, announce, need_gpu
from paper_1601_03184_amd import inputs, mrhs

pytestmark = pytest.mark.gpu


def residuals(case, block, prec, n, seed):
    op = case.op(block, prec=prec, short_len=4)
    b = op.pack(torch.from_numpy(inputs.test_vectors(case.L, n, seed)))
    x = op.empty(n)
    mrhs.sap_smooth_mrhs(op.handle, b, x, n, 1, 2, op.workspace(n))
    ref = torch.full((n,), -1.0, dtype=torch.float64, device="cuda")
    mrhs.mrhs_residual_norms(op.handle, b, x, n, ref, op.workspace(n))
    got = torch.full((n,), -2.0, dtype=torch.float64, device="cuda")
    mrhs.mrhs_residual_norms_noalloc(op.handle, b, x, n, got)
    torch.cuda.synchronize()
    op.close()
    return got.cpu().numpy(), ref.cpu().numpy()


def test_noalloc_residual_equals_workspace_call():
    need_gpu()
    announce("noalloc residual: 8x8x8x16, 4^4 blocks, 14 rhs, FP32")
    big = Case([8, 8, 8, 16], 0.3, 611, -0.2)
    got, ref = residuals(big, [4, 4, 4, 4], mrhs.PREC_F32, 14, 612)
    assert np.all(ref > 0) and np.all(ref < 1)
    assert np.array_equal(got, ref)
    # second call, smaller input: the scratch keeps the first call's partial sums, which the
    # smaller call must not pick up
    announce("noalloc residual: 4^4, 2^4 blocks, 3 rhs, FP64")
    small = Case([4, 4, 4, 4], 0.3, 613, -0.1)
    got, ref = residuals(small, [2, 2, 2, 2], mrhs.PREC_F64, 3, 614)
    assert np.all(ref > 0) and np.all(ref < 1)
    assert np.array_equal(got, ref)


def test_noalloc_residual_refuses_oversized_request():
    """65536 blocks of one site x 40 right-hand sides need 42 MB of partial sums: refused
    on the host (EUNSUPPORTED), nothing is launched."""
    need_gpu()
    L = [16, 16, 16, 16]
    U = torch.from_numpy(inputs.unit_gauge_field(L))
    op = mrhs.Operator(L, [1, 1, 1, 1], [2, 2, 2, 2], U, -0.1, 1.0, prec=mrhs.PREC_F32, short_len=4)
    b = op.empty(40)
    out = torch.zeros(40, dtype=torch.float64, device="cuda")
    with pytest.raises(mrhs.MrhsError) as e:
        mrhs.mrhs_residual_norms_noalloc(op.handle, b, b, 40, out)
    assert e.value.code == mrhs.MRHS_EUNSUPPORTED
    op.close()
