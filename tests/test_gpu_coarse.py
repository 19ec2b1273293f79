"""GPU parity of block Gram-Schmidt (block_orthonormalize) and the coarse operator
(coarse_op_build) against the FP64 oracle, through the C-ABI."""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import Case, announce, need_gpu, per_agg_half_rel
from paper_1601_03184_amd import inputs
from paper_1601_03184_amd import mrhs

pytestmark = pytest.mark.gpu

F64, F32, F16 = mrhs.PREC_F64, mrhs.PREC_F32, mrhs.PREC_F32_F16STORE
D64, D32, D16 = mrhs.DTYPE_F64, mrhs.DTYPE_F32, mrhs.DTYPE_F16


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def run_gs(op, vn, vdt, qdt, n, in_place=False):
    status = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    Q = vn if in_place else op.empty(n, qdt)
    mrhs.block_orthonormalize(op.handle, vn, vdt, Q, qdt, n, status, op.workspace(n))
    torch.cuda.synchronize()
    return Q, int(status.item())


GS_CASES = [
    # (L, block, agg, prec, S, n, vdt, qdt, in_place, smooth)
    ([4, 4, 4, 4], [2, 2, 2, 2], [2, 2, 2, 2], F64, 4, 8, D64, D64, False, True),
    ([4, 4, 4, 4], [2, 2, 2, 2], [2, 2, 2, 2], F64, 4, 8, D64, D64, True, True),
    ([8, 8, 4, 8], [4, 4, 4, 4], [4, 4, 4, 4], F32, 4, 20, D32, D64, False, True),
    ([8, 8, 4, 8], [4, 4, 4, 4], [4, 4, 4, 4], F32, 4, 20, D32, D32, True, False),
    ([8, 4, 4, 8], [4, 4, 4, 4], [4, 4, 4, 4], F16, 4, 24, D16, D64, False, False),
    ([8, 4, 8, 4], [4, 4, 4, 4], [2, 4, 4, 2], F32, 8, 13, D32, D64, False, False),  # aggregates != blocks
    ([4, 4, 4, 8], [2, 2, 2, 2], [4, 4, 4, 4], F64, 2, 32, D64, D64, False, False),  # aggregate = 16 blocks
    ([8, 8, 4, 8], [4, 4, 4, 4], [4, 4, 4, 4], F32, 4, 20, D32, D16, False, True),   # FP16 storage of Q
    ([8, 4, 4, 8], [4, 4, 4, 4], [4, 4, 4, 4], F16, 4, 24, D16, D16, True, False),   # FP16 in place
    ([8, 4, 4, 16], [4, 4, 4, 4], [4, 4, 4, 8], F32, 4, 12, D32, D64, False, False),  # 512 sites: two stagings
]


@pytest.mark.parametrize("L,block,agg,prec,S,n,vdt,qdt,in_place,smooth", GS_CASES)
def test_gs_parity(L, block, agg, prec, S, n, vdt, qdt, in_place, smooth):
    need_gpu()
    case = Case(L, 0.3, 301, -0.2)
    announce("gs L=%s agg=%s n=%d vdt=%d qdt=%d inplace=%d" % (L, agg, n, vdt, qdt, in_place))
    op = case.op(block, agg=agg, prec=prec, short_len=S)
    v = inputs.test_vectors(L, n, 302)
    if smooth:
        v = oracle.sap(L, block, case.U, case.A, v, 2, 3)
    vn = op.pack(torch.from_numpy(v), vdt)
    vin = op.unpack(vn, n, vdt).cpu().numpy()  # the values the kernel reads
    Q, status = run_gs(op, vn, vdt, qdt, n, in_place)
    assert status == 0
    got = op.unpack(Q, n, qdt).cpu().numpy()
    ref = oracle.block_gs(L, agg, vin)
    # FP16 storage: one rounding of each entry (relative 2^-12 at most); Q is compared per
    # (aggregate, spin half), the unit in which the factorisation is defined
    tol = {D64: 1e-12, D32: 1e-6, D16: 1e-3}[qdt]
    err = per_agg_half_rel(got, ref, L, agg)
    assert err < tol, err
    op.close()


def test_gs_rank_deficiency_flagged():
    need_gpu()
    L = [4, 4, 4, 4]
    case = Case(L, 0.3, 301, -0.2)
    op = case.op([2, 2, 2, 2], prec=F64, short_len=4)
    v = inputs.test_vectors(L, 4, 303)
    v[3] = 0.5 * v[0] - 2j * v[2]
    announce("gs rank deficiency")
    vn = op.pack(torch.from_numpy(v))
    _, status = run_gs(op, vn, D64, D64, 4)
    assert status == 1  # aggregate 0, half 0 is the first flagged
    op.close()


COARSE_CASES = [
    # (L, block, agg, prec, S, n, qdt)
    ([4, 4, 4, 4], [2, 2, 2, 2], [2, 2, 2, 2], F64, 4, 8, D32),
    ([4, 4, 4, 4], [2, 2, 2, 2], [2, 2, 2, 2], F64, 4, 8, D64),
    ([8, 8, 4, 8], [4, 4, 4, 4], [4, 4, 4, 4], F32, 4, 20, D32),
    ([8, 4, 8, 4], [4, 4, 4, 4], [2, 4, 4, 2], F32, 8, 13, D32),
    ([4, 4, 2, 4], [2, 2, 2, 2], [2, 4, 2, 2], F32, 4, 4, D32),   # coarse extents 2 and 1
    ([8, 4, 4, 8], [4, 4, 4, 4], [4, 4, 4, 4], F32, 4, 32, D32),
    ([8, 8, 4, 8], [4, 4, 4, 4], [4, 4, 4, 4], F32, 4, 20, D16),   # FP16 storage of Q
    ([4, 4, 4, 4], [2, 2, 2, 2], [2, 2, 2, 2], F64, 4, 8, D16),
]


@pytest.mark.parametrize("L,block,agg,prec,S,n,qdt", COARSE_CASES)
def test_coarse_parity(L, block, agg, prec, S, n, qdt):
    need_gpu()
    case = Case(L, 0.3, 311, -0.2)
    announce("coarse L=%s agg=%s n=%d qdt=%d" % (L, agg, n, qdt))
    op = case.op(block, agg=agg, prec=prec, short_len=S)
    v = inputs.test_vectors(L, n, 312)
    q = oracle.block_gs(L, agg, v)
    qn = op.pack(torch.from_numpy(q), qdt)
    qin = op.unpack(qn, n, qdt).cpu().numpy()
    nc = 2 * n
    Dc = torch.full((op.n_agg * 9 * nc * nc * 2,), float("nan"), dtype=torch.float32, device="cuda")
    mrhs.coarse_op_build(op.handle, qn, qdt, n, Dc, op.workspace(n))
    torch.cuda.synchronize()
    got = Dc.cpu().numpy().astype(np.float64).view(np.complex128).reshape(op.n_agg, 9, nc, nc)
    ref = oracle.coarse_op(L, agg, case.U, case.A, qin)
    assert np.all(np.isfinite(got))
    for d in range(9):
        assert rel(got[:, d], ref[:, d]) < 1e-5, (d, rel(got[:, d], ref[:, d]))
    # the self block is sigma3-hermitian (an exact property of the Galerkin operator)
    s3 = np.diag([1.0] * n + [-1.0] * n)
    for i in range(op.n_agg):
        assert rel(s3 @ got[i, 0], got[i, 0].conj().T @ s3) < 1e-5
    op.close()



def test_coarse_needs_no_workspace():
    """coarse_op_build takes no workspace: a null one gives the same D_c bit for bit."""
    need_gpu()
    L, block, agg, n, S = [8, 4, 8, 4], [4, 4, 4, 4], [2, 4, 4, 2], 13, 4
    case = Case(L, 0.3, 311, -0.2)
    announce("coarse without workspace")
    op = case.op(block, agg=agg, prec=F32, short_len=S)
    q = oracle.block_gs(L, agg, inputs.test_vectors(L, n, 312))
    qn = op.pack(torch.from_numpy(q), D32)
    nc = 2 * n
    a = torch.zeros(op.n_agg * 9 * nc * nc * 2, dtype=torch.float32, device="cuda")
    b = torch.full_like(a, float("nan"))
    mrhs.coarse_op_build(op.handle, qn, D32, n, a, op.workspace(n))
    mrhs.coarse_op_build(op.handle, qn, D32, n, b, None)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    op.close()
