"""GPU parity of the layout conversion and the Wilson-clover stencil (dirac_apply_mrhs)
against the FP64 oracle, through the C-ABI."""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import Case, announce, need_gpu, per_rhs_rel
from paper_1601_03184_amd import inputs
from paper_1601_03184_amd import mrhs

pytestmark = pytest.mark.gpu

F64, F32, F16 = mrhs.PREC_F64, mrhs.PREC_F32, mrhs.PREC_F32_F16STORE
TOL = {F64: 1e-13, F32: 1e-6, F16: 2e-3}


@pytest.mark.parametrize("prec,S,n", [(F64, 1, 1), (F64, 4, 6), (F32, 4, 8), (F16, 4, 5), (F32, 8, 3), (F32, 2, 4)])
def test_pack_roundtrip(prec, S, n):
    need_gpu()
    case = Case([4, 4, 4, 4], 0.3, 101, -0.1)
    announce("pack roundtrip prec=%d S=%d n=%d" % (prec, S, n))
    op = case.op([2, 2, 2, 2], prec=prec, short_len=S)
    v = inputs.test_vectors(case.L, n, 102)
    nat = op.pack(torch.from_numpy(v))
    back = op.unpack(nat, n).cpu().numpy()
    if prec == F64:
        assert np.array_equal(back, v)
    elif prec == F32:
        assert np.array_equal(back, v.real.astype(np.float32) + 1j * v.imag.astype(np.float32))
    else:
        assert np.array_equal(back, v.real.astype(np.float16).astype(np.float64)
                              + 1j * v.imag.astype(np.float16).astype(np.float64))
    # padding lanes of the last group are zero
    if n % S:
        full = op.unpack(nat, (n + S - 1) // S * S).cpu().numpy()
        assert np.all(full[n:] == 0)
    op.close()


def test_pack_fp16_range_error():
    need_gpu()
    case = Case([4, 4, 4, 4], 0.3, 101, -0.1)
    op = case.op([2, 2, 2, 2], prec=F16)
    v = inputs.test_vectors(case.L, 2, 103)
    v[1, 7, 2, 1] = 7e4
    announce("pack fp16 overflow")
    with pytest.raises(mrhs.MrhsError) as e:
        op.pack(torch.from_numpy(v))
    assert e.value.code == mrhs.MRHS_ERANGE
    op.close()


DIRAC_CASES = [
    # (L, block, sigma, seed, m0, prec, S, n, tile)
    ([4, 4, 4, 4], [2, 2, 2, 2], 0.3, 101, -0.1, F64, 1, 1, 1),
    ([4, 4, 4, 4], [2, 2, 2, 2], 0.3, 101, -0.1, F64, 4, 8, 1),
    ([8, 4, 4, 8], [4, 4, 4, 4], 0.3, 111, -0.3, F32, 4, 6, 4),
    ([8, 4, 4, 8], [4, 4, 4, 4], 0.3, 111, -0.3, F32, 4, 6, 2),
    ([8, 4, 4, 8], [4, 4, 4, 4], 0.3, 111, -0.3, F32, 4, 6, 1),
    ([12, 4, 8, 4], [4, 4, 4, 4], 0.25, 121, -0.33, F16, 4, 7, 4),
    ([6, 6, 2, 4], [2, 2, 2, 2], 0.3, 131, -0.2, F32, 8, 9, 4),   # odd block counts, ragged
    ([4, 2, 2, 4], [4, 2, 2, 2], 0.3, 141, 0.2, F64, 2, 3, 2),    # a block spans a direction
    # tile 4 on a short length of 4 (two groups per workgroup): 16-site blocks and an odd
    # number of groups, and 24-site blocks (a workgroup of 192 threads)
    ([4, 4, 4, 4], [2, 2, 2, 2], 0.3, 151, -0.2, F32, 4, 11, 4),
    ([4, 4, 4, 6], [2, 2, 2, 3], 0.3, 161, -0.25, F32, 4, 13, 4),
]


@pytest.mark.parametrize("L,block,sigma,seed,m0,prec,S,n,tile", DIRAC_CASES)
def test_dirac_parity(L, block, sigma, seed, m0, prec, S, n, tile):
    need_gpu()
    case = Case(L, sigma, seed, m0)
    announce("dirac L=%s block=%s prec=%d S=%d n=%d tile=%d" % (L, block, prec, S, n, tile))
    op = case.op(block, prec=prec, short_len=S)
    mrhs.mrhs_set_tiles(op.handle, 0, tile)
    v = inputs.test_vectors(L, n, seed + 1)
    x = op.pack(torch.from_numpy(v))
    xin = op.unpack(x, n).cpu().numpy()  # the values the kernel reads
    y = op.empty(n)
    mrhs.dirac_apply_mrhs(op.handle, x, y, n)
    torch.cuda.synchronize()
    got = op.unpack(y, n).cpu().numpy()
    ref = oracle.dirac(L, case.U, case.A, xin)
    err = per_rhs_rel(got, ref)
    assert err < TOL[prec], err
    op.close()


def test_dirac_c2_full_size():
    """16^4, 20 right-hand sides, FP32: every output against the oracle."""
    need_gpu()
    L = [16, 16, 16, 16]
    case = Case(L, 0.3, 201, -0.3)
    announce("dirac c2 full 16^4 n=20 fp32")
    op = case.op([4, 4, 4, 4], prec=F32, short_len=4)
    v = inputs.test_vectors(L, 20, 202)
    x = op.pack(torch.from_numpy(v))
    xin = op.unpack(x, 20).cpu().numpy()
    y = op.empty(20)
    mrhs.dirac_apply_mrhs(op.handle, x, y, 20)
    torch.cuda.synchronize()
    got = op.unpack(y, 20).cpu().numpy()
    ref = oracle.dirac(L, case.U, case.A, xin)
    assert per_rhs_rel(got, ref) < 1e-6
    op.close()


def test_abi_rejects_bad_arguments():
    need_gpu()
    case = Case([4, 4, 4, 4], 0.3, 101, -0.1)
    op = case.op([2, 2, 2, 2], prec=F32)
    x = op.empty(4)
    with pytest.raises(mrhs.MrhsError) as e:
        mrhs.dirac_apply_mrhs(op.handle, x, x, 4)
    assert e.value.code == mrhs.MRHS_EINVAL
    with pytest.raises(mrhs.MrhsError) as e:
        mrhs.dirac_apply_mrhs(op.handle, x, op.empty(4), 0)
    assert e.value.code == mrhs.MRHS_EINVAL
    with pytest.raises(mrhs.MrhsError) as e:
        mrhs.sap_smooth_mrhs(op.handle, x, x, 4, 1, 1, None)
    assert e.value.code == mrhs.MRHS_EINVAL
    with pytest.raises(mrhs.MrhsError) as e:
        mrhs.mrhs_set_tiles(op.handle, 3, 0)
    assert e.value.code == mrhs.MRHS_EINVAL
    # FP64 tiles above 2 are not built (they would spill): refused, the op keeps its tiles
    op64 = case.op([2, 2, 2, 2], prec=F64, short_len=4)
    for sap_tile, dirac_tile in ((4, 0), (0, 4)):
        with pytest.raises(mrhs.MrhsError) as e:
            mrhs.mrhs_set_tiles(op64.handle, sap_tile, dirac_tile)
        assert e.value.code == mrhs.MRHS_EUNSUPPORTED
    op64.close()
    with pytest.raises(mrhs.MrhsError) as e:
        mrhs.Operator([4, 4, 4, 6], [2, 2, 2, 4], [2, 2, 2, 2], torch.from_numpy(inputs.gauge_field([4, 4, 4, 6], 0.3, 1)),
                      0.0, 1.0)
    assert e.value.code == mrhs.MRHS_EINVAL
    op.close()
