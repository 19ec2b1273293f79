"""GPU parity of the MRHS Schwarz smoother (sap_smooth_mrhs) and the FP64 residual check
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
TOL = {F64: 1e-12, F32: 1e-5, F16: 5e-3}


def run_sap(op, v, n_sap, n_mr):
    n = v.shape[0]
    b = op.pack(torch.from_numpy(v))
    x = op.empty(n)
    ws = op.workspace(n)
    mrhs.sap_smooth_mrhs(op.handle, b, x, n, n_sap, n_mr, ws)
    torch.cuda.synchronize()
    return b, x, op.unpack(x, n).cpu().numpy()


SAP_CASES = [
    # (L, block, sigma, seed, m0, prec, S, n, n_sap, n_mr, tile)
    ([4, 4, 4, 4], [2, 2, 2, 2], 0.3, 101, -0.1, F64, 4, 8, 2, 3, 1),   # the 4^4 complex128 workload
    ([4, 4, 4, 4], [2, 2, 2, 2], 0.3, 101, -0.1, F64, 1, 1, 2, 3, 1),
    ([8, 8, 4, 8], [4, 4, 4, 4], 0.3, 211, -0.3, F32, 4, 20, 3, 4, 4),
    ([8, 8, 4, 8], [4, 4, 4, 4], 0.3, 211, -0.3, F32, 4, 20, 3, 4, 2),
    ([8, 8, 4, 8], [4, 4, 4, 4], 0.3, 211, -0.3, F32, 4, 20, 3, 4, 1),
    ([8, 8, 4, 8], [4, 4, 4, 4], 0.25, 311, -0.33, F16, 4, 6, 3, 4, 4),
    ([12, 12, 4, 4], [4, 4, 4, 4], 0.3, 401, -0.3, F32, 4, 8, 3, 4, 4),  # 3 blocks per direction
    ([6, 6, 2, 2], [2, 2, 2, 2], 0.3, 151, -0.2, F64, 2, 3, 2, 5, 2),     # odd counts, same-colour wrap
    ([2, 2, 2, 4], [2, 2, 2, 4], 0.3, 161, 0.2, F64, 1, 1, 1, 20, 1),     # one block spans the lattice
    ([8, 4, 4, 4], [4, 4, 4, 4], 0.3, 171, -0.1, F32, 4, 5, 1, 0, 4),     # n_mr = 0
    ([8, 4, 4, 4], [4, 4, 4, 4], 0.3, 171, -0.1, F32, 4, 5, 0, 3, 4),     # n_sap = 0
]


@pytest.mark.parametrize("L,block,sigma,seed,m0,prec,S,n,n_sap,n_mr,tile", SAP_CASES)
def test_sap_parity(L, block, sigma, seed, m0, prec, S, n, n_sap, n_mr, tile):
    need_gpu()
    case = Case(L, sigma, seed, m0)
    announce("sap L=%s block=%s prec=%d S=%d n=%d %dx%d tile=%d" % (L, block, prec, S, n, n_sap, n_mr, tile))
    op = case.op(block, prec=prec, short_len=S)
    mrhs.mrhs_set_tiles(op.handle, tile, 0)
    v = inputs.test_vectors(L, n, seed + 1)
    _, _, got = run_sap(op, v, n_sap, n_mr)
    ref = oracle.sap(L, block, case.U, case.A, v, n_sap, n_mr)
    if n_sap == 0 or n_mr == 0:
        assert np.all(got == 0) and np.all(ref == 0)
    else:
        err = per_rhs_rel(got, ref)
        assert err < TOL[prec], err
    op.close()


def test_sap_padding_lanes_stay_zero():
    """n_rhs not a multiple of S: the zero padding right-hand sides give alpha = 0, not NaN."""
    need_gpu()
    case = Case([8, 4, 4, 4], 0.3, 171, -0.1)
    op = case.op([4, 4, 4, 4], prec=F32, short_len=4)
    v = inputs.test_vectors(case.L, 5, 172)
    announce("sap padding lanes")
    _, x, got = run_sap(op, v, 2, 3)
    full = op.unpack(x, 8).cpu().numpy()
    assert np.all(full[5:] == 0)
    assert np.all(np.isfinite(got))
    op.close()


def test_sap_mrhs_equals_looped_srhs():
    """The MRHS result equals a loop of single-RHS calls (same kernels, T = S = 1)."""
    need_gpu()
    L = [8, 8, 4, 8]
    case = Case(L, 0.3, 211, -0.3)
    v = inputs.test_vectors(L, 8, 212)
    announce("sap mrhs vs srhs fp64")
    opm = case.op([4, 4, 4, 4], prec=F64, short_len=4)
    mrhs.mrhs_set_tiles(opm.handle, 2, 0)
    _, _, xm = run_sap(opm, v, 3, 4)
    ops = case.op([4, 4, 4, 4], prec=F64, short_len=1)
    xs = np.concatenate([run_sap(ops, v[k:k + 1], 3, 4)[2] for k in range(8)])
    assert per_rhs_rel(xm, xs) < 1e-13
    opm.close()
    ops.close()


@pytest.mark.parametrize("prec", [F64, F32, F16])
def test_residual_norms(prec):
    need_gpu()
    L = [8, 4, 4, 8]
    case = Case(L, 0.3, 221, -0.3)
    op = case.op([4, 4, 4, 4], prec=prec, short_len=4)
    v = inputs.test_vectors(L, 6, 222)
    announce("residual prec=%d" % prec)
    b, x, got = run_sap(op, v, 2, 3)
    out = torch.empty(6, dtype=torch.float64, device="cuda")
    mrhs.mrhs_residual_norms(op.handle, b, x, 6, out, op.workspace(6))
    torch.cuda.synchronize()
    bin_ = op.unpack(b, 6).cpu().numpy()
    ref = oracle.residual_norms(L, case.U, case.A, bin_, got)
    assert np.max(np.abs(out.cpu().numpy() - ref) / ref) < 1e-12
    assert np.all(ref < 0.5)
    op.close()


def test_sap_c2_full_size_sampled():
    """16^4, 20 right-hand sides, 3 x 4, FP32 in the launch configuration of the benchmark;
    right-hand sides are independent, so two sampled ones are checked against the oracle."""
    need_gpu()
    L = [16, 16, 16, 16]
    case = Case(L, 0.3, 201, -0.3)
    op = case.op([4, 4, 4, 4], prec=F32, short_len=4)
    v = inputs.test_vectors(L, 20, 202)
    announce("sap c2 full 16^4 n=20 fp32")
    _, _, got = run_sap(op, v, 3, 4)
    for k in (0, 13):
        ref = oracle.sap(L, [4, 4, 4, 4], case.U, case.A, v[k:k + 1], 3, 4)
        assert per_rhs_rel(got[k:k + 1], ref) < 1e-5
    op.close()


GUESS_CASES = [
    # (L, block, sigma, seed, m0, prec, S, n, n_sap, n_mr, tile)
    ([4, 4, 4, 4], [2, 2, 2, 2], 0.3, 101, -0.1, F64, 4, 8, 2, 3, 1),
    ([8, 8, 4, 8], [4, 4, 4, 4], 0.3, 211, -0.3, F32, 4, 20, 3, 4, 2),
    ([8, 8, 4, 8], [4, 4, 4, 4], 0.25, 311, -0.33, F16, 4, 6, 3, 4, 4),
    ([6, 6, 2, 2], [2, 2, 2, 2], 0.3, 151, -0.2, F64, 2, 3, 2, 5, 2),     # odd counts: snapshot path
    ([8, 4, 4, 4], [4, 4, 4, 4], 0.3, 171, -0.1, F32, 4, 5, 0, 3, 4),     # n_sap = 0 keeps the guess
]


@pytest.mark.parametrize("L,block,sigma,seed,m0,prec,S,n,n_sap,n_mr,tile", GUESS_CASES)
def test_sap_from_guess_parity(L, block, sigma, seed, m0, prec, S, n, n_sap, n_mr, tile):
    """SAP started from a given x (the refinement phase, Alg. 1 and 2) against the oracle."""
    need_gpu()
    case = Case(L, sigma, seed, m0)
    announce("sap from guess L=%s prec=%d n=%d %dx%d" % (L, prec, n, n_sap, n_mr))
    op = case.op(block, prec=prec, short_len=S)
    mrhs.mrhs_set_tiles(op.handle, tile, 0)
    v = inputs.test_vectors(L, n, seed + 1)
    x0 = 0.3 * inputs.test_vectors(L, n, seed + 2)
    b = op.pack(torch.from_numpy(v))
    x = op.pack(torch.from_numpy(x0))
    x0_read = op.unpack(x, n).cpu().numpy()  # the guess in the storage precision
    mrhs.sap_smooth_mrhs_guess(op.handle, b, x, n, n_sap, n_mr, op.workspace(n))
    got = op.unpack(x, n).cpu().numpy()
    if n_sap == 0:
        assert np.array_equal(got, x0_read)
    else:
        ref = oracle.sap(L, block, case.U, case.A, v, n_sap, n_mr, x0=x0_read)
        assert per_rhs_rel(got, ref) < TOL[prec]
    # from a zero guess the result is the initial-phase SAP, bit for bit
    xz = op.empty(n)
    xz.zero_()
    mrhs.sap_smooth_mrhs_guess(op.handle, b, xz, n, n_sap, n_mr, op.workspace(n))
    _, _, plain = run_sap(op, v, n_sap, n_mr)
    assert np.array_equal(op.unpack(xz, n).cpu().numpy(), plain)
    op.close()
