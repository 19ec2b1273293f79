"""The coarse apply on a coarse lattice of 8^4 sites (16^4 fine sites, 2^4 aggregates), large
enough that the library takes one workgroup per coarse site (the kernel used at 48^3x96),
against the oracle: FP32 and binary16 D_c, n_tv 32, 20 and 5, and the coarse solves (plain and
even-odd GMRES, FP32 and half precision) that are built on it.  D_c is random here (the apply
does not depend on where its blocks come from), with the self blocks made diagonally
dominant so that the even-odd solve's self-block inverses are well conditioned.

Tolerances: FP32 arithmetic on O(1) entries with sums of 9 x 2N terms, 1e-5 relative per
right-hand side; against the oracle on the binary16 values themselves the same."""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import Case, announce, need_gpu
from paper_1601_03184_amd import mrhs
from test_gpu_transfer import coarse_from_native, coarse_to_native, per_rhs_rel

pytestmark = pytest.mark.gpu

F32 = mrhs.PREC_F32
L, BLOCK, AGG = [16, 16, 16, 16], [4, 4, 4, 4], [2, 2, 2, 2]


def make_op():
    return Case(L, 0.3, 351, -0.2).op(BLOCK, agg=AGG, prec=F32, short_len=4)


def random_dc(Vc, N, seed):
    """complex64-representable D_c [Vc][9][2N][2N]: Gaussian blocks / sqrt(2N), self + 4 I"""
    rng = np.random.default_rng(seed)
    n2 = 2 * N
    d = (rng.standard_normal((Vc, 9, n2, n2)) + 1j * rng.standard_normal((Vc, 9, n2, n2))) / np.sqrt(n2)
    d[:, 0] += 4.0 * np.eye(n2)
    d = d.real.astype(np.float32) + 1j * d.imag.astype(np.float32)
    t = torch.from_numpy(np.ascontiguousarray(d.astype(np.complex64)).view(np.float32).reshape(-1)).cuda()
    return d.astype(np.complex128), t


def random_coarse(n, Vc, N, seed):
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((n, Vc, 2, N)) + 1j * rng.standard_normal((n, Vc, 2, N))
    return (z.real.astype(np.float32) + 1j * z.imag.astype(np.float32)).astype(np.complex128)


@pytest.mark.parametrize("n_tv,n", [(32, 32), (20, 13), (5, 1)])
@pytest.mark.parametrize("f16", [False, True])
def test_coarse_apply_per_site_kernel(n_tv, n, f16):
    need_gpu()
    announce("coarse apply 8^4 coarse sites n_tv=%d n=%d f16=%d" % (n_tv, n, f16))
    op = make_op()
    Vc = op.n_agg
    assert Vc == 4096
    dh, dt = random_dc(Vc, n_tv, 352)
    if f16:
        d16 = dt.half()
        dh = d16.cpu().double().numpy().view(np.complex128).reshape(Vc, 9, 2 * n_tv, 2 * n_tv)
    zc = random_coarse(n, Vc, n_tv, 353)
    zn = coarse_to_native(zc, (n + 3) // 4 * 4)
    out = op.coarse_empty(n_tv, n)
    out.fill_(float("nan"))
    if f16:
        mrhs.coarse_apply_f16_mrhs(op.handle, d16, n_tv, zn, out, n)
    else:
        mrhs.coarse_apply_mrhs(op.handle, dt, n_tv, zn, out, n)
    got = coarse_from_native(out, Vc, n_tv, n)
    assert per_rhs_rel(got, oracle.coarse_apply(L, AGG, dh, zc)) < 1e-5
    op.close()


@pytest.mark.parametrize("kind", ["f32", "f16", "eo"])
def test_coarse_solves_per_site_kernel(kind):
    """GMRES with m iterations (tol 0: every right-hand side takes all of them) against the
    oracle's GMRES on the same D_c values."""
    need_gpu()
    n_tv, n, m = 8, 5, 6
    announce("coarse solve 8^4 coarse sites kind=%s" % kind)
    op = make_op()
    Vc = op.n_agg
    dh, dt = random_dc(Vc, n_tv, 354)
    bc = random_coarse(n, Vc, n_tv, 355)
    bn = coarse_to_native(bc, (n + 3) // 4 * 4)
    un = op.coarse_empty(n_tv, n)
    un.fill_(float("nan"))
    res = torch.empty(n, dtype=torch.float64, device="cuda")
    its = torch.empty(n, dtype=torch.int32, device="cuda")
    if kind == "f32":
        ws = torch.empty(mrhs.mrhs_coarse_solve_workspace_bytes(op.handle, n_tv, n, m), dtype=torch.uint8,
                         device="cuda")
        mrhs.coarse_solve_mrhs(op.handle, dt, n_tv, bn, un, n, m, 0.0, ws, res, its)
        ref, rref, iref = oracle.coarse_gmres(L, AGG, dh, bc, m, 0.0)
        tol = 1e-5
    elif kind == "f16":
        d16 = dt.half()
        dh = d16.cpu().double().numpy().view(np.complex128).reshape(Vc, 9, 2 * n_tv, 2 * n_tv)
        ws = torch.empty(mrhs.mrhs_coarse_solve_f16_workspace_bytes(op.handle, n_tv, n, m), dtype=torch.uint8,
                         device="cuda")
        mrhs.coarse_solve_f16_mrhs(op.handle, d16, n_tv, bn, un, n, m, 0.0, ws, res, its)
        ref, rref, iref = oracle.coarse_gmres(L, AGG, dh, bc, m, 0.0)
        tol = 5e-3  # the Krylov basis stored in binary16
    else:
        Dinv = torch.empty(Vc * (2 * n_tv) ** 2 * 2, dtype=torch.float32, device="cuda")
        st = torch.full((1,), -7, dtype=torch.int32, device="cuda")
        mrhs.coarse_self_invert(op.handle, dt, n_tv, Dinv, st)
        torch.cuda.synchronize()
        assert int(st.item()) == 0
        ws = torch.empty(mrhs.mrhs_coarse_solve_eo_workspace_bytes(op.handle, n_tv, n, m), dtype=torch.uint8,
                         device="cuda")
        mrhs.coarse_solve_eo_mrhs(op.handle, dt, Dinv, n_tv, bn, un, n, m, 0.0, ws, res, its)
        ref, rref, iref = oracle.coarse_gmres_eo(L, AGG, dh, bc, m, 0.0)
        tol = 1e-5
    got = coarse_from_native(un, Vc, n_tv, n)
    assert per_rhs_rel(got, ref) < tol
    assert np.array_equal(its.cpu().numpy(), iref)
    op.close()
