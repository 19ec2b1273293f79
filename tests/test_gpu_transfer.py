"""Parity of the coarse-grid correction's building blocks through the C-ABI: restriction
(Alg. 3), prolongation and the coarse-operator apply, against the oracle on the same
seeded inputs; and the Galerkin property D_c y_c = R D P y_c on the GPU at full size."""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import Case, announce, need_gpu
from paper_1601_03184_amd import inputs
from paper_1601_03184_amd import mrhs

pytestmark = pytest.mark.gpu

F64, F32, F16 = mrhs.PREC_F64, mrhs.PREC_F32, mrhs.PREC_F32_F16STORE
D64, D32, D16 = mrhs.DTYPE_F64, mrhs.DTYPE_F32, mrhs.DTYPE_F16


def per_rhs_rel(got, ref):
    n = ref.shape[0]
    g, r = got.reshape(n, -1), ref.reshape(n, -1)
    return float(np.max(np.linalg.norm(g - r, axis=1) / np.linalg.norm(r, axis=1)))


def coarse_to_native(yc, ldc):
    """canonical complex [n][Vc][2][N] -> FP32 coarse vectors [Vc][2N][2][ldc] (documented layout)"""
    n, Vc, _, N = yc.shape
    t = torch.view_as_real(torch.from_numpy(np.ascontiguousarray(yc))).reshape(n, Vc, 2 * N, 2)
    out = torch.zeros((Vc, 2 * N, 2, ldc), dtype=torch.float32)
    out[..., :n] = t.permute(1, 2, 3, 0).float()
    return out.reshape(-1).cuda()


def coarse_from_native(native, Vc, N, n):
    ldc = (n + 3) // 4 * 4
    t = native.view(Vc, 2 * N, 2, ldc).cpu().double()
    pad = t[..., n:]
    assert torch.all(pad == 0), "coarse padding entries must be zero"
    c = torch.complex(t[:, :, 0, :n], t[:, :, 1, :n])  # [Vc][2N][n]
    return c.permute(2, 0, 1).reshape(n, Vc, 2, N).numpy()


CASES = [
    # (L, block, agg, prec, S, n_tv, n, qdt)
    ([8, 8, 4, 8], [4, 4, 4, 4], [4, 4, 4, 4], F32, 4, 20, 20, D32),
    ([8, 8, 4, 8], [4, 4, 4, 4], [4, 4, 4, 4], F32, 4, 20, 13, D64),
    ([8, 4, 8, 4], [4, 4, 4, 4], [2, 4, 4, 2], F32, 8, 13, 7, D32),     # aggregates != blocks, S = 8
    ([4, 4, 2, 4], [2, 2, 2, 2], [2, 4, 2, 2], F64, 4, 4, 3, D64),      # coarse extents 2 and 1
    ([8, 4, 4, 8], [4, 4, 4, 4], [4, 4, 4, 4], F16, 4, 32, 32, D32),    # FP16 fine vectors
    ([8, 8, 4, 8], [4, 4, 4, 4], [4, 4, 4, 4], F32, 4, 20, 13, D16),    # FP16 storage of Q
    ([8, 4, 4, 8], [4, 4, 4, 4], [4, 4, 4, 4], F16, 4, 32, 32, D16),    # FP16 vectors and Q
]


def _setup(L, block, agg, prec, S, n_tv, qdt):
    case = Case(L, 0.3, 321, -0.2)
    op = case.op(block, agg=agg, prec=prec, short_len=S)
    q = oracle.block_gs(L, agg, inputs.test_vectors(L, n_tv, 322))
    qn = op.pack(torch.from_numpy(q), qdt)
    qin = op.unpack(qn, n_tv, qdt).cpu().numpy()  # the values the kernels read
    return case, op, qn, qin


@pytest.mark.parametrize("L,block,agg,prec,S,n_tv,n,qdt", CASES)
def test_restrict_prolong_parity(L, block, agg, prec, S, n_tv, n, qdt):
    need_gpu()
    announce("restrict/prolong L=%s agg=%s n_tv=%d n=%d" % (L, agg, n_tv, n))
    case, op, qn, qin = _setup(L, block, agg, prec, S, n_tv, qdt)
    Vc = op.n_agg
    ydt = op.dtype
    y = inputs.test_vectors(L, n, 323)
    yn = op.pack(torch.from_numpy(y))
    yin = op.unpack(yn, n).cpu().numpy()
    yc = op.coarse_empty(n_tv, n)
    yc.fill_(float("nan"))
    mrhs.restrict_mrhs(op.handle, qn, qdt, n_tv, yn, ydt, yc, n)
    got = coarse_from_native(yc, Vc, n_tv, n)
    ref = oracle.restrict(L, agg, qin, yin)
    assert per_rhs_rel(got, ref) < 1e-5
    # prolongation of a random coarse vector
    rng = np.random.default_rng(324)
    zc = rng.standard_normal((n, Vc, 2, n_tv)) + 1j * rng.standard_normal((n, Vc, 2, n_tv))
    zc32 = zc.real.astype(np.float32) + 1j * zc.imag.astype(np.float32)
    zn = coarse_to_native(zc32, (n + 3) // 4 * 4)
    out = op.empty(n)
    out.fill_(float("nan"))
    mrhs.prolong_mrhs(op.handle, qn, qdt, n_tv, zn, out, ydt, n)
    got = op.unpack(out, n).cpu().numpy()
    ref = oracle.prolong(L, agg, qin, zc32.astype(np.complex128))
    tol = 5e-3 if ydt == D16 else 1e-5
    assert per_rhs_rel(got, ref) < tol
    # the padding lanes of the last group are written as zero
    full = op.unpack(out, (n + S - 1) // S * S).cpu().numpy()
    assert np.all(full[n:] == 0)
    op.close()


@pytest.mark.parametrize("L,block,agg,prec,S,n_tv,n,qdt", CASES[:4] + CASES[5:6])
def test_coarse_apply_parity(L, block, agg, prec, S, n_tv, n, qdt):
    need_gpu()
    announce("coarse apply L=%s agg=%s n_tv=%d n=%d" % (L, agg, n_tv, n))
    case, op, qn, qin = _setup(L, block, agg, prec, S, n_tv, qdt)
    Vc, nc = op.n_agg, 2 * n_tv
    Dc = torch.zeros(Vc * 9 * nc * nc * 2, dtype=torch.float32, device="cuda")
    mrhs.coarse_op_build(op.handle, qn, qdt, n_tv, Dc, None)
    Dh = Dc.cpu().double().numpy().view(np.complex128).reshape(Vc, 9, nc, nc)
    rng = np.random.default_rng(325)
    zc = rng.standard_normal((n, Vc, 2, n_tv)) + 1j * rng.standard_normal((n, Vc, 2, n_tv))
    zc32 = zc.real.astype(np.float32) + 1j * zc.imag.astype(np.float32)
    zn = coarse_to_native(zc32, (n + 3) // 4 * 4)
    out = op.coarse_empty(n_tv, n)
    out.fill_(float("nan"))
    mrhs.coarse_apply_mrhs(op.handle, Dc, n_tv, zn, out, n)
    got = coarse_from_native(out, Vc, n_tv, n)
    ref = oracle.coarse_apply(L, agg, Dh, zc32.astype(np.complex128))
    assert per_rhs_rel(got, ref) < 1e-5
    with pytest.raises(mrhs.MrhsError):
        mrhs.coarse_apply_mrhs(op.handle, Dc, n_tv, zn, zn, n)  # output overlaps input
    op.close()


def test_galerkin_full_size_16():
    """16^4, 20 test vectors, 20 right-hand sides, FP32: D_c y_c and R D P y_c agree on the
    GPU (a property of the Galerkin operator at any size)."""
    need_gpu()
    L, n_tv, n = [16, 16, 16, 16], 20, 20
    case = Case(L, 0.3, 201, -0.3)
    op = case.op([4, 4, 4, 4], prec=F32, short_len=4)
    announce("galerkin 16^4 n_tv=20")
    v = op.pack(torch.from_numpy(inputs.test_vectors(L, n_tv, 202)))
    x = op.empty(n_tv)
    mrhs.sap_smooth_mrhs(op.handle, v, x, n_tv, 3, 4, op.workspace(n_tv))
    Q = op.empty(n_tv)
    mrhs.block_orthonormalize(op.handle, x, D32, Q, D32, n_tv, None, None)
    Vc, nc = op.n_agg, 2 * n_tv
    Dc = torch.zeros(Vc * 9 * nc * nc * 2, dtype=torch.float32, device="cuda")
    mrhs.coarse_op_build(op.handle, Q, D32, n_tv, Dc, None)
    rng = np.random.default_rng(326)
    zc = rng.standard_normal((n, Vc, 2, n_tv)) + 1j * rng.standard_normal((n, Vc, 2, n_tv))
    zn = coarse_to_native(zc, (n + 3) // 4 * 4)
    a = op.coarse_empty(n_tv, n)
    mrhs.coarse_apply_mrhs(op.handle, Dc, n_tv, zn, a, n)
    p, dp, b = op.empty(n), op.empty(n), op.coarse_empty(n_tv, n)
    mrhs.prolong_mrhs(op.handle, Q, D32, n_tv, zn, p, D32, n)
    mrhs.dirac_apply_mrhs(op.handle, p, dp, n)
    mrhs.restrict_mrhs(op.handle, Q, D32, n_tv, dp, D32, b, n)
    ga, gb = coarse_from_native(a, Vc, n_tv, n), coarse_from_native(b, Vc, n_tv, n)
    assert per_rhs_rel(ga, gb) < 1e-5
    op.close()


GMRES_CASES = [
    # (L, block, agg, prec, S, n_tv, n, m, tol)
    ([8, 8, 4, 8], [4, 4, 4, 4], [4, 4, 4, 4], F32, 4, 20, 13, 10, 0.0),
    ([8, 8, 4, 8], [4, 4, 4, 4], [4, 4, 4, 4], F32, 4, 20, 20, 30, 0.05),
    ([4, 4, 2, 4], [2, 2, 2, 2], [2, 4, 2, 2], F32, 4, 4, 3, 6, 0.0),   # coarse extents 2 and 1
    ([4, 4, 4, 4], [2, 2, 2, 2], [2, 2, 2, 2], F32, 4, 32, 32, 4, 0.0),
]


@pytest.mark.parametrize("L,block,agg,prec,S,n_tv,n,m,tol", GMRES_CASES)
def test_coarse_gmres_parity(L, block, agg, prec, S, n_tv, n, m, tol):
    """The low-accuracy coarse solve (Alg. 1) against the oracle's GMRES on the same D_c."""
    need_gpu()
    announce("coarse gmres L=%s n_tv=%d n=%d m=%d tol=%g" % (L, n_tv, n, m, tol))
    case, op, qn, qin = _setup(L, block, agg, prec, S, n_tv, D32)
    Vc, nc = op.n_agg, 2 * n_tv
    Dc = torch.zeros(Vc * 9 * nc * nc * 2, dtype=torch.float32, device="cuda")
    mrhs.coarse_op_build(op.handle, qn, D32, n_tv, Dc, None)
    Dh = Dc.cpu().double().numpy().view(np.complex128).reshape(Vc, 9, nc, nc)
    rng = np.random.default_rng(334)
    bc = rng.standard_normal((n, Vc, 2, n_tv)) + 1j * rng.standard_normal((n, Vc, 2, n_tv))
    bc32 = (bc.real.astype(np.float32) + 1j * bc.imag.astype(np.float32)).astype(np.complex128)
    bn = coarse_to_native(bc32, (n + 3) // 4 * 4)
    un = op.coarse_empty(n_tv, n)
    un.fill_(float("nan"))
    res = torch.empty(n, dtype=torch.float64, device="cuda")
    its = torch.empty(n, dtype=torch.int32, device="cuda")
    ws = torch.empty(mrhs.mrhs_coarse_solve_workspace_bytes(op.handle, n_tv, n, m), dtype=torch.uint8, device="cuda")
    mrhs.coarse_solve_mrhs(op.handle, Dc, n_tv, bn, un, n, m, tol, ws, res, its)
    got = coarse_from_native(un, Vc, n_tv, n)
    ref, rref, iref = oracle.coarse_gmres(L, agg, Dh, bc32, m, tol)
    assert per_rhs_rel(got, ref) < 1e-5
    assert np.array_equal(its.cpu().numpy(), iref)
    r = res.cpu().numpy()
    assert np.all(np.abs(r - rref) <= 1e-3 * rref + 1e-6)
    if tol > 0:
        assert np.all(r <= tol)
    op.close()


@pytest.mark.parametrize("f16", [False, True])
def test_coarse_gmres_zero_rhs_and_early_stop(f16):
    """Right-hand sides that are zero never iterate (solution 0, 0 iterations, residual 0),
    and with a loose tolerance every other one stops after its first iteration, so the later
    Arnoldi steps of the fixed launch sequence find no right-hand side iterating: the result
    is still the oracle's GMRES, and the solution of a zero right-hand side is exactly zero."""
    need_gpu()
    L, block, agg, n_tv, n, m, tol = [8, 8, 4, 8], [4, 4, 4, 4], [4, 4, 4, 4], 20, 6, 8, 0.9
    announce("coarse gmres zero rhs, tol %g, f16=%d" % (tol, f16))
    case, op, qn, qin = _setup(L, block, agg, F32, 4, n_tv, D32)
    Vc, nc = op.n_agg, 2 * n_tv
    Dc = torch.zeros(Vc * 9 * nc * nc * 2, dtype=torch.float32, device="cuda")
    mrhs.coarse_op_build(op.handle, qn, D32, n_tv, Dc, None)
    D16 = Dc.half()
    Dh = (D16 if f16 else Dc).cpu().double().numpy().view(np.complex128).reshape(Vc, 9, nc, nc)
    rng = np.random.default_rng(336)
    bc = rng.standard_normal((n, Vc, 2, n_tv)) + 1j * rng.standard_normal((n, Vc, 2, n_tv))
    bc[[1, 4]] = 0
    bc32 = (bc.real.astype(np.float32) + 1j * bc.imag.astype(np.float32)).astype(np.complex128)
    bn = coarse_to_native(bc32, (n + 3) // 4 * 4)
    un = op.coarse_empty(n_tv, n)
    un.fill_(float("nan"))
    res = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
    its = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    if f16:
        ws = torch.empty(mrhs.mrhs_coarse_solve_f16_workspace_bytes(op.handle, n_tv, n, m), dtype=torch.uint8,
                         device="cuda")
        mrhs.coarse_solve_f16_mrhs(op.handle, D16, n_tv, bn, un, n, m, tol, ws, res, its)
    else:
        ws = torch.empty(mrhs.mrhs_coarse_solve_workspace_bytes(op.handle, n_tv, n, m), dtype=torch.uint8,
                         device="cuda")
        mrhs.coarse_solve_mrhs(op.handle, Dc, n_tv, bn, un, n, m, tol, ws, res, its)
    got = coarse_from_native(un, Vc, n_tv, n)
    ref, rref, iref = oracle.coarse_gmres(L, agg, Dh, bc32, m, tol)
    it, r = its.cpu().numpy(), res.cpu().numpy()
    assert np.all(got[[1, 4]] == 0)
    assert it[1] == 0 and it[4] == 0 and r[1] == 0 and r[4] == 0
    live = [0, 2, 3, 5]
    assert np.all(it[live] == 1), it
    assert np.array_equal(it, iref)
    assert per_rhs_rel(got[live], ref[live]) < (5e-3 if f16 else 1e-5)
    assert np.all(r[live] <= tol)
    op.close()


EO_GMRES_CASES = [
    # (L, block, agg, prec, S, n_tv, n, m, tol): every coarse extent even
    ([8, 8, 8, 8], [4, 4, 4, 4], [4, 4, 4, 4], F32, 4, 20, 13, 8, 0.0),
    ([8, 8, 8, 8], [4, 4, 4, 4], [4, 4, 4, 4], F32, 4, 20, 20, 30, 0.05),
    ([4, 4, 4, 4], [2, 2, 2, 2], [2, 2, 2, 2], F32, 4, 4, 3, 6, 0.0),
    ([4, 4, 4, 4], [2, 2, 2, 2], [2, 2, 2, 2], F32, 4, 32, 32, 4, 0.0),   # 64 x 64 self blocks
]


@pytest.mark.parametrize("L,block,agg,prec,S,n_tv,n,m,tol", EO_GMRES_CASES)
def test_coarse_gmres_eo_parity(L, block, agg, prec, S, n_tv, n, m, tol):
    """The even-odd preconditioned coarse solve (GMRES on the even-site Schur complement of
    D_c, then the odd sites) and the self-block inverses against the oracle."""
    need_gpu()
    announce("coarse gmres eo L=%s n_tv=%d n=%d m=%d tol=%g" % (L, n_tv, n, m, tol))
    case, op, qn, qin = _setup(L, block, agg, prec, S, n_tv, D32)
    Vc, nc = op.n_agg, 2 * n_tv
    Dc = torch.zeros(Vc * 9 * nc * nc * 2, dtype=torch.float32, device="cuda")
    mrhs.coarse_op_build(op.handle, qn, D32, n_tv, Dc, None)
    Dh = Dc.cpu().double().numpy().view(np.complex128).reshape(Vc, 9, nc, nc)
    Dinv = torch.full((Vc * nc * nc * 2,), float("nan"), dtype=torch.float32, device="cuda")
    st = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    mrhs.coarse_self_invert(op.handle, Dc, n_tv, Dinv, st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    inv = Dinv.cpu().double().numpy().view(np.complex128).reshape(Vc, nc, nc)
    ref_inv = oracle.coarse_self_inverse(Dh)
    assert np.max(np.linalg.norm((inv - ref_inv).reshape(Vc, -1), axis=1) /
                  np.linalg.norm(ref_inv.reshape(Vc, -1), axis=1)) < 1e-5
    rng = np.random.default_rng(335)
    bc = rng.standard_normal((n, Vc, 2, n_tv)) + 1j * rng.standard_normal((n, Vc, 2, n_tv))
    bc32 = (bc.real.astype(np.float32) + 1j * bc.imag.astype(np.float32)).astype(np.complex128)
    bn = coarse_to_native(bc32, (n + 3) // 4 * 4)
    un = op.coarse_empty(n_tv, n)
    un.fill_(float("nan"))
    res = torch.empty(n, dtype=torch.float64, device="cuda")
    its = torch.empty(n, dtype=torch.int32, device="cuda")
    ws = torch.empty(mrhs.mrhs_coarse_solve_eo_workspace_bytes(op.handle, n_tv, n, m), dtype=torch.uint8, device="cuda")
    mrhs.coarse_solve_eo_mrhs(op.handle, Dc, Dinv, n_tv, bn, un, n, m, tol, ws, res, its)
    got = coarse_from_native(un, Vc, n_tv, n)
    ref, rref, iref = oracle.coarse_gmres_eo(L, agg, Dh, bc32, m, tol)
    assert per_rhs_rel(got, ref) < 1e-5
    assert np.array_equal(its.cpu().numpy(), iref)
    r = res.cpu().numpy()
    assert np.all(np.abs(r - rref) <= 1e-3 * rref + 1e-6)
    if tol > 0:
        assert np.all(r <= tol)
    op.close()


def test_coarse_eo_errors():
    """an odd coarse extent is rejected; a singular self block is reported by site"""
    need_gpu()
    announce("coarse eo errors")
    case, op, qn, qin = _setup([8, 8, 4, 8], [4, 4, 4, 4], [4, 4, 4, 4], F32, 4, 4, D32)  # coarse extent 1 in z
    Vc, nc, n = op.n_agg, 8, 2
    Dc = torch.zeros(Vc * 9 * nc * nc * 2, dtype=torch.float32, device="cuda")
    mrhs.coarse_op_build(op.handle, qn, D32, 4, Dc, None)
    Dinv = torch.empty(Vc * nc * nc * 2, dtype=torch.float32, device="cuda")
    bn, un = op.coarse_empty(4, n), op.coarse_empty(4, n)
    ws = torch.empty(mrhs.mrhs_coarse_solve_eo_workspace_bytes(op.handle, 4, n, 2), dtype=torch.uint8, device="cuda")
    with pytest.raises(mrhs.MrhsError) as ei:
        mrhs.coarse_solve_eo_mrhs(op.handle, Dc, Dinv, 4, bn, un, n, 2, 0.0, ws)
    assert ei.value.code == mrhs.MRHS_EUNSUPPORTED
    Dc.view(Vc, 9, -1)[3, 0] = 0.0  # site 3: zero self block
    st = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    mrhs.coarse_self_invert(op.handle, Dc, 4, Dinv, st)
    torch.cuda.synchronize()
    assert int(st.item()) == 4
    assert torch.all(Dinv.view(Vc, -1)[3] == 0)
    op.close()


@pytest.mark.parametrize("prec,qdt", [(F32, D32), (F64, D32), (F32, D16)])
def test_setup_refine_parity(prec, qdt):
    """One refinement pass over all test vectors (Alg. 2, N_b = n_tv) against the oracle's
    composition restrict -> GMRES -> prolong -> SAP from the guess, on the same inputs."""
    need_gpu()
    L, block, n_tv, m = [8, 8, 4, 8], [4, 4, 4, 4], 20, 4
    case = Case(L, 0.3, 341, -0.2)
    announce("setup refine prec=%d qdt=%d" % (prec, qdt))
    op = case.op(block, prec=prec, short_len=4)
    vdt = op.dtype
    b0 = op.pack(torch.from_numpy(inputs.test_vectors(L, n_tv, 342)))
    V = op.empty(n_tv)
    mrhs.sap_smooth_mrhs(op.handle, b0, V, n_tv, 2, 3, op.workspace(n_tv))  # initial phase
    Q = op.empty(n_tv, qdt)
    mrhs.block_orthonormalize(op.handle, V, vdt, Q, qdt, n_tv, None, None)
    nc = 2 * n_tv
    Dc = torch.zeros(op.n_agg * 9 * nc * nc * 2, dtype=torch.float32, device="cuda")
    mrhs.coarse_op_build(op.handle, Q, qdt, n_tv, Dc, None)
    vin = op.unpack(V, n_tv).cpu().numpy()
    qin = op.unpack(Q, n_tv, qdt).cpu().numpy()
    Dh = Dc.cpu().double().numpy().view(np.complex128).reshape(op.n_agg, 9, nc, nc)
    ws = torch.empty(mrhs.mrhs_refine_workspace_bytes(op.handle, n_tv, m), dtype=torch.uint8, device="cuda")
    mrhs.setup_refine_mrhs(op.handle, V, n_tv, Q, qdt, Dc, 3, 4, m, 0.0, ws)
    got = op.unpack(V, n_tv).cpu().numpy()
    vc = oracle.restrict(L, block, qin, vin)
    uc, _, _ = oracle.coarse_gmres(L, block, Dh, vc, m)
    u = oracle.prolong(L, block, qin, uc)
    ref = oracle.sap(L, block, case.U, case.A, vin, 3, 4, x0=u)
    # the coarse-grid correction runs in FP32 whatever the fine precision, so its FP32
    # rounding (relative 1e-7 of u) enters the result; the smoother then contracts it
    assert per_rhs_rel(got, ref) < 1e-5
    op.close()
