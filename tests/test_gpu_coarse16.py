"""The half-precision coarse grid through the C-ABI: D_c stored in binary16
(coarse_op_build_f16), the coarse apply with it (coarse_apply_f16_mrhs) and the coarse
GMRES with D_c and the Krylov basis in binary16 (coarse_solve_f16_mrhs), all with FP32
arithmetic, against the FP64 oracle on the same seeded inputs.

Tolerance: a binary16 entry carries a relative rounding error of at most u = 2^-11
(4.9e-4), so the coarse apply is off by at most u |D_c| |y| entry-wise, which for these
O(1), diagonally dominated blocks is a few u relative per right-hand side; the 5e-3 of
FP16 storage is met with a margin of several.  Against the oracle run on the binary16
values themselves (exact in FP64) only the FP32 arithmetic remains (1e-5)."""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import Case, announce, need_gpu
from paper_1601_03184_amd import inputs
from paper_1601_03184_amd import mrhs
from test_gpu_transfer import coarse_from_native, coarse_to_native, per_rhs_rel

pytestmark = pytest.mark.gpu

F64, F32 = mrhs.PREC_F64, mrhs.PREC_F32
D64, D32 = mrhs.DTYPE_F64, mrhs.DTYPE_F32
U16 = 2.0 ** -11


def setup(L, block, agg, prec, n_tv):
    case = Case(L, 0.3, 341, -0.2)
    op = case.op(block, agg=agg, prec=prec, short_len=4)
    q = oracle.block_gs(L, agg, inputs.test_vectors(L, n_tv, 342))
    qn = op.pack(torch.from_numpy(q), D32)
    qin = op.unpack(qn, n_tv, D32).cpu().numpy()
    Vc, nc = op.n_agg, 2 * n_tv
    Dc = torch.zeros(Vc * 9 * nc * nc * 2, dtype=torch.float32, device="cuda")
    mrhs.coarse_op_build(op.handle, qn, D32, n_tv, Dc, None)
    D16 = torch.full((Vc * 9 * nc * nc * 2,), float("nan"), dtype=torch.float16, device="cuda")
    mrhs.coarse_op_build_f16(op.handle, qn, D32, n_tv, D16)
    torch.cuda.synchronize()
    d32 = Dc.cpu().double().numpy().view(np.complex128).reshape(Vc, 9, nc, nc)
    d16 = D16.cpu().double().numpy().view(np.complex128).reshape(Vc, 9, nc, nc)
    return case, op, qn, qin, Dc, D16, d32, d16


def random_coarse(n, Vc, n_tv, seed):
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((n, Vc, 2, n_tv)) + 1j * rng.standard_normal((n, Vc, 2, n_tv))
    return (z.real.astype(np.float32) + 1j * z.imag.astype(np.float32)).astype(np.complex128)


BUILD_CASES = [
    # (L, block, agg, prec, n_tv)
    ([8, 8, 4, 8], [4, 4, 4, 4], [4, 4, 4, 4], F32, 20),
    ([4, 4, 2, 4], [2, 2, 2, 2], [2, 4, 2, 2], F32, 4),    # coarse extents 2 and 1
    ([4, 4, 4, 4], [2, 2, 2, 2], [2, 2, 2, 2], F32, 32),
    ([4, 4, 4, 8], [2, 2, 2, 2], [2, 2, 2, 4], F64, 12),   # FP64 fields
]


@pytest.mark.parametrize("L,block,agg,prec,n_tv", BUILD_CASES)
def test_coarse_op_build_f16(L, block, agg, prec, n_tv):
    """Every binary16 entry is the FP32 build's entry rounded once (the same sums), and the
    blocks are within the binary16 resolution of the oracle's FP64 D_c."""
    need_gpu()
    announce("coarse op f16 L=%s agg=%s n_tv=%d" % (L, agg, n_tv))
    case, op, qn, qin, Dc, D16, d32, d16 = setup(L, block, agg, prec, n_tv)
    assert torch.equal(Dc.half(), D16)
    ref = oracle.coarse_op(L, agg, case.U, case.A, qin)
    for d in range(9):
        err = np.linalg.norm(d16[:, d] - ref[:, d]) / np.linalg.norm(ref[:, d])
        assert err < 2 * U16, (d, err)
    op.close()


APPLY_CASES = [
    # (L, block, agg, prec, n_tv, n)
    ([8, 8, 4, 8], [4, 4, 4, 4], [4, 4, 4, 4], F32, 20, 13),
    ([4, 4, 2, 4], [2, 2, 2, 2], [2, 4, 2, 2], F32, 4, 3),
    ([4, 4, 4, 4], [2, 2, 2, 2], [2, 2, 2, 2], F32, 32, 32),
]


@pytest.mark.parametrize("L,block,agg,prec,n_tv,n", APPLY_CASES)
def test_coarse_apply_f16_parity(L, block, agg, prec, n_tv, n):
    need_gpu()
    announce("coarse apply f16 L=%s n_tv=%d n=%d" % (L, n_tv, n))
    case, op, qn, qin, Dc, D16, d32, d16 = setup(L, block, agg, prec, n_tv)
    Vc = op.n_agg
    zc = random_coarse(n, Vc, n_tv, 343)
    zn = coarse_to_native(zc, (n + 3) // 4 * 4)
    out = op.coarse_empty(n_tv, n)
    out.fill_(float("nan"))
    mrhs.coarse_apply_f16_mrhs(op.handle, D16, n_tv, zn, out, n)
    got = coarse_from_native(out, Vc, n_tv, n)
    # the binary16 values themselves (exact in FP64): only the FP32 arithmetic differs
    assert per_rhs_rel(got, oracle.coarse_apply(L, agg, d16, zc)) < 1e-5
    # the FP64 operator: within the storage tolerance
    ref = oracle.coarse_apply(L, agg, oracle.coarse_op(L, agg, case.U, case.A, qin), zc)
    assert per_rhs_rel(got, ref) < 5e-3
    with pytest.raises(mrhs.MrhsError):
        mrhs.coarse_apply_f16_mrhs(op.handle, D16, n_tv, zn, zn, n)  # output overlaps input
    op.close()


GMRES_CASES = [
    # (L, block, agg, prec, n_tv, n, m, tol)
    ([8, 8, 4, 8], [4, 4, 4, 4], [4, 4, 4, 4], F32, 20, 13, 10, 0.0),
    ([8, 8, 4, 8], [4, 4, 4, 4], [4, 4, 4, 4], F32, 20, 20, 30, 0.05),
    ([4, 4, 2, 4], [2, 2, 2, 2], [2, 4, 2, 2], F32, 4, 3, 6, 0.0),
    ([4, 4, 4, 4], [2, 2, 2, 2], [2, 2, 2, 2], F32, 32, 32, 4, 0.0),
]


@pytest.mark.parametrize("L,block,agg,prec,n_tv,n,m,tol", GMRES_CASES)
def test_coarse_gmres_f16_parity(L, block, agg, prec, n_tv, n, m, tol):
    """GMRES with D_c and the Krylov basis in binary16 against the oracle's FP64 GMRES on the
    same D_c values: the solutions within the storage tolerance, the residual estimate within
    that tolerance of the true residual of the solution (both relative to ||b||), the stop at
    the oracle's iteration or a neighbouring one (a basis rounded to binary16 moves the
    estimate by about its resolution)."""
    need_gpu()
    announce("coarse gmres f16 L=%s n_tv=%d n=%d m=%d tol=%g" % (L, n_tv, n, m, tol))
    case, op, qn, qin, Dc, D16, d32, d16 = setup(L, block, agg, prec, n_tv)
    Vc = op.n_agg
    bc = random_coarse(n, Vc, n_tv, 344)
    bn = coarse_to_native(bc, (n + 3) // 4 * 4)
    un = op.coarse_empty(n_tv, n)
    un.fill_(float("nan"))
    res = torch.empty(n, dtype=torch.float64, device="cuda")
    its = torch.empty(n, dtype=torch.int32, device="cuda")
    ws = torch.empty(mrhs.mrhs_coarse_solve_f16_workspace_bytes(op.handle, n_tv, n, m), dtype=torch.uint8,
                     device="cuda")
    assert ws.numel() < mrhs.mrhs_coarse_solve_workspace_bytes(op.handle, n_tv, n, m)
    mrhs.coarse_solve_f16_mrhs(op.handle, D16, n_tv, bn, un, n, m, tol, ws, res, its)
    got = coarse_from_native(un, Vc, n_tv, n)
    ref, rref, iref = oracle.coarse_gmres(L, agg, d16, bc, m, tol)
    assert per_rhs_rel(got, ref) < 5e-3
    it = its.cpu().numpy()
    assert np.all(np.abs(it - iref) <= 1), (it, iref)
    r = res.cpu().numpy()
    # the true relative residual of the solution with the binary16 operator
    true = np.linalg.norm((bc - oracle.coarse_apply(L, agg, d16, got)).reshape(n, -1), axis=1) / \
        np.linalg.norm(bc.reshape(n, -1), axis=1)
    assert np.all(np.abs(true - r) <= 5e-3)
    if tol > 0:
        assert np.all(r <= tol)
        assert np.all(true <= tol + 5e-3)
    op.close()


@pytest.mark.parametrize("f16", [False, True])
def test_coarse_solve_graph_replay(f16):
    """The coarse solve enqueues a fixed sequence of launches with no host round trip, so it
    can be captured into a graph: every replay (with eager work and synchronisations between
    the replays) reproduces the eagerly computed solution bit for bit."""
    need_gpu()
    L, block, agg, n_tv, n, m, tol = [8, 8, 4, 8], [4, 4, 4, 4], [4, 4, 4, 4], 20, 13, 8, 0.05
    announce("coarse solve graph replay f16=%d" % f16)
    case, op, qn, qin, Dc, D16, d32, d16 = setup(L, block, agg, F32, n_tv)
    Vc = op.n_agg
    bn = coarse_to_native(random_coarse(n, Vc, n_tv, 345), (n + 3) // 4 * 4)
    wsb = (mrhs.mrhs_coarse_solve_f16_workspace_bytes if f16 else mrhs.mrhs_coarse_solve_workspace_bytes)(
        op.handle, n_tv, n, m)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    un = op.coarse_empty(n_tv, n)

    def solve(stream=None):
        if f16:
            mrhs.coarse_solve_f16_mrhs(op.handle, D16, n_tv, bn, un, n, m, tol, ws, stream=stream)
        else:
            mrhs.coarse_solve_mrhs(op.handle, Dc, n_tv, bn, un, n, m, tol, ws, stream=stream)

    solve()
    torch.cuda.synchronize()
    eager = un.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            solve(stream=s)
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        un.fill_(float("nan"))
        ws.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(un, eager), rep
    op.close()
