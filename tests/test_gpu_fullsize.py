"""Parity at the full sizes of the two large workloads, on sampled outputs.

32^3 x 64 (sigma 0.25, m0 -0.33, 24 test vectors): SAP 3 x 4 with FP16 storage and with
FP32 storage, two sampled right-hand sides against the oracle (right-hand sides are
independent); then FP64 block Gram-Schmidt of the FP16 result on 4^4 aggregates, sampled
aggregates against the oracle run on that aggregate alone (the factorisation of an
aggregate depends only on its own rows).

48^3 x 96 (sigma 0.2, m0 -0.34, 32 test vectors): the whole setup step -- FP32 SAP, FP64
Gram-Schmidt into FP32 Q, D_c -- with a sampled right-hand side of SAP, sampled
aggregates of Q, and all 9 blocks of D_c at a sampled coarse site.  The oracle's D_c of
that site is computed on a 12^4 window of 3^4 aggregates centred on it: every link,
clover term and Q entry the centre aggregate's blocks involve lies inside the window.

32^3 x 64 again with the even-odd block solver: two sampled right-hand sides of SAP against
the oracle's even-odd SAP.

Inputs come from the device generators (seeded; the host generators would take minutes
at these sizes); the test vectors are packed four at a time.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import announce, need_gpu, per_agg_half_rel, per_rhs_rel
from paper_1601_03184_amd import inputs
from paper_1601_03184_amd import mrhs

pytestmark = pytest.mark.gpu

F32, F16 = mrhs.PREC_F32, mrhs.PREC_F32_F16STORE
D64, D32, D16 = mrhs.DTYPE_F64, mrhs.DTYPE_F32, mrhs.DTYPE_F16
S = 4
BLOCK = [4, 4, 4, 4]


def group_view(op, native, g, n_rhs):
    """The native storage of test vectors g*S .. g*S + S - 1 (one contiguous group)."""
    ge = 24 * op.V * S
    return native[g * ge:(g + 1) * ge]


def pack_all(op, native, dtype, L, n, seed):
    for g in range((n + S - 1) // S):
        m = min(S, n - g * S)
        canon = inputs.test_vectors_device(L, m, seed, "cuda", first=g * S)
        mrhs.mrhs_pack(op.handle, torch.view_as_real(canon), group_view(op, native, g, n), dtype, m)
        del canon


def unpack_rhs(op, native, dtype, n, k):
    """canonical complex128 [V][4][3] of right-hand side k, on the host"""
    g, t = divmod(k, S)
    m = min(S, n - g * S)
    out = torch.zeros((m, op.V, 4, 3, 2), dtype=torch.float64, device="cuda")
    mrhs.mrhs_unpack(op.handle, group_view(op, native, g, n), dtype, out, m)
    return torch.view_as_complex(out[t]).cpu().numpy()


def gather_sites(op, native, dtype, n, sites):
    """canonical complex128 [n][len(sites)][4][3] of all right-hand sides at some sites"""
    idx = torch.as_tensor(sites, device="cuda")
    out = []
    for g in range((n + S - 1) // S):
        m = min(S, n - g * S)
        buf = torch.zeros((m, op.V, 4, 3, 2), dtype=torch.float64, device="cuda")
        mrhs.mrhs_unpack(op.handle, group_view(op, native, g, n), dtype, buf, m)
        out.append(torch.view_as_complex(buf[:, idx]).cpu().numpy())
        del buf
    return np.concatenate(out, axis=0)


def agg_site_index(L, a, i, window=1):
    """canonical site indices of aggregate i (local sites lexicographic); with window = 3,
    of the 3^4 aggregates centred on it (window sites lexicographic)."""
    na = [L[m] // a[m] for m in range(4)]
    ac = []
    r = i
    for m in range(4):
        ac.append(r % na[m])
        r //= na[m]
    ext = [window * a[m] for m in range(4)]
    w = np.indices(ext[::-1]).reshape(4, -1)[::-1]  # x fastest
    x = [(w[m] + (ac[m] - (window // 2)) * a[m]) % L[m] for m in range(4)]
    return x[0] + L[0] * (x[1] + L[1] * (x[2] + L[2] * x[3]))


def check_gs_sampled(L, agg, op, vn, vdt, Q, qdt, n, aggs, tol):
    for i in aggs:
        sites = agg_site_index(L, agg, i)
        v = gather_sites(op, vn, vdt, n, sites)
        q = gather_sites(op, Q, qdt, n, sites)
        ref = oracle.block_gs(agg, agg, v)
        err = per_agg_half_rel(q, ref, agg, agg)   # per spin half of the aggregate
        assert err < tol, (i, err)


@pytest.mark.timeout(900)
def test_c3_fp16_storage_sap_and_gs():
    need_gpu()
    L, n, seed_u, seed_v, m0 = [32, 32, 32, 64], 24, 301, 302, -0.33
    announce("full size 32^3x64 n=24: inputs")
    U = inputs.gauge_field_device(L, 0.25, seed_u, "cuda")
    res = {}
    for prec, dt in ((F16, D16), (F32, D32)):
        announce("full size 32^3x64: SAP prec=%d" % prec)
        op = mrhs.Operator(L, BLOCK, BLOCK, U, m0, 1.0, prec=prec, short_len=S)
        b = op.empty(n)
        pack_all(op, b, dt, L, n, seed_v)
        x = op.empty(n)
        mrhs.sap_smooth_mrhs(op.handle, b, x, n, 3, 4, op.workspace(n))
        norms = torch.empty(n, dtype=torch.float64, device="cuda")
        mrhs.mrhs_residual_norms(op.handle, b, x, n, norms, op.workspace(n))
        torch.cuda.synchronize()
        res[prec] = (op, b, x, norms.cpu().numpy())
    Uh = U.cpu().numpy()
    del U
    A = oracle.clover(L, Uh, 1.0, m0)
    for k in (0, n - 1):
        announce("full size 32^3x64: oracle SAP rhs %d" % k)
        bk = inputs.test_vectors_device(L, 1, seed_v, "cuda", first=k).cpu().numpy()
        ref = oracle.sap(L, BLOCK, Uh, A, bk, 3, 4)
        got16 = unpack_rhs(res[F16][0], res[F16][2], D16, n, k)
        got32 = unpack_rhs(res[F32][0], res[F32][2], D32, n, k)
        assert per_rhs_rel(got32[None], ref) < 1e-5
        assert per_rhs_rel(got16[None], ref) < 5e-3
    # both storages leave a residual well below that of the zero start (1)
    assert np.all(res[F16][3] < 0.5) and np.all(res[F32][3] < 0.5)
    del A
    res[F32][0].close()
    op, b, x, _ = res[F16]
    announce("full size 32^3x64: FP64 Gram-Schmidt of the FP16 result")
    Q = op.empty(n, D64)
    status = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    mrhs.block_orthonormalize(op.handle, x, D16, Q, D64, n, status, op.workspace(n))
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    check_gs_sampled(L, BLOCK, op, x, D16, Q, D64, n, (0, 4321, op.n_agg - 1), 1e-11)
    op.close()


@pytest.mark.timeout(900)
def test_c5_full_setup_step():
    need_gpu()
    L, n, seed_u, seed_v, m0 = [48, 48, 48, 96], 32, 501, 502, -0.34
    agg = [4, 4, 4, 4]
    announce("full size 48^3x96 n=32: inputs")
    U = inputs.gauge_field_device(L, 0.2, seed_u, "cuda")
    op = mrhs.Operator(L, BLOCK, agg, U, m0, 1.0, prec=F32, short_len=S)
    b = op.empty(n)
    pack_all(op, b, D32, L, n, seed_v)
    x = op.empty(n)
    announce("full size 48^3x96: SAP")
    mrhs.sap_smooth_mrhs(op.handle, b, x, n, 3, 4, op.workspace(n))
    announce("full size 48^3x96: Gram-Schmidt")
    Q = op.empty(n, D32)
    status = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    mrhs.block_orthonormalize(op.handle, x, D32, Q, D32, n, status, None)
    announce("full size 48^3x96: D_c")
    nc = 2 * n
    Dc = torch.full((op.n_agg * 9 * nc * nc * 2,), float("nan"), dtype=torch.float32, device="cuda")
    mrhs.coarse_op_build(op.handle, Q, D32, n, Dc, None)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    Uh = U.cpu().numpy()
    del U
    del b
    A = oracle.clover(L, Uh, 1.0, m0)
    for k in (n - 1,):  # one sampled vector: the oracle takes about two minutes per vector here
        announce("full size 48^3x96: oracle SAP rhs %d" % k)
        bk = inputs.test_vectors_device(L, 1, seed_v, "cuda", first=k).cpu().numpy()
        ref = oracle.sap(L, BLOCK, Uh, A, bk, 3, 4)
        assert per_rhs_rel(unpack_rhs(op, x, D32, n, k)[None], ref) < 1e-5
        del ref, bk
    del A
    announce("full size 48^3x96: sampled aggregates")
    check_gs_sampled(L, agg, op, x, D32, Q, D32, n, (0, op.n_agg - 1), 1e-6)
    i = 12345
    sites = agg_site_index(L, agg, i, window=3)
    Lw = [3 * a for a in agg]
    Uw = np.ascontiguousarray(Uh[:, sites])
    Aw = oracle.clover(Lw, Uw, 1.0, m0)
    qw = gather_sites(op, Q, D32, n, sites)
    centre = 1 + 3 * (1 + 3 * (1 + 3 * 1))
    ref = oracle.coarse_op(Lw, agg, Uw, Aw, qw, agg_list=[centre])[centre]
    got = Dc.view(op.n_agg, 9, nc, nc, 2)[i].double().cpu().numpy()
    got = got[..., 0] + 1j * got[..., 1]
    assert np.all(np.isfinite(got))
    for d in range(9):
        err = float(np.linalg.norm(got[d] - ref[d]) / np.linalg.norm(ref[d]))
        assert err < 1e-5, (d, err)
    announce("full size 48^3x96: every coarse site")
    check_dc_all_sites(op, Q, Dc, n)
    op.close()


def check_dc_all_sites(op, Q, Dc, n_tv, n=4, seed=531):
    """Properties of D_c that hold at every coarse site, checked on the whole lattice:
    every self block is sigma3-hermitian (sigma3 = diag(1, -1) over the spin halves:
    gamma5-hermiticity of D carried to the coarse grid), and D_c y_c = R D P y_c for random
    coarse vectors y_c (the Galerkin operator, Sec. 2), with R, D and P applied by the
    library's restriction, stencil and prolongation."""
    nc = 2 * n_tv
    A = torch.view_as_complex(Dc.view(op.n_agg, 9, nc, nc, 2)[:, 0])
    s3 = torch.ones(nc, dtype=torch.float32, device="cuda")
    s3[n_tv:] = -1
    herm = s3[:, None] * A.conj().transpose(-1, -2) * s3[None, :]
    e = ((A - herm).abs().pow(2).sum((-1, -2)) / A.abs().pow(2).sum((-1, -2))).sqrt()
    assert bool(torch.isfinite(e).all())
    assert float(e.max()) < 1e-5, float(e.max())
    del herm, e
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    ldc = (n + 3) // 4 * 4
    zc = op.coarse_empty(n_tv, n)
    zv = zc.view(-1, ldc)
    zv[:, :n] = torch.randn((zv.shape[0], n), generator=gen, device="cuda")
    a = op.coarse_empty(n_tv, n)
    mrhs.coarse_apply_mrhs(op.handle, Dc, n_tv, zc, a, n)
    p, dp = op.empty(n, D32), op.empty(n, D32)
    b = op.coarse_empty(n_tv, n)
    mrhs.prolong_mrhs(op.handle, Q, D32, n_tv, zc, p, D32, n)
    mrhs.dirac_apply_mrhs(op.handle, p, dp, n)
    mrhs.restrict_mrhs(op.handle, Q, D32, n_tv, dp, D32, b, n)
    av, bv = a.view(-1, ldc)[:, :n].double(), b.view(-1, ldc)[:, :n].double()
    err = ((av - bv).pow(2).sum(0).sqrt() / bv.pow(2).sum(0).sqrt()).max()
    assert float(err) < 1e-5, float(err)


@pytest.mark.timeout(900)
def test_c3_even_odd_sap_sampled():
    """32^3 x 64, 24 test vectors, SAP 3 x 4 with the even-odd block solver in FP32: two
    sampled right-hand sides against the oracle's even-odd SAP"""
    need_gpu()
    L, n, seed_u, seed_v, m0 = [32, 32, 32, 64], 24, 301, 302, -0.33
    announce("full size 32^3x64 n=24: even-odd SAP")
    U = inputs.gauge_field_device(L, 0.25, seed_u, "cuda")
    op = mrhs.Operator(L, BLOCK, BLOCK, U, m0, 1.0, prec=F32, short_len=S)
    mrhs.mrhs_set_block_solver(op.handle, mrhs.BLOCK_EO_MR)
    b = op.empty(n)
    pack_all(op, b, D32, L, n, seed_v)
    x = op.empty(n)
    mrhs.sap_smooth_mrhs(op.handle, b, x, n, 3, 4, op.workspace(n))
    torch.cuda.synchronize()
    Uh = U.cpu().numpy()
    del U
    A = oracle.clover(L, Uh, 1.0, m0)
    Ainv = oracle.clover_inverse(A)
    for k in (0, n - 1):
        announce("full size 32^3x64: oracle even-odd SAP rhs %d" % k)
        bk = inputs.test_vectors_device(L, 1, seed_v, "cuda", first=k).cpu().numpy()
        ref = oracle.sap(L, BLOCK, Uh, A, bk, 3, 4, eo=True, Ainv=Ainv)
        assert per_rhs_rel(unpack_rhs(op, x, D32, n, k)[None], ref) < 1e-5
    op.close()
