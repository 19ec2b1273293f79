"""Pins of the oracle's even-odd preconditioned coarse solve (GMRES on the Schur complement
over the even coarse sites, then the odd sites).  CPU only.

The references split the dense coarse matrix (assembled from the 9 blocks per site, pinned
to R D P in test_oracle_coarse) by the parity of the coarse coordinate sum and use plain
dense linear algebra for the Schur complement, its right-hand side and the odd sites."""
import numpy as np
import pytest

import oracle
from oracle_helpers import coarse_dense, rel
from test_oracle_coarse import _coarse_problem

L4, A2, LC = [4, 4, 4, 4], [2, 2, 2, 2], [2, 2, 2, 2]


@pytest.fixture(scope="module")
def problem():
    n_tv, n = 2, 3
    Dc, bc = _coarse_problem(L4, A2, n_tv, n, 611)
    M = coarse_dense(LC, Dc)
    nc = 2 * n_tv
    Vc = Dc.shape[0]
    c = np.array(np.unravel_index(np.arange(Vc), LC[::-1])[::-1]).T
    par = c.sum(axis=1) % 2
    ev = np.concatenate([np.arange(nc) + nc * i for i in range(Vc) if par[i] == 0])
    od = np.concatenate([np.arange(nc) + nc * i for i in range(Vc) if par[i] == 1])
    return Dc, bc, M, ev, od


def _schur(M, ev, od):
    Mee, Meo, Moe, Moo = M[np.ix_(ev, ev)], M[np.ix_(ev, od)], M[np.ix_(od, ev)], M[np.ix_(od, od)]
    return Mee - Meo @ np.linalg.solve(Moo, Moe), Meo, Moe, Moo


def test_coarse_parity_structure(problem):
    """each hop block joins opposite parities: the same-parity parts of D_c are the self blocks"""
    Dc, _, M, ev, od = problem
    nc = Dc.shape[-1]
    for idx in (ev, od):
        sub = M[np.ix_(idx, idx)]
        blockdiag = np.zeros_like(sub)
        for s in range(len(idx) // nc):
            sl = slice(s * nc, (s + 1) * nc)
            blockdiag[sl, sl] = sub[sl, sl]
        assert np.array_equal(sub, blockdiag)


def test_coarse_eo_exact(problem):
    """with as many iterations as Schur unknowns the even-odd solve is exact: u = D_c^-1 b"""
    Dc, bc, M, ev, od = problem
    n = bc.shape[0]
    u, res, its = oracle.coarse_gmres_eo(L4, A2, Dc, bc, m=len(ev))
    exact = np.linalg.solve(M, bc.reshape(n, -1).T).T.reshape(bc.shape)
    assert rel(u, exact) < 1e-10
    assert np.all(res < 1e-10)


def test_coarse_eo_one_step_and_residual(problem):
    """one iteration: u_e = alpha bhat (minimal residual on S), u_o = D_oo^-1 (b_o - D_oe u_e);
    the residual estimate equals the true Schur residual ||bhat - S u_e|| / ||bhat||"""
    Dc, bc, M, ev, od = problem
    n = bc.shape[0]
    S, Meo, Moe, Moo = _schur(M, ev, od)
    u1, _, its1 = oracle.coarse_gmres_eo(L4, A2, Dc, bc, m=1)
    assert np.all(its1 == 1)
    for k in range(n):
        b = bc[k].reshape(-1)
        bh = b[ev] - Meo @ np.linalg.solve(Moo, b[od])
        sb = S @ bh
        alpha = np.vdot(sb, bh) / np.vdot(sb, sb)
        ue = alpha * bh
        uo = np.linalg.solve(Moo, b[od] - Moe @ ue)
        got = u1[k].reshape(-1)
        assert rel(got[ev], ue) < 1e-12 and rel(got[od], uo) < 1e-12
    for m in (2, 3, 5):
        u, res, _ = oracle.coarse_gmres_eo(L4, A2, Dc, bc, m=m)
        for k in range(n):
            b = bc[k].reshape(-1)
            bh = b[ev] - Meo @ np.linalg.solve(Moo, b[od])
            ue = u[k].reshape(-1)[ev]
            true = np.linalg.norm(bh - S @ ue) / np.linalg.norm(bh)
            assert abs(true - res[k]) < 1e-10 * true + 1e-14
            # the full residual of D_c u equals the Schur residual on the even sites (odd sites exact)
            full = b - M @ u[k].reshape(-1)
            assert np.linalg.norm(full[od]) < 1e-11 * np.linalg.norm(b)
            assert abs(np.linalg.norm(full[ev]) - np.linalg.norm(bh - S @ ue)) < 1e-11 * np.linalg.norm(b)


def test_coarse_eo_tolerance_and_odd_extent(problem):
    Dc, bc, M, ev, od = problem
    u, res, its = oracle.coarse_gmres_eo(L4, A2, Dc, bc, m=20, tol=0.3)
    for k in range(bc.shape[0]):
        assert res[k] <= 0.3
        if its[k] > 1:
            _, r_prev, _ = oracle.coarse_gmres_eo(L4, A2, Dc, bc[k:k + 1], m=int(its[k]) - 1)
            assert r_prev[0] > 0.3
    L, a = [6, 4, 4, 4], [2, 2, 2, 2]
    Dc2, bc2 = _coarse_problem(L, a, 2, 1, 621)
    with pytest.raises(ValueError):
        oracle.coarse_gmres_eo(L, a, Dc2, bc2, m=2)
