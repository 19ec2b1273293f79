"""Plain FP64 CPU oracle of the MRHS DD-alpha-AMG setup path (ctypes wrapper).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
CPU-baseline leg of the benchmark.  The GPU library never imports or calls it,
and the two share no code.  All arrays are numpy complex128 in the canonical
layout: links [4][V][3][3], vectors [n_rhs][V][4][3] (component 3*spin + colour),
site index x0 + L0*(x1 + L1*(x2 + L2*x3)).

Every function cites the passage of the paper (Richtmann, Heybrock, Wettig,
Lattice 2015) it follows; the Wilson-clover operator, SAP and MR are the
standard definitions the paper cites but does not print (readings listed in
oracle.c).
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")


def build(force=False):
    """Compile oracle.c with plain gcc (no intrinsics, no fast-math)."""
    if not force and os.path.exists(_LIB_PATH) and os.path.getmtime(_LIB_PATH) >= os.path.getmtime(_SRC):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp"
    subprocess.check_call(["gcc", "-std=gnu99", "-O2", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"])
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = ctypes.CDLL(_LIB_PATH)
        p, i, d, l = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_long
        sig = {
            "oracle_gamma": (i, [i, p]),
            "oracle_clover": (None, [p, p, d, d, p]),
            "oracle_dirac": (None, [p, p, p, p, p, i]),
            "oracle_block_dirac": (None, [p, p, p, p, p, p, i]),
            "oracle_mr": (None, [p, p, p, p, l, p, i, p, p]),
            "oracle_sap": (i, [p, p, p, p, p, p, i, i, i]),
            "oracle_residual_norms": (None, [p, p, p, p, p, i, p]),
            "oracle_block_gs": (i, [p, p, p, i, p, p]),
            "oracle_restrict": (None, [p, p, p, i, p, p, i]),
            "oracle_prolong": (None, [p, p, p, i, p, p, i]),
            "oracle_coarse_apply": (None, [p, p, p, i, p, p, i]),
            "oracle_sap_from": (i, [p, p, p, p, p, p, i, i, i]),
            "oracle_coarse_gmres": (None, [p, p, p, i, p, p, i, i, ctypes.c_double, p, p]),
            "oracle_coarse_op": (None, [p, p, p, p, p, i, p, p, l]),
            "oracle_eo_block": (i, [p, p, p, p, p, l, p, i, p, p]),
            "oracle_coarse_gmres_eo": (i, [p, p, p, p, i, p, p, i, i, ctypes.c_double, p, p]),
            "oracle_sap_from_eo": (i, [p, p, p, p, p, p, p, i, i, i]),
        }
        for name, (res, args) in sig.items():
            f = getattr(_lib, name)
            f.restype = res
            f.argtypes = args
    return _lib


def _ext(L):
    return np.ascontiguousarray(L, dtype=np.int32)


def _c128(a):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    return a


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def volume(L):
    return int(np.prod(L))


def gamma(mu):
    """g_mu (mu = 0..3, DeGrand-Rossi chiral basis) or g5 = g0 g1 g2 g3 (mu = 4)."""
    out = np.zeros((4, 4), np.complex128)
    if lib().oracle_gamma(mu, _ptr(out)) != 0:
        raise ValueError(mu)
    return out


def clover(L, U, csw, m0):
    """A(x) = (4 + m0) + C(x) per site, [V][12][12] (the Dirac operator of Sec. 2's 12V vectors)."""
    L = _ext(L)
    U = _c128(U)
    A = np.zeros((volume(L), 12, 12), np.complex128)
    lib().oracle_clover(_ptr(L), _ptr(U), float(csw), float(m0), _ptr(A))
    return A


def _vecs(x, L):
    x = _c128(x)
    V = volume(L)
    n = x.size // (12 * V)
    if x.size != n * 12 * V:
        raise ValueError("vector size is not a multiple of 12 V")
    return x, n


def dirac(L, U, A, x):
    """y = D x for a stack of vectors [n][V][4][3]."""
    L = _ext(L)
    x, n = _vecs(x, L)
    y = np.zeros_like(x)
    lib().oracle_dirac(_ptr(L), _ptr(_c128(U)), _ptr(_c128(A)), _ptr(x), _ptr(y), n)
    return y


def block_dirac(L, b, U, A, x):
    """y = sum_j I_j D_j I_j^T x: D with hops between different blocks dropped."""
    L, b = _ext(L), _ext(b)
    x, n = _vecs(x, L)
    y = np.zeros_like(x)
    lib().oracle_block_dirac(_ptr(L), _ptr(b), _ptr(_c128(U)), _ptr(_c128(A)), _ptr(x), _ptr(y), n)
    return y


def mr(L, b, U, A, j, r, n_mr):
    """Minimal residual on block j for one full-lattice residual r: returns (e, ||rho|| history)."""
    L, b = _ext(L), _ext(b)
    r, n = _vecs(r, L)
    assert n == 1
    e = np.zeros_like(r)
    norms = np.zeros(n_mr + 1)
    lib().oracle_mr(_ptr(L), _ptr(b), _ptr(_c128(U)), _ptr(_c128(A)), int(j), _ptr(r), int(n_mr), _ptr(e), _ptr(norms))
    return e, norms


def clover_inverse(A):
    """A(x)^-1 per site, [V][12][12] (numpy's inverse: the even-odd block solver's A_oo^-1)."""
    return np.ascontiguousarray(np.linalg.inv(_c128(A)))


def eo_block(L, b, U, A, j, r, n_mr, Ainv=None):
    """The even-odd block solve of D_j e = r on block j (Schur complement over the block's
    even sites, n_mr MR steps, then the odd sites): returns (e, ||rho_e|| history)."""
    L, b = _ext(L), _ext(b)
    r, n = _vecs(r, L)
    assert n == 1
    if Ainv is None:
        Ainv = clover_inverse(A)
    e = np.zeros_like(r)
    norms = np.zeros(n_mr + 1)
    rc = lib().oracle_eo_block(_ptr(L), _ptr(b), _ptr(_c128(U)), _ptr(_c128(A)), _ptr(_c128(Ainv)), int(j), _ptr(r),
                               int(n_mr), _ptr(e), _ptr(norms))
    if rc != 0:
        raise ValueError("oracle_eo_block: block extents must be even")
    return e, norms


def sap(L, b, U, A, rhs, n_sap, n_mr, x0=None, eo=False, Ainv=None):
    """x = SAP(rhs) per vector, from a zero start (the initial setup phase of Sec. 2) or from
    the starting guess x0 (the refinement phase, Alg. 1 and 2); eo=True: the even-odd block
    solver (eo_block) instead of plain MR."""
    L, b = _ext(L), _ext(b)
    rhs, n = _vecs(rhs, L)
    if eo:
        if Ainv is None:
            Ainv = clover_inverse(A)
        x = np.zeros_like(rhs) if x0 is None else np.array(_c128(x0), copy=True).reshape(rhs.shape)
        rc = lib().oracle_sap_from_eo(_ptr(L), _ptr(b), _ptr(_c128(U)), _ptr(_c128(A)), _ptr(_c128(Ainv)), _ptr(rhs),
                                      _ptr(x), n, int(n_sap), int(n_mr))
        if rc != 0:
            raise ValueError("oracle_sap_from_eo: block extents must be even")
        return x
    if x0 is None:
        x = np.zeros_like(rhs)
        fn = lib().oracle_sap
    else:
        x = np.array(_c128(x0), copy=True).reshape(rhs.shape)
        fn = lib().oracle_sap_from
    rc = fn(_ptr(L), _ptr(b), _ptr(_c128(U)), _ptr(_c128(A)), _ptr(rhs), _ptr(x), n, int(n_sap), int(n_mr))
    if rc != 0:
        raise ValueError("oracle_sap: bad geometry")
    return x


def residual_norms(L, U, A, rhs, x):
    """||b_k - D x_k|| / ||b_k|| per vector."""
    L = _ext(L)
    rhs, n = _vecs(rhs, L)
    x, n2 = _vecs(x, L)
    assert n == n2
    out = np.zeros(n)
    lib().oracle_residual_norms(_ptr(L), _ptr(_c128(U)), _ptr(_c128(A)), _ptr(rhs), _ptr(x), n, _ptr(out))
    return out


def n_aggregates(L, a):
    return volume([L[m] // a[m] for m in range(4)])


def block_gs(L, a, V, return_T=False):
    """Per aggregate and spin half: V^h_i = Q^h_i T^h_i (setup of R, P = R^dag; Sec. 2, Alg. 3).

    Returns Q (same shape as V) [and T [n_agg][2][n_tv][n_tv]]; raises on rank deficiency."""
    L, a = _ext(L), _ext(a)
    V, n_tv = _vecs(V, L)
    Q = np.zeros_like(V)
    T = np.zeros((n_aggregates(L, a), 2, n_tv, n_tv), np.complex128)
    rc = lib().oracle_block_gs(_ptr(L), _ptr(a), _ptr(V), n_tv, _ptr(Q), _ptr(T))
    if rc < 0:
        raise ValueError("oracle_block_gs: bad geometry")
    if rc > 0:
        raise np.linalg.LinAlgError("rank-deficient aggregate half %d" % (rc - 1))
    return (Q, T) if return_T else Q


def restrict(L, a, Q, y):
    """y_c = R y, R = Q^dag per aggregate half (Alg. 3)."""
    L, a = _ext(L), _ext(a)
    Q, n_tv = _vecs(Q, L)
    y, n = _vecs(y, L)
    yc = np.zeros((n, n_aggregates(L, a), 2, n_tv), np.complex128)
    lib().oracle_restrict(_ptr(L), _ptr(a), _ptr(Q), n_tv, _ptr(y), _ptr(yc), n)
    return yc


def prolong(L, a, Q, yc):
    """y = P y_c, P = Q (Sec. 2: P = R^dag)."""
    L, a = _ext(L), _ext(a)
    Q, n_tv = _vecs(Q, L)
    yc = _c128(yc)
    n = yc.size // (n_aggregates(L, a) * 2 * n_tv)
    y = np.zeros((n, volume(L), 4, 3), np.complex128)
    lib().oracle_prolong(_ptr(L), _ptr(a), _ptr(Q), n_tv, _ptr(yc), _ptr(y), n)
    return y


def coarse_apply(L, a, Dc, yc):
    """y_c -> D_c y_c on the coarse lattice from the 9 blocks per coarse site (the operator
    of the coarse solve, Alg. 1); yc [n][Vc][2][n_tv]."""
    L, a = _ext(L), _ext(a)
    Dc = _c128(Dc)
    yc = _c128(yc)
    nc = Dc.shape[-1]
    n = yc.size // (n_aggregates(L, a) * nc)
    out = np.zeros_like(yc)
    lib().oracle_coarse_apply(_ptr(L), _ptr(a), _ptr(Dc), nc // 2, _ptr(yc), _ptr(out), n)
    return out


def coarse_gmres(L, a, Dc, bc, m, tol=0.0):
    """u_c ~ D_c^-1 b_c by GMRES from zero, at most m iterations, per right-hand side stopped
    at residual estimate tol * ||b_c|| (the low-accuracy coarse solve, Alg. 1).
    Returns (u_c, relative residual estimates, iteration counts)."""
    L, a = _ext(L), _ext(a)
    Dc = _c128(Dc)
    bc = _c128(bc)
    nc = Dc.shape[-1]
    n = bc.size // (n_aggregates(L, a) * nc)
    u = np.zeros_like(bc)
    res = np.zeros(n)
    its = np.zeros(n, np.int32)
    lib().oracle_coarse_gmres(_ptr(L), _ptr(a), _ptr(Dc), nc // 2, _ptr(bc), _ptr(u), n, int(m), float(tol), _ptr(res),
                              _ptr(its))
    return u, res, its


def coarse_op(L, a, U, A, Q, agg_list=None):
    """D_c = R D P as 9 blocks per coarse site [self,+x,+y,+z,+t,-x,-y,-z,-t], each
    2 n_tv x 2 n_tv (Sec. 2: coarse-grid operator from the test vectors)."""
    L, a = _ext(L), _ext(a)
    Q, n_tv = _vecs(Q, L)
    nc = 2 * n_tv
    Dc = np.zeros((n_aggregates(L, a), 9, nc, nc), np.complex128)
    if agg_list is None:
        lst, nl = None, 0
    else:
        lst = np.ascontiguousarray(agg_list, dtype=np.int64)
        nl = lst.size
    lib().oracle_coarse_op(_ptr(L), _ptr(a), _ptr(_c128(U)), _ptr(_c128(A)), _ptr(Q), n_tv, _ptr(Dc),
                           None if lst is None else _ptr(lst), nl)
    return Dc


def coarse_self_inverse(Dc):
    """The inverse of every coarse site's self block, [Vc][2N][2N] (numpy's inverse)."""
    Dc = _c128(Dc)
    return np.ascontiguousarray(np.linalg.inv(Dc[:, 0]))


def coarse_gmres_eo(L, a, Dc, bc, m, tol=0.0, Ainv=None):
    """Even-odd preconditioned coarse solve (GMRES on the Schur complement over the even
    coarse sites, then the odd sites): returns (u [n][Vc][2][N], res, iters); res and iters
    refer to the Schur system."""
    L, a = _ext(L), _ext(a)
    Dc = _c128(Dc)
    bc = _c128(bc)
    nc = Dc.shape[-1]
    n = bc.size // (n_aggregates(L, a) * nc)
    N = nc // 2
    if Ainv is None:
        Ainv = coarse_self_inverse(Dc)
    u = np.zeros_like(bc)
    res = np.zeros(n)
    its = np.zeros(n, np.int32)
    rc = lib().oracle_coarse_gmres_eo(_ptr(L), _ptr(a), _ptr(Dc), _ptr(_c128(Ainv)), N, _ptr(bc), _ptr(u), n, int(m),
                                      float(tol), _ptr(res), _ptr(its))
    if rc != 0:
        raise ValueError("oracle_coarse_gmres_eo: coarse extents must be even")
    return u, res, its
