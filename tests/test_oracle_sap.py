"""Pins of the oracle's minimal-residual block solver and Schwarz alternating procedure
(the smoother of the initial setup phase, Sec. 2).  CPU only."""
import numpy as np
import pytest

import oracle
from paper_1601_03184_amd import inputs
from oracle_helpers import colour_rotate, gauge_rotate_links, rel, shift_field, shift_vectors

L4 = [4, 4, 4, 4]
B2 = [2, 2, 2, 2]


@pytest.fixture(scope="module")
def field():
    U = inputs.gauge_field(L4, 0.3, 101)
    A = oracle.clover(L4, U, 1.0, -0.1)
    return U, A


def _block_mask(L, b, j):
    c = inputs.site_coords(L)
    nb = [L[m] // b[m] for m in range(4)]
    bc = c // np.array(b)
    bid = bc[:, 0] + nb[0] * (bc[:, 1] + nb[1] * (bc[:, 2] + nb[2] * bc[:, 3]))
    return bid == j


def _dense_block_ops(L, b, U, A):
    """Dense D_j for every block, from block_dirac on unit vectors placed at the same
    local site of every block at once (blocks decouple in the block operator)."""
    V = inputs.volume(L)
    Vb = int(np.prod(b))
    c = inputs.site_coords(L)
    loc = c % np.array(b)
    lidx = loc[:, 0] + b[0] * (loc[:, 1] + b[1] * (loc[:, 2] + b[2] * loc[:, 3]))
    nb = [L[m] // b[m] for m in range(4)]
    bc = c // np.array(b)
    bid = bc[:, 0] + nb[0] * (bc[:, 1] + nb[1] * (bc[:, 2] + nb[2] * bc[:, 3]))
    nblk = int(np.prod(nb))
    src = np.zeros((Vb * 12, V, 12), np.complex128)
    for k in range(Vb):
        for comp in range(12):
            src[k * 12 + comp, lidx == k, comp] = 1.0
    out = oracle.block_dirac(L, b, U, A, src.reshape(-1, V, 4, 3)).reshape(Vb * 12, V, 12)
    ops = np.zeros((nblk, Vb * 12, Vb * 12), np.complex128)
    for j in range(nblk):
        sites = np.where(bid == j)[0]
        order = sites[np.argsort(lidx[sites])]
        # column (k, comp) read at the block's sites in local order
        ops[j] = out[:, order, :].reshape(Vb * 12, Vb * 12).T
    return ops, bid, lidx


def test_T8_mr_properties(field):
    U, A = field
    r = inputs.test_vectors(L4, 1, 7)
    j = 5
    mask = _block_mask(L4, B2, j)
    # monotone residual norms
    e, norms = oracle.mr(L4, B2, U, A, j, r, 8)
    assert np.all(np.diff(norms) <= 1e-15 * norms[0])
    assert np.isclose(norms[0], np.linalg.norm(r[:, mask]), rtol=1e-14)
    assert np.max(np.abs(e[:, ~mask])) == 0.0
    # one step: e = alpha r with alpha = <D_j r, r> / ||D_j r||^2
    e1, _ = oracle.mr(L4, B2, U, A, j, r, 1)
    rj = r * mask[None, :, None, None]
    q = oracle.block_dirac(L4, B2, U, A, rj)
    alpha = np.vdot(q, rj) / np.vdot(q, q).real
    assert rel(e1, alpha * rj) < 1e-14
    # many steps converge to the dense block solve
    ops, bid, lidx = _dense_block_ops(L4, B2, U, A)
    sites = np.where(bid == j)[0]
    order = sites[np.argsort(lidx[sites])]
    rl = r[0][order].reshape(-1)
    el = np.linalg.solve(ops[j], rl)
    e60, norms60 = oracle.mr(L4, B2, U, A, j, r, 60)
    assert rel(e60[0][order].reshape(-1), el) < 1e-10


def test_T8_mr_zero_residual(field):
    """A zero block residual gives <q,q> = 0: step length 0, no NaN."""
    U, A = field
    r = np.zeros((1, 256, 4, 3), np.complex128)
    e, norms = oracle.mr(L4, B2, U, A, 3, r, 4)
    assert np.all(e == 0) and np.all(norms == 0)


def test_T9_exact_block_solves(field):
    """With block solves driven to convergence, SAP is the textbook multiplicative Schwarz
    iteration x <- x + K_c (b - D x), K_c = sum_{j of colour c} I_j D_j^-1 I_j^T."""
    U, A = field
    bvec = inputs.test_vectors(L4, 1, 9)
    ops, bid, lidx = _dense_block_ops(L4, B2, U, A)
    nb = [2, 2, 2, 2]
    colour = np.array([sum(np.unravel_index(j, nb[::-1])) % 2 for j in range(16)])
    x = np.zeros_like(bvec)
    for sweep in range(2):
        for c in (0, 1):
            r = bvec - oracle.dirac(L4, U, A, x)
            for j in np.where(colour == c)[0]:
                sites = np.where(bid == j)[0]
                order = sites[np.argsort(lidx[sites])]
                ej = np.linalg.solve(ops[j], r[0][order].reshape(-1))
                x[0][order] += ej.reshape(-1, 4, 3)
    got = oracle.sap(L4, B2, U, A, bvec, 2, 200)
    assert rel(got, x) < 1e-10


def test_colour_convention(field):
    """Block colour is the parity of the block-coordinate sum; red (0) goes first: after
    a single red half-sweep worth of work, only red blocks are non-zero.  Checked through
    n_sap = 1 against an explicit red-then-black construction with 1 MR step."""
    U, A = field
    bvec = inputs.test_vectors(L4, 1, 13)
    x = np.zeros_like(bvec)
    c = inputs.site_coords(L4)
    colour_site = (c // 2).sum(axis=1) % 2
    for col in (0, 1):
        r = bvec - oracle.dirac(L4, U, A, x)
        for j in range(16):
            m = _block_mask(L4, B2, j)
            if colour_site[m][0] != col:
                continue
            e, _ = oracle.mr(L4, B2, U, A, j, r, 1)
            x = x + e
    got = oracle.sap(L4, B2, U, A, bvec, 1, 1)
    assert rel(got, x) < 1e-14


def test_T10_homogeneity(field):
    U, A = field
    bvec = inputs.test_vectors(L4, 1, 15)
    c = 0.37 - 2.1j
    x1 = oracle.sap(L4, B2, U, A, c * bvec, 2, 3)
    x2 = c * oracle.sap(L4, B2, U, A, bvec, 2, 3)
    assert rel(x1, x2) < 1e-13


def test_sap_not_additive(field):
    """SAP with a fixed MR step count is not linear (the step lengths depend on b)."""
    U, A = field
    v = inputs.test_vectors(L4, 2, 16)
    lhs = oracle.sap(L4, B2, U, A, v[:1] + v[1:], 2, 3)
    rhs = oracle.sap(L4, B2, U, A, v[:1], 2, 3) + oracle.sap(L4, B2, U, A, v[1:], 2, 3)
    assert rel(lhs, rhs) > 1e-4


@pytest.mark.parametrize("mu,s", [(3, 4), (0, 4), (1, 4)])
def test_T11_shift_covariance(mu, s):
    """Shifting field and source by two blocks (colour-preserving) shifts the result."""
    L = [8, 8, 4, 8]
    U = inputs.gauge_field(L, 0.3, 111)
    A = oracle.clover(L, U, 1.0, -0.1)
    bvec = inputs.test_vectors(L, 1, 112)
    x = oracle.sap(L, B2, U, A, bvec, 2, 3)
    Us = shift_field(L, U, mu, s)
    As = oracle.clover(L, Us, 1.0, -0.1)
    xs = oracle.sap(L, B2, Us, As, shift_vectors(L, bvec, mu, s), 2, 3)
    assert rel(xs, shift_vectors(L, x, mu, s)) < 1e-13


def test_T11_odd_shift_breaks_covariance():
    """A shift by one block swaps the colours, and the result changes (the pin is sharp)."""
    L = [8, 4, 4, 4]
    U = inputs.gauge_field(L, 0.3, 113)
    A = oracle.clover(L, U, 1.0, -0.1)
    bvec = inputs.test_vectors(L, 1, 114)
    x = oracle.sap(L, B2, U, A, bvec, 1, 2)
    Us = shift_field(L, U, 0, 2)
    As = oracle.clover(L, Us, 1.0, -0.1)
    xs = oracle.sap(L, B2, Us, As, shift_vectors(L, bvec, 0, 2), 1, 2)
    assert rel(xs, shift_vectors(L, x, 0, 2)) > 1e-3


def test_T12_gauge_covariance(field):
    U, A = field
    W = inputs.gauge_transform(L4, 121)
    UW = gauge_rotate_links(L4, U, W)
    AW = oracle.clover(L4, UW, 1.0, -0.1)
    bvec = inputs.test_vectors(L4, 2, 122)
    x = oracle.sap(L4, B2, U, A, bvec, 2, 3)
    xw = oracle.sap(L4, B2, UW, AW, colour_rotate(W, bvec), 2, 3)
    assert rel(xw, colour_rotate(W, x)) < 1e-13


def test_T13_mrhs_equals_loop(field):
    U, A = field
    v = inputs.test_vectors(L4, 3, 131)
    xm = oracle.sap(L4, B2, U, A, v, 2, 3)
    for k in range(3):
        assert np.array_equal(xm[k:k + 1], oracle.sap(L4, B2, U, A, v[k:k + 1], 2, 3))


def test_T14_residual_decreases(field):
    U, A = field
    v = inputs.test_vectors(L4, 2, 141)
    prev = np.ones(2)
    for n_sap in (1, 2, 3, 4):
        x = oracle.sap(L4, B2, U, A, v, n_sap, 3)
        res = oracle.residual_norms(L4, U, A, v, x)
        assert np.all(res < prev)
        prev = res
    assert np.all(prev < 0.05)


def test_residual_norms_definition(field):
    """The final residual check (a6): ||b_k - D x_k||_2 / ||b_k||_2 per vector, at a non-zero
    residual.  x = 0 gives exactly 1 whatever the norm of b (a wrong denominator such as
    ||b||^2 fails); a random x is checked against the norm computed in numpy from D x; the
    value is invariant under a common complex scale of b and x, and the vectors are
    independent (a vector's value does not depend on the others of the stack).  The oracle
    sums with OpenMP reductions, so repeated values agree to rounding, not bit for bit."""
    U, A = field
    rng = np.random.default_rng(171)
    b = inputs.test_vectors(L4, 3, 172) * np.array([0.25, 1.0, 7.0])[:, None, None, None]
    x = 0.3 * (rng.standard_normal(b.shape) + 1j * rng.standard_normal(b.shape))
    assert np.allclose(oracle.residual_norms(L4, U, A, b, np.zeros_like(b)), 1.0, rtol=1e-14, atol=0)
    got = oracle.residual_norms(L4, U, A, b, x)
    r = (b - oracle.dirac(L4, U, A, x)).reshape(3, -1)
    want = np.linalg.norm(r, axis=1) / np.linalg.norm(b.reshape(3, -1), axis=1)
    assert np.all(want > 0.1)
    assert np.allclose(got, want, rtol=1e-13, atol=0)
    c = 2.5 - 1.5j
    assert np.allclose(oracle.residual_norms(L4, U, A, c * b, c * x), got, rtol=1e-13, atol=0)
    assert np.allclose(oracle.residual_norms(L4, U, A, b[1:2], x[1:2]), got[1:2], rtol=1e-14, atol=0)


def test_odd_block_count_same_colour_neighbours():
    """12^4-like case (3 blocks per direction): same-coloured blocks touch across the wrap.
    All blocks of a colour use the residual computed before the colour's updates, so the
    result does not depend on the block visiting order: checked against a dense sweep."""
    L = [6, 6, 2, 2]
    b = [2, 2, 2, 2]
    U = inputs.gauge_field(L, 0.3, 151)
    A = oracle.clover(L, U, 1.0, -0.2)
    bvec = inputs.test_vectors(L, 1, 152)
    ops, bid, lidx = _dense_block_ops(L, b, U, A)
    nb = [3, 3, 1, 1]
    nblk = 9
    coords = [np.unravel_index(j, nb[::-1])[::-1] for j in range(nblk)]
    colour = np.array([sum(cc) % 2 for cc in coords])
    x = np.zeros_like(bvec)
    for c in (0, 1):
        r = bvec - oracle.dirac(L, U, A, x)
        for j in np.where(colour == c)[0][::-1]:  # reverse order on purpose
            sites = np.where(bid == j)[0]
            order = sites[np.argsort(lidx[sites])]
            ej = np.linalg.solve(ops[j], r[0][order].reshape(-1))
            x[0][order] += ej.reshape(-1, 4, 3)
    got = oracle.sap(L, b, U, A, bvec, 1, 300)
    assert rel(got, x) < 1e-10


def test_block_spanning_direction_keeps_wrap_hop():
    """A block that spans a whole direction: D_j = I_j^T D I_j keeps the wrap-around hop.
    With one block in total, SAP with converged MR is an exact solve of D."""
    L = [2, 2, 2, 4]
    b = [2, 2, 2, 4]
    U = inputs.gauge_field(L, 0.3, 161)
    A = oracle.clover(L, U, 1.0, 0.2)
    bvec = inputs.test_vectors(L, 1, 162)
    x = oracle.sap(L, b, U, A, bvec, 1, 400)
    assert oracle.residual_norms(L, U, A, bvec, x)[0] < 1e-10


def test_T9b_sap_from_guess():
    """SAP from a starting guess (the refinement phase, Alg. 1 and 2): from zero it is the
    initial-phase SAP, from the exact solution it stays there (zero residual, alpha = 0),
    and sweeps compose (3 sweeps = 1 sweep, then 2 more from its result)."""
    L, b = [2, 2, 2, 4], [2, 2, 2, 2]
    U = inputs.gauge_field(L, 0.3, 181)
    A = oracle.clover(L, U, 1.0, -0.1)
    v = inputs.test_vectors(L, 2, 182)
    assert np.array_equal(oracle.sap(L, b, U, A, v, 2, 3, x0=np.zeros_like(v)), oracle.sap(L, b, U, A, v, 2, 3))
    V = 32
    eye = np.eye(12 * V).reshape(12 * V, V, 4, 3)
    D = oracle.dirac(L, U, A, eye).reshape(12 * V, 12 * V).T
    xs = np.linalg.solve(D, v.reshape(2, -1).T).T.reshape(v.shape)
    got = oracle.sap(L, b, U, A, v, 3, 4, x0=xs)
    assert np.max(np.abs(got - xs)) < 1e-12 * np.max(np.abs(xs))
    rng = np.random.default_rng(183)
    x0 = rng.standard_normal(v.shape) + 1j * rng.standard_normal(v.shape)
    three = oracle.sap(L, b, U, A, v, 3, 4, x0=x0)
    one = oracle.sap(L, b, U, A, v, 1, 4, x0=x0)
    assert np.array_equal(three, oracle.sap(L, b, U, A, v, 2, 4, x0=one))
    # and it reduces the residual of a poor start
    r0 = oracle.residual_norms(L, U, A, v, x0)
    r3 = oracle.residual_norms(L, U, A, v, three)
    assert np.all(r3 < 0.5 * r0)
