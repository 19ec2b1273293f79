"""Pins of the oracle's Wilson-clover operator (the 12V-dimensional operator of the
paper's Sec. 2) against identities, closed forms and invariants.  CPU only."""
import numpy as np
import pytest

import oracle
from paper_1601_03184_amd import inputs
from oracle_helpers import colour_rotate, gauge_rotate_links, rel


def test_T1_gamma_algebra():
    """Clifford algebra, hermiticity, g5 = diag(1,1,-1,-1) (chiral basis)."""
    g = [oracle.gamma(m) for m in range(4)]
    for m in range(4):
        assert np.allclose(g[m], g[m].conj().T, atol=0)
        for n in range(4):
            anti = g[m] @ g[n] + g[n] @ g[m]
            assert np.array_equal(anti, 2.0 * (m == n) * np.eye(4))
    assert np.array_equal(oracle.gamma(4), np.diag([1, 1, -1, -1]).astype(complex))
    assert np.array_equal(g[0] @ g[1] @ g[2] @ g[3], oracle.gamma(4))


def _g5(v):
    return v * np.array([1, 1, -1, -1])[None, None, :, None]


@pytest.mark.parametrize("L,csw", [([4, 4, 4, 4], 1.0), ([2, 4, 6, 4], 1.7)])
def test_T2_gamma5_hermiticity(L, csw):
    """<phi, g5 D g5 psi> = <D phi, psi> for a random SU(3) field."""
    U = inputs.gauge_field(L, 0.3, 11)
    A = oracle.clover(L, U, csw, -0.2)
    v = inputs.test_vectors(L, 2, 12)
    phi, psi = v[:1], v[1:]
    lhs = np.vdot(phi, _g5(oracle.dirac(L, U, A, _g5(psi))))
    rhs = np.vdot(oracle.dirac(L, U, A, phi), psi)
    assert abs(lhs - rhs) / abs(rhs) < 1e-13


@pytest.mark.parametrize("n", [(0, 0, 0, 0), (1, 0, 2, 1), (3, 1, 5, 3), (2, 1, 3, 0)])
def test_T3_free_field_plane_wave(n):
    """U = 1: D e^{ipx} u = e^{ipx} [m0 + sum(1 - cos p) + i sum g_mu sin p_mu] u."""
    L = [4, 2, 6, 4]
    m0 = -0.3
    U = inputs.unit_gauge_field(L)
    A = oracle.clover(L, U, 1.0, m0)
    p = np.array([2 * np.pi * n[m] / L[m] for m in range(4)])
    x = inputs.site_coords(L)
    phase = np.exp(1j * (x @ p))
    rng = np.random.default_rng(3)
    u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
    psi = phase[None, :, None, None] * u[None, None]
    M = (m0 + np.sum(1 - np.cos(p))) * np.eye(4) + 1j * sum(oracle.gamma(m) * np.sin(p[m]) for m in range(4))
    expect = phase[None, :, None, None] * (M @ u)[None, None]
    got = oracle.dirac(L, U, A, psi)
    assert rel(got, expect) < 1e-13
    # the spectrum of M is m0 + sum(1-cos) +- i |sin p|, each twice
    ev = np.linalg.eigvals(M)
    ev = ev[np.argsort(ev.imag)]
    s = np.sqrt(np.sum(np.sin(p) ** 2))
    re = m0 + np.sum(1 - np.cos(p))
    assert np.allclose(ev, np.array([re - 1j * s] * 2 + [re + 1j * s] * 2), atol=1e-13)


def test_T4_pure_gauge():
    """U_mu(x) = W(x) W(x+mu)^dag: clover vanishes and D[U] (W psi) = W D_free psi."""
    L = [4, 4, 2, 4]
    m0 = 0.1
    W = inputs.gauge_transform(L, 5)
    U = gauge_rotate_links(L, inputs.unit_gauge_field(L), W)
    A = oracle.clover(L, U, 1.0, m0)
    assert np.max(np.abs(A - (4 + m0) * np.eye(12))) < 1e-13
    Uf = inputs.unit_gauge_field(L)
    Af = oracle.clover(L, Uf, 1.0, m0)
    psi = inputs.test_vectors(L, 1, 6)
    got = oracle.dirac(L, U, A, colour_rotate(W, psi))
    expect = colour_rotate(W, oracle.dirac(L, Uf, Af, psi))
    assert rel(got, expect) < 1e-13


def test_T5_gauge_covariance():
    """D[U^W](W psi) = W D[U] psi and A[U^W](x) = W(x) A[U](x) W(x)^dag."""
    L = [4, 4, 4, 2]
    U = inputs.gauge_field(L, 0.4, 21)
    W = inputs.gauge_transform(L, 22)
    UW = gauge_rotate_links(L, U, W)
    A = oracle.clover(L, U, 1.0, -0.1)
    AW = oracle.clover(L, UW, 1.0, -0.1)
    Wbig = np.einsum("st,xab->xsatb", np.eye(4), W).reshape(-1, 12, 12)
    assert rel(AW, Wbig @ A @ np.conj(np.swapaxes(Wbig, -1, -2))) < 1e-13
    psi = inputs.test_vectors(L, 2, 23)
    got = oracle.dirac(L, UW, AW, colour_rotate(W, psi))
    expect = colour_rotate(W, oracle.dirac(L, U, A, psi))
    assert rel(got, expect) < 1e-13


@pytest.mark.parametrize("k", [1, 2])
def test_T6_uniform_flux_clover(k):
    """U_0(x) = exp(i f x_1 lam), lam = diag(1,-1,0), f = 2 pi k / L_1, other links 1:
    the site block of D is (4+m0) + (i csw/2) g0 g1 (x) diag(sin f, -sin f, 0).
    Probed with point sources (column by column)."""
    L = [4, 6, 3, 4]
    m0, csw = -0.25, 1.3
    f = 2 * np.pi * k / L[1]
    U = inputs.unit_gauge_field(L)
    x = inputs.site_coords(L)
    lam = np.array([1.0, -1.0, 0.0])
    U[0] = np.exp(1j * f * x[:, 1, None] * lam[None, :])[:, :, None] * np.eye(3)[None]
    A = oracle.clover(L, U, csw, m0)
    g0, g1 = oracle.gamma(0), oracle.gamma(1)
    expect = (4 + m0) * np.eye(12) + (1j * csw / 2) * np.kron(g0 @ g1, np.diag([np.sin(f), -np.sin(f), 0]))
    V = inputs.volume(L)
    x0 = 37
    src = np.zeros((12, V, 12), np.complex128)
    for c in range(12):
        src[c, x0, c] = 1.0
    out = oracle.dirac(L, U, A, src.reshape(12, V, 4, 3)).reshape(12, V, 12)
    block = out[:, x0, :].T  # column c = D applied to unit vector c, read at x0
    assert np.max(np.abs(block - expect)) < 1e-13
    assert np.max(np.abs(A - expect[None])) < 1e-13


def test_T7_clover_hermitian_chiral_blocks():
    L = [4, 4, 4, 4]
    U = inputs.gauge_field(L, 0.3, 31)
    m0 = -0.1
    A = oracle.clover(L, U, 1.0, m0)
    C = A - (4 + m0) * np.eye(12)
    assert np.max(np.abs(C - np.conj(np.swapaxes(C, -1, -2)))) < 1e-14
    assert np.max(np.abs(C[:, :6, 6:])) == 0.0
    assert np.max(np.abs(C[:, 6:, :6])) == 0.0
    assert np.max(np.abs(C)) > 0.1  # a non-trivial field gives a non-trivial clover term


def test_block_operator_is_restriction():
    """block_dirac on a vector supported on block j equals (D x) restricted to block j,
    and is zero outside the block."""
    L = [4, 4, 4, 4]
    b = [2, 2, 2, 2]
    U = inputs.gauge_field(L, 0.3, 41)
    A = oracle.clover(L, U, 1.0, -0.1)
    x = inputs.test_vectors(L, 1, 42)
    c = inputs.site_coords(L)
    in_block = np.all((c // np.array(b)) == np.array([1, 0, 1, 1]), axis=1)
    xs = x * in_block[None, :, None, None]
    y = oracle.block_dirac(L, b, U, A, xs)
    full = oracle.dirac(L, U, A, xs)
    assert rel(y[:, in_block], full[:, in_block]) < 1e-15
    assert np.max(np.abs(y[:, ~in_block])) == 0.0
    # the full operator does couple the block to its neighbours
    assert np.max(np.abs(full[:, ~in_block])) > 0.1
