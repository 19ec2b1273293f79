"""Test-side helpers for pinning the oracle: colour/spin actions written out in numpy.

These are independent re-statements used only to build test inputs and expected
values (gauge transformations, lattice shifts, plane waves); they never call the
GPU library.
"""
import numpy as np

from paper_1601_03184_amd import inputs


def colour_rotate(Om, psi):
    """(Omega psi)(x) = Omega(x) psi(x) on every spin component; psi [n][V][4][3]."""
    return np.einsum("xab,nxsb->nxsa", Om, psi)


def gauge_rotate_links(L, U, Om):
    """U^Omega_mu(x) = Omega(x) U_mu(x) Omega(x+mu)^dag."""
    out = np.empty_like(U)
    V = inputs.volume(L)
    for mu in range(4):
        fwd = shift_index(L, mu, +1)
        out[mu] = Om @ U[mu] @ np.conj(np.swapaxes(Om[fwd], -1, -2))
    assert out.shape == (4, V, 3, 3)
    return out


def shift_index(L, mu, step):
    """Index array: site x -> site x + step*mu (periodic)."""
    c = inputs.site_coords(L)
    c = c.copy()
    c[:, mu] = (c[:, mu] + step) % L[mu]
    return c[:, 0] + L[0] * (c[:, 1] + L[1] * (c[:, 2] + L[2] * c[:, 3]))


def shift_field(L, U, mu, s):
    """(T U)_nu(x) = U_nu(x - s mu)."""
    src = shift_index(L, mu, -s)
    return U[:, src]


def shift_vectors(L, v, mu, s):
    src = shift_index(L, mu, -s)
    return v[:, src]


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def coarse_neighbour(Lc, i, d):
    """Coarse site reached from i by slot d of the 9-block stencil."""
    c = []
    r = i
    for mu in range(4):
        c.append(r % Lc[mu])
        r //= Lc[mu]
    if d > 0:
        mu = (d - 1) % 4
        step = 1 if d <= 4 else -1
        c[mu] = (c[mu] + step) % Lc[mu]
    return c[0] + Lc[0] * (c[1] + Lc[1] * (c[2] + Lc[2] * c[3]))


def coarse_apply(Lc, Dc, yc):
    """(D_c y_c)(i) = sum_d Dc[i][d] y_c(neighbour_d(i)); yc [n][Vc][2][n_tv]."""
    n, Vc = yc.shape[0], yc.shape[1]
    nc = Dc.shape[-1]
    y = yc.reshape(n, Vc, nc)
    out = np.zeros_like(y)
    for i in range(Vc):
        for d in range(9):
            j = coarse_neighbour(Lc, i, d)
            out[:, i] += y[:, j] @ Dc[i, d].T
    return out.reshape(yc.shape)


def coarse_dense(Lc, Dc):
    """Dense coarse matrix assembled from the 9 per-direction blocks (coinciding blocks sum)."""
    Vc = Dc.shape[0]
    nc = Dc.shape[-1]
    M = np.zeros((Vc * nc, Vc * nc), np.complex128)
    for i in range(Vc):
        for d in range(9):
            j = coarse_neighbour(Lc, i, d)
            M[i * nc:(i + 1) * nc, j * nc:(j + 1) * nc] += Dc[i, d]
    return M
