"""Seeded synthetic inputs shared by the GPU tests, the benchmark and the oracle tests.

This module draws random numbers and nothing else of the method: gauge links, test
vectors and gauge transformations.  It holds none of the setup's arithmetic, so
both the oracle side and the GPU side may import it.

Gauge links follow the recipe of the synthetic workloads: per link, A = N(0,1) +
i N(0,1) (3x3), H = (A + A^dag)/2 made traceless, U = exp(i sigma H) through an
eigen-decomposition, then re-unitarised (normalise row 0, Gram-Schmidt row 1,
row 2 = conj(row0 x row1)) so that U is in SU(3) to rounding.  Draw order:
direction-major, then site, then the 9 real parts, then the 9 imaginary parts.
"""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_CHUNK = 1 << 18  # links per generation chunk (bounds host memory on big lattices)


def volume(L):
    return int(np.prod(L))


def _su3_from_draws(d, sigma):
    A = d[:, 0] + 1j * d[:, 1]
    H = 0.5 * (A + np.conj(np.swapaxes(A, -1, -2)))
    tr = np.trace(H, axis1=-2, axis2=-1).real / 3.0
    H = H - tr[:, None, None] * np.eye(3)
    w, v = np.linalg.eigh(H)
    U = (v * np.exp(1j * sigma * w)[:, None, :]) @ np.conj(np.swapaxes(v, -1, -2))
    r0 = U[:, 0, :]
    r0 = r0 / np.linalg.norm(r0, axis=-1, keepdims=True)
    r1 = U[:, 1, :]
    r1 = r1 - np.sum(np.conj(r0) * r1, axis=-1, keepdims=True) * r0
    r1 = r1 / np.linalg.norm(r1, axis=-1, keepdims=True)
    r2 = np.conj(np.cross(r0, r1))
    return np.stack([r0, r1, r2], axis=1)


def random_su3(n, sigma, rng):
    """n SU(3) matrices from the recipe above, drawing from the Generator rng.

    Chunks are drawn in order and turned into matrices on a thread pool (numpy releases
    the interpreter lock in its array kernels); the result does not depend on the
    number of threads."""
    out = np.empty((n, 3, 3), np.complex128)
    starts = list(range(0, n, _CHUNK))
    workers = max(1, min(16, len(os.sched_getaffinity(0)), len(starts)))

    def work(s, d):
        out[s:s + d.shape[0]] = _su3_from_draws(d, sigma)

    with ThreadPoolExecutor(workers) as ex:
        for w0 in range(0, len(starts), workers):
            batch = [(s, rng.standard_normal((min(_CHUNK, n - s), 2, 3, 3))) for s in starts[w0:w0 + workers]]
            list(ex.map(lambda sd: work(*sd), batch))
    return out


def gauge_field(L, sigma, seed):
    """Links U_mu(x), complex128 [4][V][3][3], canonical site order."""
    V = volume(L)
    rng = np.random.default_rng(seed)
    return random_su3(4 * V, sigma, rng).reshape(4, V, 3, 3)


def unit_gauge_field(L):
    V = volume(L)
    U = np.zeros((4, V, 3, 3), np.complex128)
    U[:, :] = np.eye(3)
    return U


def gauge_transform(L, seed, sigma=3.0):
    """A random SU(3) matrix per site, complex128 [V][3][3]."""
    rng = np.random.default_rng(seed)
    return random_su3(volume(L), sigma, rng)


def test_vectors(L, n, seed):
    """n complex Gaussian vectors (re, im ~ N(0,1)), complex128 [n][V][4][3]."""
    V = volume(L)
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((n, V, 12, 2))
    return (d[..., 0] + 1j * d[..., 1]).reshape(n, V, 4, 3)


def site_coords(L):
    """Integer coordinates [V][4] of every site, x fastest."""
    V = volume(L)
    s = np.arange(V)
    out = np.empty((V, 4), np.int64)
    for mu in range(4):
        out[:, mu] = s % L[mu]
        s = s // L[mu]
    return out
