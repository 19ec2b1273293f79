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


# ---------------------------------------------------------------------------------------
# Generators on a torch device, for lattices whose inputs are too large to draw on the
# host in reasonable time (the full-size workloads).  Same distributions as above, with
# torch's generator of that device; the exponential is a Taylor series instead of an
# eigen-decomposition (the same matrix up to rounding).
# ---------------------------------------------------------------------------------------

def _su3_exp_device(A, sigma):
    """U = exp(i sigma H), H = (A + A^dag)/2 made traceless, re-unitarised as above.
    exp by scaling and squaring: (sum_{n<=20} (X/4)^n / n!)^4, X = i sigma H."""
    import torch
    H = 0.5 * (A + A.conj().transpose(-1, -2))
    tr = torch.diagonal(H, dim1=-2, dim2=-1).sum(-1).real / 3.0
    eye = torch.eye(3, dtype=A.dtype, device=A.device)
    H = H - tr[:, None, None] * eye
    X = (1j * sigma / 4.0) * H
    term = eye.expand_as(X).clone()
    E = term.clone()
    for n in range(1, 21):
        term = term @ X / n
        E = E + term
    E = E @ E
    U = E @ E
    r0 = U[:, 0, :]
    r0 = r0 / torch.linalg.vector_norm(r0, dim=-1, keepdim=True)
    r1 = U[:, 1, :]
    r1 = r1 - (r0.conj() * r1).sum(-1, keepdim=True) * r0
    r1 = r1 / torch.linalg.vector_norm(r1, dim=-1, keepdim=True)
    r2 = torch.linalg.cross(r0, r1).conj()
    return torch.stack([r0, r1, r2], dim=1)


def gauge_field_device(L, sigma, seed, device):
    """Links U_mu(x), complex128 [4][V][3][3] on `device`, canonical site order.  Draws:
    a generator of that device seeded with `seed`, chunks of 2^22 links in order, each a
    (m, 2, 3, 3) standard normal tensor (real parts, then imaginary parts)."""
    import torch
    V = volume(L)
    n = 4 * V
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    out = torch.empty((n, 3, 3), dtype=torch.complex128, device=device)
    chunk = 1 << 22
    for s in range(0, n, chunk):
        m = min(chunk, n - s)
        d = torch.randn((m, 2, 3, 3), generator=gen, dtype=torch.float64, device=device)
        out[s:s + m] = _su3_exp_device(torch.complex(d[:, 0], d[:, 1]), sigma)
    return out.reshape(4, V, 3, 3)


def test_vectors_device(L, n, seed, device, first=0):
    """Test vectors first .. first + n - 1 of a set, complex128 [n][V][4][3] on `device`:
    vector k has re, im ~ N(0,1) from a generator of that device seeded with
    seed * 1000003 + k, so any subset is reproducible on its own."""
    import torch
    V = volume(L)
    out = torch.empty((n, V, 4, 3), dtype=torch.complex128, device=device)
    gen = torch.Generator(device=device)
    for j in range(n):
        gen.manual_seed(seed * 1000003 + first + j)
        d = torch.randn((V, 12, 2), generator=gen, dtype=torch.float64, device=device)
        out[j] = torch.complex(d[..., 0], d[..., 1]).reshape(V, 4, 3)
    return out
