"""CPU checks of the error measures the GPU parity tests use."""
import numpy as np

from gpu_helpers import per_agg_half_rel, per_rhs_rel
from paper_1601_03184_amd import inputs


def test_per_agg_half_rel_isolates_one_aggregate_half():
    """A perturbation of one (aggregate, spin half) shows at its own relative size, not
    diluted by the other halves (a whole-set norm would report it about sqrt(2 n_agg)
    times smaller)."""
    L, agg = [4, 4, 2, 4], [2, 2, 2, 2]
    ref = inputs.test_vectors(L, 3, 11)
    got = ref.copy()
    c = inputs.site_coords(L)
    # aggregate with coordinates (1, 0, 0, 1): lexicographic index 1 + 2 * (0 + 2 * (0 + 1 * 1)) = 5
    sites = np.where((c[:, 0] // 2 == 1) & (c[:, 1] // 2 == 0) & (c[:, 2] // 2 == 0) & (c[:, 3] // 2 == 1))[0]
    blk = ref[:, sites, 2:4, :]        # spin half r of that aggregate
    got[:, sites, 2:4, :] = 1.01 * blk
    assert abs(per_agg_half_rel(got, ref, L, agg) - 0.01) < 1e-12
    whole = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert whole < 0.01 / 4
    assert per_agg_half_rel(ref, ref, L, agg) == 0.0


def test_per_rhs_rel_is_the_max_over_vectors():
    ref = inputs.test_vectors([2, 2, 2, 2], 4, 12)
    got = ref.copy()
    got[2] *= 1.0 + 3e-3
    assert abs(per_rhs_rel(got, ref) - 3e-3) < 1e-12


def test_average_plaquette_of_the_bench():
    """The bench's plaquette statistic: 1 for unit links, invariant under a random gauge
    transformation, and equal to the plaquettes summed site by site with numpy on a lattice
    with extents 2, 3, 2, 3 (so that a swapped axis or shift direction shows)."""
    import torch
    import bench

    L = [2, 3, 2, 3]
    V = int(np.prod(L))
    unit = torch.eye(3, dtype=torch.complex128).expand(4, V, 3, 3).contiguous()
    assert abs(bench.average_plaquette(unit, L) - 1.0) < 1e-14
    U = inputs.gauge_field(L, 0.4, 21)
    c = inputs.site_coords(L)

    def shift(x, mu):
        y = c[x].copy()
        y[mu] = (y[mu] + 1) % L[mu]
        return int(y[0] + L[0] * (y[1] + L[1] * (y[2] + L[2] * y[3])))

    tot = 0.0
    for x in range(V):
        for mu in range(4):
            for nu in range(mu + 1, 4):
                p = U[mu, x] @ U[nu, shift(x, mu)] @ U[mu, shift(x, nu)].conj().T @ U[nu, x].conj().T
                tot += np.trace(p).real
    ref = tot / (3 * 6 * V)
    got = bench.average_plaquette(torch.from_numpy(U), L)
    assert abs(got - ref) < 1e-12
    # a gauge transformation g(x): U_mu(x) -> g(x) U_mu(x) g(x + mu)^dag leaves it unchanged
    g = inputs.gauge_field(L, 0.9, 22)[0]
    Ug = np.stack([np.stack([g[x] @ U[mu, x] @ g[shift(x, mu)].conj().T for x in range(V)]) for mu in range(4)])
    assert abs(bench.average_plaquette(torch.from_numpy(Ug), L) - ref) < 1e-12
    assert abs(ref - 1.0) > 1e-3
