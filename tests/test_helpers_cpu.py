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
