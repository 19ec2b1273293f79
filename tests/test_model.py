"""T22: the paper's worked numbers (Sec. 6 and Sec. 7) from the byte/flop model."""
import json
import os

import pytest

from paper_1601_03184_amd import perfmodel as pm

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.json")))


def test_matvec_and_matmat_bandwidth():
    knc = GOLD["knc"]
    big = 1e9  # K, M large
    bpc = pm.paper_required_bytes_per_cycle(big, big, lanes=knc["sp_lanes"])
    assert bpc == pytest.approx(GOLD["matvec_bytes_per_cycle_per_core"]["value"], rel=1e-6)
    gbs = pm.paper_required_gbs(bpc, knc["cores"], knc["clock_ghz"])
    assert round(gbs) == GOLD["matvec_required_gbs"]["value"]
    bpc_mm = pm.paper_required_bytes_per_cycle(big, big, n_rhs=16, lanes=knc["sp_lanes"])
    assert bpc_mm == pytest.approx(GOLD["matmat_bytes_per_cycle_per_core"]["value"], rel=1e-6)
    gbs_mm = pm.paper_required_gbs(bpc_mm, knc["cores"], knc["clock_ghz"])
    assert round(gbs_mm) == GOLD["matmat_required_gbs"]["value"]
    assert gbs_mm <= GOLD["stream_gbs"]["high"]  # "within reach" of the sustained bandwidth
    assert gbs > 10 * GOLD["stream_gbs"]["high"]


def test_matvec_formula_small_sizes():
    # 32 (2/K + 1 + 1/M) with K = 4, M = 8
    assert pm.paper_required_bytes_per_cycle(4, 8) == pytest.approx(32 * (2 / 4 + 1 + 1 / 8))
    assert pm.paper_required_bytes_per_cycle(4, 8, n_rhs=16) == pytest.approx(32 * (2 / 4 + 1 / 16 + 1 / 8))


def test_memory_accounting():
    r = pm.coarse_fine_memory_ratio(16, 4 ** 4)
    assert round(100 * r) == GOLD["coarse_over_fine_memory_percent"]["value"]
    f = pm.setup_memory_factor(GOLD["fine_vectors"]["mrhs"], GOLD["coarse_vectors"]["mrhs"],
                               GOLD["fine_vectors"]["srhs"], GOLD["coarse_vectors"]["srhs"], r)
    assert round(f, 1) == GOLD["memory_factor"]["value"]
    assert GOLD["coarse_vectors"]["mrhs"] == 16 * GOLD["fine_vectors"]["mrhs"]


def test_stencil_bytes():
    # FP32 fields and spinors, 20 RHS: 144*4/20 + 48*4 = 220.8 B per site-RHS
    assert pm.stencil_bytes_per_site_rhs(20, 4, 4) == pytest.approx(220.8)
    # single-RHS FP64: 144*8 + 48*8 = 1536
    assert pm.stencil_bytes_per_site_rhs(1, 8, 8) == pytest.approx(1536)
