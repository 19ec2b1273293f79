"""The execution-tile autotuner picks valid tiles, and the smoother's result with them
matches the FP64 oracle to the FP32 tolerance (tiles change execution, not the method)."""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import Case, announce, need_gpu, per_rhs_rel
from paper_1601_03184_amd import autotune, inputs, mrhs

pytestmark = pytest.mark.gpu


def test_autotune_choice_and_result(tmp_path):
    need_gpu()
    L = [8, 8, 4, 8]
    case = Case(L, 0.3, 211, -0.3)
    op = case.op([4, 4, 4, 4], prec=mrhs.PREC_F32, short_len=4)
    announce("autotune 8x8x4x8 n=12")
    path = str(tmp_path / "tiles.json")
    choice = autotune.autotune(op, 12, 3, 4, path=path)
    assert choice["sap"] in (1, 2, 4) and choice["dirac"] in (1, 2, 4)
    assert set(choice["sap_ms"]) <= {"1", "2", "4"} and len(choice["sap_ms"]) >= 2
    # cached: a second call returns the same choice without timing
    assert autotune.autotune(op, 12, 3, 4, path=path)["sap"] == choice["sap"]
    v = inputs.test_vectors(L, 12, 213)
    b = op.pack(torch.from_numpy(v))
    x = op.empty(12)
    mrhs.sap_smooth_mrhs(op.handle, b, x, 12, 3, 4, op.workspace(12))
    torch.cuda.synchronize()
    got = op.unpack(x, 12).cpu().numpy()
    ref = oracle.sap(L, [4, 4, 4, 4], case.U, case.A, v, 3, 4)
    assert per_rhs_rel(got, ref) < 1e-5
    op.close()
