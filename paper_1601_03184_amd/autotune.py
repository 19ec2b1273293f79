"""Execution-tile autotuner for the SAP and stencil kernels.

A tile is the number of right-hand sides one workgroup handles (1, 2 or 4; it must divide
the native short length S and fit the block and the LDS).  It changes only the execution
(occupancy, register use, how many lanes share one field load), never the result beyond
reduction order: the SAP block size and the aggregates are part of the problem, not tiles.

autotune(op, n_rhs) times every valid tile with HIP events on the stream the kernels run
on, keeps the fastest, applies it with mrhs_set_tiles, and caches the choice per
(device, lattice, block, precision, S, n_rhs, block solver, n_sap, n_mr) in memory and, if a
path is given, in a JSON file.  The plain and the even-odd block solver run different kernels
(other occupancy and register use), so a choice made for one is never reused for the other.
"""
import json
import os

import torch

from . import mrhs

TILES = (1, 2, 4)
_cache = {}


def _key(op, n_rhs, n_sap, n_mr):
    dev = torch.cuda.get_device_name(op.device)
    return "%s|L=%s|b=%s|prec=%d|S=%d|n=%d|solver=%d|sap=%dx%d" % (
        dev, "x".join(map(str, op.L)), "x".join(map(str, op.block)), op.prec, op.S, n_rhs,
        mrhs.mrhs_op_block_solver(op.handle), n_sap, n_mr)


def _time(fn, reps=3):
    fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def _valid_tiles(op, which):
    out = []
    for t in TILES:
        try:
            if which == "sap":
                mrhs.mrhs_set_tiles(op.handle, t, 0)
            else:
                mrhs.mrhs_set_tiles(op.handle, 0, t)
            out.append(t)
        except mrhs.MrhsError:
            pass
    return out


def autotune(op, n_rhs, n_sap=3, n_mr=4, path=None, reps=3, b=None, x=None):
    """Pick the fastest SAP and stencil tiles for (op, n_rhs); returns {"sap": t, "dirac": t, ...}.

    b, x: optional native vector sets of the op for n_rhs right-hand sides to time on (b with
    zero padding lanes, as mrhs_pack writes them; x is overwritten); by default random ones
    are allocated for the timing."""
    key = _key(op, n_rhs, n_sap, n_mr)
    if key not in _cache and path and os.path.exists(path):
        with open(path) as f:
            _cache.update(json.load(f))
    if key in _cache:
        choice = _cache[key]
        mrhs.mrhs_set_tiles(op.handle, choice["sap"], choice["dirac"])
        return choice
    if b is None:
        # packed from canonical vectors, so that the padding lanes of the last group are zero
        canon = torch.randn(n_rhs, op.V, 4, 3, dtype=torch.complex128, device=op.device)
        b = op.pack(canon)
        del canon
    if x is None:
        x = op.empty(n_rhs)
    ws = op.workspace(n_rhs)
    sap_ms = {}
    for t in _valid_tiles(op, "sap"):
        mrhs.mrhs_set_tiles(op.handle, t, 0)
        sap_ms[t] = _time(lambda: mrhs.sap_smooth_mrhs(op.handle, b, x, n_rhs, n_sap, n_mr, ws), reps)
    dirac_ms = {}
    for t in _valid_tiles(op, "dirac"):
        mrhs.mrhs_set_tiles(op.handle, 0, t)
        dirac_ms[t] = _time(lambda: mrhs.dirac_apply_mrhs(op.handle, b, x, n_rhs), reps)
    choice = {"sap": min(sap_ms, key=sap_ms.get), "dirac": min(dirac_ms, key=dirac_ms.get),
              "sap_ms": {str(k): v for k, v in sap_ms.items()}, "dirac_ms": {str(k): v for k, v in dirac_ms.items()}}
    mrhs.mrhs_set_tiles(op.handle, choice["sap"], choice["dirac"])
    _cache[key] = choice
    if path:
        with open(path, "w") as f:
            json.dump(_cache, f, indent=1)
    return choice
