"""Benchmark of the MRHS setup path on one MI355X.

One step = the initial setup phase on all test vectors at once, inputs resident in HBM:
  sap_smooth_mrhs     SAP from x = 0 on N_tv vectors (FP32),
  mrhs_residual_norms FP64 check ||b - D x|| / ||b|| per vector,
  block_orthonormalize FP64 block Gram-Schmidt on the aggregates -> Q (FP32),
  coarse_op_build     D_c (9 blocks of 2N_tv x 2N_tv complex64 per coarse site).
Workload: 16^4 Wilson-clover lattice (synthetic links, sigma = 0.3), m0 = -0.3, csw = 1,
N_tv = 20 complex Gaussian test vectors, 4^4 SAP blocks and aggregates, 3 SAP sweeps x
4 MR steps.

Prints one JSON line.  value = site-RHS updates per second of the whole step
(V * N_tv * n_SAP / step time).  Also reports: the roofline of the dominant kernel
(SAP half-sweep, FP32 ALU bound) with HIP-event timing over the timed region, the
stencil's HBM roofline, the single-RHS FP64 GPU path for the same SAP (speedup), and the
CPU oracle on a bounded sample (baseline only).
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_1601_03184_amd import autotune, inputs, mrhs  # noqa: E402
from paper_1601_03184_amd import perfmodel as pm  # noqa: E402

L = [16, 16, 16, 16]
BLOCK = [4, 4, 4, 4]
AGG = [4, 4, 4, 4]
SIGMA, SEED_U, SEED_V = 0.3, 201, 202
M0, CSW = -0.3, 1.0
N_TV, N_SAP, N_MR = 20, 3, 4
HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3      # published, with packed FP32 FMA
FP32_ISSUE_PEAK_TFLOPS = 78.6        # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz, no packed FP32
# HBM traffic of the dominant kernel (SAP half-sweep, 16^4, N_tv 20, FP32), per launch and
# execution tile: rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE (KiB per dispatch, mean over the
# half-sweeps of the bench's calls), each scaled by what the counter reads for a plain 1 GiB
# device copy (FETCH x2.0, WRITE x1.0).  Valid only for the kernel sources they were taken
# with (SHA-1 of the files below); otherwise the bench reports traffic as null.
SAP_SOURCES = ["paper_1601_03184_amd/csrc/sap.hip", "paper_1601_03184_amd/csrc/stencil.h",
               "paper_1601_03184_amd/csrc/internal.h"]
SAP_TRAFFIC = {"sources_sha1": "c9b58bbecf8b0bd911d292b613501feab0e227b6", "fetch_scale": 2.0, "write_scale": 1.0,
               "kib": {1: (190998, 86481), 2: (187957, 64908), 4: (205072, 71680)}}


def sap_traffic_bytes(tile):
    h = hashlib.sha1()
    for f in SAP_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != SAP_TRAFFIC["sources_sha1"] or tile not in SAP_TRAFFIC["kib"]:
        return None
    fk, wk = SAP_TRAFFIC["kib"][tile]
    return (fk * SAP_TRAFFIC["fetch_scale"] + wk * SAP_TRAFFIC["write_scale"]) * 1024


WORKLOAD = ("16^4 Wilson-clover (sigma=0.3 links, m0=-0.3, csw=1), N_tv=20, SAP 4^4 blocks 3x4 FP32, "
            "FP64 residual check, FP64 block Gram-Schmidt on 4^4 aggregates, D_c FP32")


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def sap_flops_per_call(V, n, n_sap, n_mr, block):
    """Arithmetic the SAP call needs: block-operator MR steps on every site, the residual
    (skipped where x is still zero: the first red half-sweep, and same-colour blocks in the
    first black half-sweep)."""
    Vb = int(np.prod(block))
    inner = sum((Vb - Vb // b) for b in block) * 2 / (8.0 * Vb)   # fraction of hops inside a block
    hop = 1320.0
    rest = pm.STENCIL_FLOP - hop
    mr = n_mr * (rest + hop * inner + pm.MR_EXTRA_FLOP)
    full_res = pm.STENCIL_FLOP + pm.RESIDUAL_EXTRA_FLOP
    first_black_res = hop * (1 - inner) + pm.RESIDUAL_EXTRA_FLOP
    half = V / 2.0 * n
    per_call = half * (mr) + half * (mr + first_black_res) + (n_sap - 1) * 2 * half * (mr + full_res)
    return per_call


def sap_bytes_per_call(V, n, n_sap, store_b, field_b):
    """Algorithmic HBM bytes of a SAP call: per half-sweep the fields of that colour's sites
    once, b and x of those sites (x read except in the first sweep), x written, and the
    x halo the residual reads (2x the block volume for 4^4 blocks, 3/8 of it read-once is
    neglected: counted once per site of the other colour)."""
    half = V // 2
    s = pm.SPINOR_REALS * store_b
    f = (4 * pm.LINK_REALS + pm.CLOVER_REALS) * field_b
    total = 0.0
    for sweep in range(n_sap):
        for c in range(2):
            total += half * f
            total += half * n * s * 2                     # b read, x written
            if sweep > 0:
                total += half * n * s                     # x read (own)
            if sweep > 0 or c == 1:
                total += half * n * s                     # halo x of the other colour
    return total


def make_inputs(dev):
    U = inputs.gauge_field(L, SIGMA, SEED_U)
    v = inputs.test_vectors(L, N_TV, SEED_V)
    return U, v


class Setup:
    def __init__(self, U, v, prec, S, gs=True):
        self.op = mrhs.Operator(L, BLOCK, AGG, torch.from_numpy(U), M0, CSW, prec=prec, short_len=S)
        self.n = v.shape[0]
        self.b = self.op.pack(torch.from_numpy(v))
        self.x = self.op.empty(self.n)
        self.ws = self.op.workspace(self.n)
        self.res = torch.empty(self.n, dtype=torch.float64, device="cuda")
        if gs:
            self.Q = self.op.empty(self.n, mrhs.DTYPE_F32)
            self.status = torch.zeros(1, dtype=torch.int32, device="cuda")
            nc = 2 * self.n
            self.Dc = torch.empty(self.op.n_agg * 9 * nc * nc * 2, dtype=torch.float32, device="cuda")

    def sap(self):
        mrhs.sap_smooth_mrhs(self.op.handle, self.b, self.x, self.n, N_SAP, N_MR, self.ws)

    def resid(self):
        mrhs.mrhs_residual_norms(self.op.handle, self.b, self.x, self.n, self.res, self.ws)

    def gs(self):
        mrhs.block_orthonormalize(self.op.handle, self.x, self.op.dtype, self.Q, mrhs.DTYPE_F32, self.n, self.status,
                                  self.ws)

    def dc(self):
        mrhs.coarse_op_build(self.op.handle, self.Q, mrhs.DTYPE_F32, self.n, self.Dc, self.ws)


def time_steps(setup, steps, warmup):
    """Returns per-step ms and per-part ms (HIP events on the stream the kernels use)."""
    parts = ["sap", "resid", "gs", "dc"]
    for _ in range(warmup):
        for p in parts:
            getattr(setup, p)()
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(len(parts) + 1)] for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        ev[s][0].record()
        for j, p in enumerate(parts):
            getattr(setup, p)()
            ev[s][j + 1].record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    per = {p: np.mean([ev[s][j].elapsed_time(ev[s][j + 1]) for s in range(steps)]) for j, p in enumerate(parts)}
    step = np.mean([ev[s][0].elapsed_time(ev[s][-1]) for s in range(steps)])
    return step, wall, per


def time_call(fn, reps, warmup=2):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def eo_bench(U, v, plain_ms, plain_res, reps=10):
    """SAP with the even-odd block solver (MR on each block's even-site Schur complement) on
    the same workload: time and the largest relative residual ||b - D x|| / ||b|| after the
    call, for n_MR = 2, 3, 4 (tile: the fastest of 1, 2, 4 at n_MR = 4), beside plain MR."""
    s = Setup(U, v, mrhs.PREC_F32, 4, gs=False)
    mrhs.mrhs_set_block_solver(s.op.handle, mrhs.BLOCK_EO_MR)
    best = None
    for tile in (1, 2, 4):
        mrhs.mrhs_set_tiles(s.op.handle, tile, 0)
        ms = time_call(s.sap, reps)
        if best is None or ms < best[1]:
            best = (tile, ms)
    mrhs.mrhs_set_tiles(s.op.handle, best[0], 0)
    out = {"tile": best[0], "plain_mr": {"n_mr": N_MR, "ms": round(plain_ms, 4), "residual_max": plain_res}}
    for n_mr in (2, 3, 4):
        fn = lambda: mrhs.sap_smooth_mrhs(s.op.handle, s.b, s.x, s.n, N_SAP, n_mr, s.ws)
        ms = time_call(fn, reps)
        fn()
        s.resid()
        torch.cuda.synchronize()
        out["eo_n_mr_%d" % n_mr] = {"ms": round(ms, 4), "residual_max": float(s.res.max().item())}
    s.op.close()
    return out


BATCH = [([8, 8, 8, 8], 401, 8), ([12, 12, 12, 12], 411, 16), ([16, 16, 16, 32], 421, 24), ([24, 24, 24, 48], 431, 32)]


def batched_bench(reps=5):
    """Uneven lattices, each with its own test vectors, FP32, 3 x 4: one batched call (one
    launch per half-sweep for all four), the same work as four separate calls, and the
    batched call replayed from a captured graph."""
    ops, bs, xs, ns, upd = [], [], [], [], 0
    for (Lb, seed, n) in BATCH:
        U = inputs.gauge_field(Lb, SIGMA, seed)
        v = inputs.test_vectors(Lb, n, seed + 1)
        op = mrhs.Operator(Lb, BLOCK, BLOCK, torch.from_numpy(U), M0, CSW, prec=mrhs.PREC_F32, short_len=4)
        ops.append(op)
        bs.append(op.pack(torch.from_numpy(v)))
        xs.append(op.empty(n))
        ns.append(n)
        upd += int(np.prod(Lb)) * n * N_SAP
    handles = [op.handle for op in ops]
    ws = torch.empty(max(256, mrhs.mrhs_batched_workspace_bytes(handles, ns)), dtype=torch.uint8, device="cuda")
    wss = [op.workspace(n) for op, n in zip(ops, ns)]
    batched = lambda: mrhs.sap_smooth_mrhs_batched(handles, bs, xs, ns, N_SAP, N_MR, ws)
    t_b = time_call(batched, reps)

    def seq():
        for op, b, x, n, w in zip(ops, bs, xs, ns, wss):
            mrhs.sap_smooth_mrhs(op.handle, b, x, n, N_SAP, N_MR, w)
    t_s = time_call(seq, reps)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            mrhs.sap_smooth_mrhs_batched(handles, bs, xs, ns, N_SAP, N_MR, ws, stream=s)
    torch.cuda.current_stream().wait_stream(s)
    t_g = time_call(g.replay, reps)
    for op in ops:
        op.close()
    return {"lattices": [b[0] for b in BATCH], "n_tv": ns, "site_rhs_updates": upd,
            "batched_ms": round(t_b, 4), "separate_calls_ms": round(t_s, 4), "graph_replay_ms": round(t_g, 4),
            "batched_updates_per_s": upd / (t_b * 1e-3), "graph_updates_per_s": upd / (t_g * 1e-3)}


def coarse_grid_bench(mr, reps=20):
    """The coarse-grid correction's building blocks (refinement phase, Alg. 2) on the step's
    Q and D_c, applied to the N_tv test vectors at once: restriction (Alg. 3), prolongation
    and the coarse-operator apply.  Algorithmic bytes: restriction and prolongation read Q
    and the fine vectors (or write them) once, FP32; the coarse apply reads D_c once and the
    coarse vectors of the site and its 8 neighbours."""
    op, n = mr.op, mr.n
    yc, zc = op.coarse_empty(n, n), op.coarse_empty(n, n)
    y = op.empty(n)
    mrhs.restrict_mrhs(op.handle, mr.Q, mrhs.DTYPE_F32, n, mr.x, op.dtype, yc, n)
    t_r = time_call(lambda: mrhs.restrict_mrhs(op.handle, mr.Q, mrhs.DTYPE_F32, n, mr.x, op.dtype, yc, n), reps)
    t_p = time_call(lambda: mrhs.prolong_mrhs(op.handle, mr.Q, mrhs.DTYPE_F32, n, yc, y, op.dtype, n), reps)
    t_a = time_call(lambda: mrhs.coarse_apply_mrhs(op.handle, mr.Dc, n, yc, zc, n), reps)
    V = int(np.prod(L))
    fine = V * 24 * 4 * n                       # n FP32 fine vectors
    coarse = op.n_agg * 2 * n * 2 * 4 * n       # n FP32 coarse vectors
    dcb = op.n_agg * 9 * (2 * n) ** 2 * 8
    out = {}
    # FP16 storage of Q (reduced-precision test vectors for R, P and D_c; FP32 arithmetic)
    D16 = mrhs.DTYPE_F16
    q16 = op.empty(n, D16)
    mrhs.block_orthonormalize(op.handle, mr.x, op.dtype, q16, D16, n, None, None)
    t_r16 = time_call(lambda: mrhs.restrict_mrhs(op.handle, q16, D16, n, mr.x, op.dtype, yc, n), reps)
    t_p16 = time_call(lambda: mrhs.prolong_mrhs(op.handle, q16, D16, n, yc, y, op.dtype, n), reps)
    dc16 = torch.empty_like(mr.Dc)
    t_dc32 = time_call(lambda: mrhs.coarse_op_build(op.handle, mr.Q, mrhs.DTYPE_F32, n, dc16, None), 5)
    t_dc16 = time_call(lambda: mrhs.coarse_op_build(op.handle, q16, D16, n, dc16, None), 5)
    for name, ms, b in (("restrict", t_r, 2 * fine + coarse), ("prolong", t_p, 2 * fine + coarse),
                        ("coarse_apply", t_a, dcb + 10 * coarse),
                        ("restrict_q16", t_r16, 1.5 * fine + coarse), ("prolong_q16", t_p16, 1.5 * fine + coarse)):
        out[name] = {"ms": round(ms, 4), "alg_GBs": round(b / ms / 1e6, 1), "frac_hbm": round(b / ms / 1e6 / HBM_PEAK_GBS, 4)}
    out["coarse_op_build_ms"] = {"q_fp32": round(t_dc32, 4), "q_fp16": round(t_dc16, 4)}
    return out


def refinement_bench(mr, m=8, tol=0.05, reps=10):
    """The refinement phase (Alg. 2 with N_b = N_tv): one pass = coarse-grid correction of
    all test vectors (restrict, GMRES to tol, prolong), SAP from it, then the new R and D_c.
    Also the paper's MRHS-vs-SRHS comparison for the coarse solve and the restriction: the
    same calls on one right-hand side at a time, looped over the test vectors."""
    op, n = mr.op, mr.n
    D32 = mrhs.DTYPE_F32
    ws = torch.empty(mrhs.mrhs_refine_workspace_bytes(op.handle, n, m), dtype=torch.uint8, device="cuda")
    V = op.empty(n)
    V.copy_(mr.x)

    def refine():
        mrhs.setup_refine_mrhs(op.handle, V, n, mr.Q, D32, mr.Dc, N_SAP, N_MR, m, tol, ws)

    def rebuild():
        mrhs.block_orthonormalize(op.handle, V, op.dtype, mr.Q, D32, n, mr.status, mr.ws)
        mrhs.coarse_op_build(op.handle, mr.Q, D32, n, mr.Dc, mr.ws)

    t_refine = time_call(refine, reps)
    t_pass = time_call(lambda: (refine(), rebuild()), reps)
    # coarse solve: all right-hand sides at once vs one at a time
    bc, uc = op.coarse_empty(n, n), op.coarse_empty(n, n)
    mrhs.restrict_mrhs(op.handle, mr.Q, D32, n, V, op.dtype, bc, n)
    its = torch.zeros(n, dtype=torch.int32, device="cuda")
    res = torch.zeros(n, dtype=torch.float64, device="cuda")
    gws = torch.empty(mrhs.mrhs_coarse_solve_workspace_bytes(op.handle, n, n, m), dtype=torch.uint8, device="cuda")
    t_cs = time_call(lambda: mrhs.coarse_solve_mrhs(op.handle, mr.Dc, n, bc, uc, n, m, tol, gws, res, its), reps)
    b1, u1 = op.coarse_empty(n, 1), op.coarse_empty(n, 1)
    gws1 = torch.empty(mrhs.mrhs_coarse_solve_workspace_bytes(op.handle, n, 1, m), dtype=torch.uint8, device="cuda")
    t_cs1 = time_call(lambda: [mrhs.coarse_solve_mrhs(op.handle, mr.Dc, n, b1, u1, 1, m, tol, gws1) for _ in range(n)],
                      max(2, reps // 4))
    t_r = time_call(lambda: mrhs.restrict_mrhs(op.handle, mr.Q, D32, n, V, op.dtype, bc, n), reps)
    y1 = op.empty(1)
    t_r1 = time_call(lambda: [mrhs.restrict_mrhs(op.handle, mr.Q, D32, n, y1, op.dtype, b1, 1) for _ in range(n)],
                     max(2, reps // 4))
    # the true relative residual ||b - D_c u|| / ||b|| per right-hand side of a coarse solution
    zc = op.coarse_empty(n, n)

    def true_res(u):
        mrhs.coarse_apply_mrhs(op.handle, mr.Dc, n, u, zc, n)
        ldc = (n + 3) // 4 * 4
        r = (bc - zc).view(-1, ldc).double()
        return float((r.pow(2).sum(0).sqrt() / bc.view(-1, ldc).double().pow(2).sum(0).sqrt())[:n].max().item())

    mrhs.coarse_solve_mrhs(op.handle, mr.Dc, n, bc, uc, n, m, tol, gws, res, its)
    true_plain = true_res(uc)
    # even-odd preconditioned coarse solve on the same system (GMRES on the even-site Schur
    # complement; the coarse extents 16 / 4 = 4 are even)
    Dinv = torch.empty(op.n_agg * (2 * n) ** 2 * 2, dtype=torch.float32, device="cuda")
    t_inv = time_call(lambda: mrhs.coarse_self_invert(op.handle, mr.Dc, n, Dinv), reps)
    its_eo = torch.zeros(n, dtype=torch.int32, device="cuda")
    res_eo = torch.zeros(n, dtype=torch.float64, device="cuda")
    gws_eo = torch.empty(mrhs.mrhs_coarse_solve_eo_workspace_bytes(op.handle, n, n, m), dtype=torch.uint8, device="cuda")
    t_cs_eo = time_call(lambda: mrhs.coarse_solve_eo_mrhs(op.handle, mr.Dc, Dinv, n, bc, uc, n, m, tol, gws_eo, res_eo,
                                                          its_eo), reps)
    true_eo = true_res(uc)
    torch.cuda.synchronize()
    return {"gmres_max_iter": m, "tol": tol, "iterations_needed": int(its.max().item()),
            "coarse_residual_max": float(res.max().item()), "coarse_true_residual_max": true_plain,
            "coarse_solve_eo_ms": round(t_cs_eo, 4), "coarse_self_invert_ms": round(t_inv, 4),
            "eo_iterations_needed": int(its_eo.max().item()), "eo_schur_residual_max": float(res_eo.max().item()),
            "eo_true_residual_max": true_eo,
            "refine_ms": round(t_refine, 4), "refine_pass_with_rebuild_ms": round(t_pass, 4),
            "refine_site_rhs_per_s": int(np.prod(L)) * n * N_SAP / (t_pass * 1e-3),
            "coarse_solve_mrhs_ms": round(t_cs, 4), "coarse_solve_srhs_looped_ms": round(t_cs1, 4),
            "coarse_solve_speedup": round(t_cs1 / t_cs, 2),
            "restrict_mrhs_ms": round(t_r, 4), "restrict_srhs_looped_ms": round(t_r1, 4),
            "restrict_speedup": round(t_r1 / t_r, 2)}


def cpu_baseline(U, v, x_gpu, budget_s=30.0):
    """The oracle on the host cores: SAP on a sample of test vectors (they are independent),
    Gram-Schmidt on all aggregates, D_c on a sample of aggregates; scaled to the full step."""
    import oracle
    cores = min(len(os.sched_getaffinity(0)), int(os.environ.get("OMP_NUM_THREADS", "1000")))
    os.environ.setdefault("OMP_NUM_THREADS", str(cores))
    t = time.perf_counter()
    A = oracle.clover(L, U, CSW, M0)
    t_clover = time.perf_counter() - t
    n_s = 2
    t = time.perf_counter()
    xs = oracle.sap(L, BLOCK, U, A, v[:n_s], N_SAP, N_MR)
    t_sap = (time.perf_counter() - t) * N_TV / n_s
    t = time.perf_counter()
    oracle.residual_norms(L, U, A, v[:n_s], xs)
    t_res = (time.perf_counter() - t) * N_TV / n_s
    t = time.perf_counter()
    Q = oracle.block_gs(L, AGG, x_gpu)
    t_gs = time.perf_counter() - t
    n_agg = oracle.n_aggregates(L, AGG)
    sample = list(range(0, n_agg, n_agg // 8))[:8]
    t = time.perf_counter()
    oracle.coarse_op(L, AGG, U, A, Q, agg_list=sample)
    t_dc = (time.perf_counter() - t) * n_agg / len(sample)
    total = t_sap + t_res + t_gs + t_dc
    V = int(np.prod(L))
    return {
        "value": V * N_TV * N_SAP / total,
        "unit": "site*RHS updates/s",
        "cores": cores,
        "kind": "oracle",
        "sample": ("SAP + residual on %d of %d test vectors (scaled x%d), block GS on all %d aggregates, "
                   "D_c on %d of %d aggregates (scaled); op set-up (%.1f s) excluded; FP64 C, OpenMP"
                   % (n_s, N_TV, N_TV // n_s, n_agg, len(sample), n_agg, t_clover)),
        "seconds": {"sap": t_sap, "resid": t_res, "gs": t_gs, "dc": t_dc},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-srhs", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-refine", action="store_true")
    ap.add_argument("--no-eo", action="store_true")
    ap.add_argument("--copy-calib", action="store_true", help="only run a plain 1 GiB device copy (counter scale)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only (the path would shard by domain decomposition; "
              "no multi-GPU run is implemented)", file=sys.stderr)
        sys.exit(2)
    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_calib:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": a.numel() * 4, "copy_bytes_written": a.numel() * 4}))
        return

    V = int(np.prod(L))
    log("generating inputs")
    U, v = make_inputs("cuda")
    log("operator set-up")
    mr = Setup(U, v, mrhs.PREC_F32, 4)
    tiles = autotune.autotune(mr.op, N_TV, N_SAP, N_MR)
    log("autotuned tiles: %s" % tiles)
    log("timing %d steps after %d warm-up" % (args.steps, args.warmup))
    step_ms, wall_ms, per = time_steps(mr, args.steps, args.warmup)
    assert int(mr.status.item()) == 0
    res = mr.res.cpu().numpy()
    log("step %.3f ms (wall %.3f): %s; residuals %.4f..%.4f" % (step_ms, wall_ms, per, res.min(), res.max()))

    value = V * N_TV * N_SAP / (step_ms * 1e-3)
    # dominant kernel: the SAP half-sweep (2 * N_SAP launches per call)
    n_launch = 2 * N_SAP
    sap_launch_ms = per["sap"] / n_launch
    flops_launch = sap_flops_per_call(V, N_TV, N_SAP, N_MR, BLOCK) / n_launch
    achieved = flops_launch / (sap_launch_ms * 1e-3) / 1e12
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved / FP32_VECTOR_PEAK_TFLOPS, 4), "traffic": sap_traffic_bytes(tiles["sap"]),
            "traffic_unit": "bytes per launch (HBM, counters)", "alg_bytes": round(sap_bytes_per_call(V, N_TV, N_SAP, 4, 4) / n_launch),
            "kernel": "k_sap_batched (FP32, tile %d)" % tiles["sap"], "launch_ms": round(sap_launch_ms, 4),
            "frac_of_issue_peak": round(achieved / FP32_ISSUE_PEAK_TFLOPS, 4)}

    # stencil HBM roofline (the HBM-bound kernel of the path)
    y = mr.op.empty(N_TV)
    d_ms = time_call(lambda: mrhs.dirac_apply_mrhs(mr.op.handle, mr.b, y, N_TV), 20)
    d_bytes = V * N_TV * pm.stencil_bytes_per_site_rhs(N_TV, 4, 4)
    stencil = {"kernel": "k_dirac (FP32, 20 RHS, tile %d)" % tiles["dirac"], "ms": round(d_ms, 4), "GBs": round(d_bytes / d_ms / 1e6, 1),
               "frac_hbm": round(d_bytes / d_ms / 1e6 / HBM_PEAK_GBS, 4),
               "site_rhs_per_s": V * N_TV / (d_ms * 1e-3)}
    sap_bytes = sap_bytes_per_call(V, N_TV, N_SAP, 4, 4)
    sap_info = {"ms_per_call": round(per["sap"], 4), "alg_GBs": round(sap_bytes / per["sap"] / 1e6, 1),
                "alg_tflops": round(sap_flops_per_call(V, N_TV, N_SAP, N_MR, BLOCK) / per["sap"] / 1e9, 3)}

    srhs = None
    if not args.no_srhs:
        log("single-RHS FP64 and MRHS FP64 paths")
        s1 = Setup(U, v[:1], mrhs.PREC_F64, 1, gs=False)
        srhs_ms = time_call(s1.sap, 5) * N_TV     # the same SAP, one vector per call, looped
        m64 = Setup(U, v, mrhs.PREC_F64, 4, gs=False)
        mrhs.mrhs_set_tiles(m64.op.handle, 2, 0)
        m64_ms = time_call(m64.sap, 5)
        srhs = {"srhs_fp64_sap_ms": round(srhs_ms, 3), "mrhs_fp64_sap_ms": round(m64_ms, 3),
                "mrhs_fp32_sap_ms": round(per["sap"], 3),
                "speedup_equal_precision": round(srhs_ms / m64_ms, 2),
                "speedup_run_precision": round(srhs_ms / per["sap"], 2)}
        log("srhs %s" % srhs)
        s1.op.close()
        m64.op.close()

    log("coarse-grid building blocks")
    coarse_grid = coarse_grid_bench(mr)
    log("coarse grid %s" % coarse_grid)

    eo = None
    if not args.no_eo:
        log("even-odd block solver")
        eo = eo_bench(U, v, per["sap"], float(res.max()))
        log("eo %s" % eo)

    refinement = None
    if not args.no_refine:
        log("refinement phase")
        refinement = refinement_bench(mr)
        log("refinement %s" % refinement)

    batched = None
    if not args.no_batched:
        log("batched uneven lattices")
        batched = batched_bench()
        log("batched %s" % batched)

    cpu = None
    if not args.no_cpu_baseline:
        log("CPU oracle baseline")
        x_gpu = mr.op.unpack(mr.x, N_TV).cpu().numpy()
        cpu = cpu_baseline(U, v, x_gpu)
        log("cpu %s" % cpu)

    out = {
        "metric": "MRHS SAP setup: site*RHS updates/s and HBM GB/s vs single-RHS, same accuracy",
        "value": value,
        "unit": "site*RHS updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "lattice": L, "n_tv": N_TV, "sap": [N_SAP, N_MR], "block": BLOCK,
                   "aggregate": AGG, "parallelism": "single GPU",
                   "tiles": {"sap": tiles["sap"], "dirac": tiles["dirac"]}},
        "parts_ms": {k: round(float(x), 4) for k, x in per.items()},
        "residual_max": float(res.max()),
        "roofline": roof,
        "stencil_roofline": stencil,
        "sap": sap_info,
        "srhs": srhs,
        "coarse_grid": coarse_grid,
        "even_odd_block_solver": eo,
        "refinement": refinement,
        "batched": batched,
        "cpu_baseline": cpu,
    }
    mr.op.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
