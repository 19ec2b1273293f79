"""Benchmark of the MRHS setup path on one MI355X.

One step = the initial setup phase on all test vectors at once, inputs resident in HBM:
  sap_smooth_mrhs      SAP from x = 0 on N_tv vectors (FP32),
  mrhs_residual_norms  FP64 check ||b - D x|| / ||b|| per vector,
  block_orthonormalize FP64 block Gram-Schmidt on the aggregates -> Q (FP32),
  coarse_op_build      D_c (9 blocks of 2N_tv x 2N_tv complex64 per coarse site).
Workload (the headline): 48^3 x 96 Wilson-clover lattice (synthetic links, sigma = 0.2),
m0 = -0.34, csw = 1, N_tv = 32 complex Gaussian test vectors, 4^4 SAP blocks and
aggregates, 3 SAP sweeps x 4 MR steps -- the lattice shape and domain size of the paper's
C101 runs (Sec. 7), with synthetic links standing in for the ensemble.

Prints one JSON line.  value = site-RHS updates per second of the whole step
(V * N_tv * n_SAP / step time).  Also reports: the roofline of the dominant kernel (the
SAP half-sweep, FP32 ALU bound) with HIP-event timing over the timed region, the
stencil's HBM roofline, a plain device copy as the practical HBM ceiling, the relative
error of every result against the FP64 oracle on sampled outputs, FP16 vector storage
on the 32^3 x 64 workload, the single-RHS FP64 GPU path for the same SAP (speedup),
the 16^4 extras (refinement phase, even-odd block solver, coarse-grid kernels, batched
uneven lattices) and the CPU oracle on a bounded sample (baseline only).
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

BLOCK = [4, 4, 4, 4]
AGG = [4, 4, 4, 4]
CSW = 1.0
N_SAP, N_MR = 3, 4
S = 4
C5 = dict(L=[48, 48, 48, 96], sigma=0.2, m0=-0.34, n_tv=32, seed_u=501, seed_v=502)
C3 = dict(L=[32, 32, 32, 64], sigma=0.25, m0=-0.33, n_tv=24, seed_u=301, seed_v=302)
C2 = dict(L=[16, 16, 16, 16], sigma=0.3, m0=-0.3, n_tv=20, seed_u=201, seed_v=202)
HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3      # published, with packed FP32 FMA
FP32_ISSUE_PEAK_TFLOPS = 78.6        # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz, no packed FP32
TOL = {"f32": 1e-5, "f16_storage": 5e-3, "f64": 1e-12}

# HBM traffic of the dominant kernel (SAP half-sweep, 48^3 x 96, N_tv 32, FP32), per launch
# and execution tile: rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE (KiB per dispatch, mean over
# the half-sweeps of the bench's calls), each scaled by what the counter reads for a plain
# device copy (FETCH x2.0, WRITE x1.0).  Valid only for the kernel sources they were taken
# with (SHA-1 of the files below); otherwise the bench reports traffic as null.
SAP_SOURCES = ["paper_1601_03184_amd/csrc/sap.hip", "paper_1601_03184_amd/csrc/stencil.h",
               "paper_1601_03184_amd/csrc/internal.h"]
SAP_TRAFFIC = {"sources_sha1": "e995143935673a2b9ee3cbc50ac794ba20eabc0a", "fetch_scale": 2.0, "write_scale": 1.0,
               "kib": {4: (37813987, 39813120)}}


def sources_sha1():
    h = hashlib.sha1()
    for f in SAP_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def sap_traffic_bytes(tile):
    if sources_sha1() != SAP_TRAFFIC["sources_sha1"] or tile not in SAP_TRAFFIC["kib"]:
        return None
    fk, wk = SAP_TRAFFIC["kib"][tile]
    return (fk * SAP_TRAFFIC["fetch_scale"] + wk * SAP_TRAFFIC["write_scale"]) * 1024


def workload_name(c):
    return ("%s Wilson-clover (sigma=%g links, m0=%g, csw=1), N_tv=%d, SAP 4^4 blocks %dx%d FP32, "
            "FP64 residual check, FP64 block Gram-Schmidt on 4^4 aggregates, D_c FP32"
            % ("x".join(map(str, c["L"])), c["sigma"], c["m0"], c["n_tv"], N_SAP, N_MR))


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def sap_flops_per_call(V, n, n_sap, n_mr, block):
    """Arithmetic the SAP call performs: the block-operator MR steps on every site, and the
    residual where x is not known to vanish, which is only the hops across block faces (in the
    first black half-sweep x vanishes on the block itself; at every later visit the block's
    residual is kept from its previous one and the face hops of the neighbours' changes of x
    are subtracted)."""
    Vb = int(np.prod(block))
    inner = sum((Vb - Vb // b) for b in block) * 2 / (8.0 * Vb)   # fraction of hops inside a block
    hop = 1320.0
    rest = pm.STENCIL_FLOP - hop
    mr = n_mr * (rest + hop * inner + pm.MR_EXTRA_FLOP)
    face_res = hop * (1 - inner) + pm.RESIDUAL_EXTRA_FLOP
    half = V / 2.0 * n
    total = 0.0
    for sweep in range(n_sap):
        for c in range(2):
            total += half * (mr + (face_res if sweep > 0 or c == 1 else 0.0))
    return total


def sap_bytes_per_call(V, n, n_sap, store_b, field_b, sigma_b=4):
    """Algorithmic HBM bytes of a SAP call: per half-sweep the fields of that colour's sites
    once; in the first sweep b read, in later ones the kept block residual (arithmetic type)
    and the own x read; x written; the other colour's x (first black half-sweep) or change of x
    (later visits) that the face hops read, counted once per site; the block residual and the
    change of x written where a later visit reads them."""
    half = V // 2
    s = pm.SPINOR_REALS * store_b
    sg = pm.SPINOR_REALS * sigma_b
    f = (4 * pm.LINK_REALS + pm.CLOVER_REALS) * field_b
    total = 0.0
    for sweep in range(n_sap):
        for c in range(2):
            total += half * f
            total += half * n * s                         # x written
            if sweep == 0:
                total += half * n * s                     # b read
            else:
                total += half * n * (sg + s)              # block residual and the own x read
            if sweep == 0 and c == 1:
                total += half * n * s                     # the other colour's x
            elif sweep > 0:
                total += half * n * sg                    # the other colour's change of x
            if sweep + 1 < n_sap:
                total += half * n * sg                    # block residual written
            if not (sweep + 1 == n_sap and c == 1):
                total += half * n * sg                    # change of x written
    return total


def group_view(op, native, g):
    """The native storage of right-hand sides g*S .. g*S + S - 1 (one contiguous group)."""
    ge = 24 * op.V * op.S
    return native[g * ge:(g + 1) * ge]


def pack_device(op, native, dtype, cfg, n):
    """Pack the seeded test vectors of a workload, one group of S at a time (the canonical
    complex128 vectors of the whole set would not fit beside the native ones)."""
    for g in range((n + op.S - 1) // op.S):
        m = min(op.S, n - g * op.S)
        canon = inputs.test_vectors_device(cfg["L"], m, cfg["seed_v"], "cuda", first=g * op.S)
        mrhs.mrhs_pack(op.handle, torch.view_as_real(canon), group_view(op, native, g), dtype, m)
        del canon


def gather_sites(op, native, dtype, n, sites):
    """canonical complex128 [n][len(sites)][4][3] of all right-hand sides at some sites (host)"""
    idx = torch.as_tensor(np.asarray(sites), device="cuda")
    out = []
    for g in range((n + op.S - 1) // op.S):
        m = min(op.S, n - g * op.S)
        buf = torch.zeros((m, op.V, 4, 3, 2), dtype=torch.float64, device="cuda")
        mrhs.mrhs_unpack(op.handle, group_view(op, native, g), dtype, buf, m)
        out.append(torch.view_as_complex(buf[:, idx]).cpu().numpy())
        del buf
    return np.concatenate(out, axis=0)


def unpack_rhs(op, native, dtype, n, k):
    """canonical complex128 [V][4][3] of right-hand side k (host)"""
    g, t = divmod(k, op.S)
    m = min(op.S, n - g * op.S)
    out = torch.zeros((m, op.V, 4, 3, 2), dtype=torch.float64, device="cuda")
    mrhs.mrhs_unpack(op.handle, group_view(op, native, g), dtype, out, m)
    return torch.view_as_complex(out[t]).cpu().numpy()


def agg_site_index(L, a, i, window=1):
    """canonical site indices of aggregate i (local sites lexicographic); with window = 3,
    of the 3^4 aggregates centred on it (window sites lexicographic, periodic)."""
    na = [L[m] // a[m] for m in range(4)]
    ac, r = [], i
    for m in range(4):
        ac.append(r % na[m])
        r //= na[m]
    ext = [window * a[m] for m in range(4)]
    w = np.indices(ext[::-1]).reshape(4, -1)[::-1]  # x fastest
    x = [(w[m] + (ac[m] - (window // 2)) * a[m]) % L[m] for m in range(4)]
    return x[0] + L[0] * (x[1] + L[1] * (x[2] + L[2] * x[3]))


class Setup:
    """One workload's operator, test vectors and outputs, all in HBM."""

    def __init__(self, cfg, U, prec=mrhs.PREC_F32, n=None, short_len=S, gs=True):
        self.cfg = cfg
        self.n = cfg["n_tv"] if n is None else n
        self.op = mrhs.Operator(cfg["L"], BLOCK, AGG, U, cfg["m0"], CSW, prec=prec, short_len=short_len)
        self.b = self.op.empty(self.n)
        pack_device(self.op, self.b, self.op.dtype, cfg, self.n)
        self.x = self.op.empty(self.n)
        self.ws = self.op.workspace(self.n)
        self.res = torch.empty(self.n, dtype=torch.float64, device="cuda")
        self.status = torch.zeros(1, dtype=torch.int32, device="cuda")
        if gs:
            self.Q = self.op.empty(self.n, mrhs.DTYPE_F32)
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

    def close(self):
        self.op.close()
        for a in ("b", "x", "ws", "Q", "Dc"):
            if hasattr(self, a):
                delattr(self, a)


def average_plaquette(U, L):
    """Sanity statistic of a gauge field (not part of the path): the mean over sites and the six
    planes mu < nu of Re tr(U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag) / 3, evaluated as
    Re tr(P Q^dag) with P = U_mu(x) U_nu(x+mu) and Q = U_nu(x) U_mu(x+nu).  U: complex [4][V][3][3],
    canonical site order (x fastest); 1 for unit links."""
    Ul = U.reshape(4, L[3], L[2], L[1], L[0], 3, 3)
    axis = {0: 3, 1: 2, 2: 1, 3: 0}  # lattice direction -> tensor axis of Ul[mu]
    total = 0.0
    for mu in range(4):
        for nu in range(mu + 1, 4):
            P = torch.matmul(Ul[mu], torch.roll(Ul[nu], shifts=-1, dims=axis[mu]).contiguous())
            Q = torch.matmul(Ul[nu], torch.roll(Ul[mu], shifts=-1, dims=axis[nu]).contiguous())
            total += float((P * Q.conj()).real.sum().item())
            del P, Q
    return total / (3.0 * 6.0 * U.shape[1])


def platform():
    """What the numbers were measured on: device, HIP runtime, and the shader clock if rocm-smi
    reports it."""
    prop = torch.cuda.get_device_properties(0)
    out = {"device": prop.name, "arch": getattr(prop, "gcnArchName", None), "compute_units": prop.multi_processor_count,
           "hip": torch.version.hip, "torch": torch.__version__}
    if any(k.startswith("ROCPROF") for k in os.environ):
        # under rocprofv3 the tool's library is loaded into every child as well, and rocm-smi
        # re-executes its interpreter after that library has opened the GPU: not queried
        return out
    try:
        import subprocess
        r = subprocess.run(["rocm-smi", "--showclocks", "--json"], capture_output=True, text=True, timeout=20)
        clocks = json.loads(r.stdout) if r.returncode == 0 else None
        if clocks:
            card = next(iter(clocks.values()))
            out["sclk"] = card.get("sclk clock speed:") or card.get("sclk")
    except Exception:  # a missing or slow rocm-smi leaves the clock unrecorded
        pass
    return out


def time_steps(setup, steps, warmup):
    """Returns per-step ms (mean), wall ms, per-part ms and the median, min and max of the
    steps (HIP events on the stream the kernels use)."""
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
        if steps > 1 and s == 0:
            log("first timed step enqueued")
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    per = {p: float(np.mean([ev[s][j].elapsed_time(ev[s][j + 1]) for s in range(steps)])) for j, p in enumerate(parts)}
    each = [ev[s][0].elapsed_time(ev[s][-1]) for s in range(steps)]
    spread = {"median": float(np.median(each)), "min": float(np.min(each)), "max": float(np.max(each))}
    return float(np.mean(each)), wall, per, spread


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


def copy_ceiling(gib=4, reps=10):
    """A plain device-to-device copy (torch's copy kernel): the practical HBM ceiling."""
    a = torch.empty(gib << 28, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    ms = time_call(lambda: b.copy_(a), reps)
    gbs = 2 * a.numel() * 4 / ms / 1e6
    del a, b
    return {"bytes_moved": 2 * (gib << 30), "ms": round(ms, 4), "GBs": round(gbs, 1),
            "frac_of_datasheet": round(gbs / HBM_PEAK_GBS, 4)}


# ------------------------------------------------------------------------------------------
# the extras on the 16^4 workload (refinement phase, even-odd block solver, coarse-grid
# kernels) and the batch of uneven lattices
# ------------------------------------------------------------------------------------------

def eo_bench(U, cfg, plain_ms, plain_res, reps=10):
    """SAP with the even-odd block solver (MR on each block's even-site Schur complement) on
    the same workload: time and the largest relative residual ||b - D x|| / ||b|| after the
    call, for n_MR = 2, 3, 4 (tile: the fastest of 1, 2, 4 at n_MR = 4), beside plain MR."""
    s = Setup(cfg, U, gs=False)
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
    s.close()
    return out


BATCH = [([8, 8, 8, 8], 401, 8), ([12, 12, 12, 12], 411, 16), ([16, 16, 16, 32], 421, 24), ([24, 24, 24, 48], 431, 32)]


def batched_bench(reps=5):
    """Uneven lattices, each with its own test vectors, FP32, 3 x 4: one batched call (one
    launch per half-sweep for all four), the same work as four separate calls, and the
    batched call replayed from a captured graph."""
    ops, bs, xs, ns, upd = [], [], [], [], 0
    for (Lb, seed, n) in BATCH:
        U = inputs.gauge_field(Lb, 0.3, seed)
        v = inputs.test_vectors(Lb, n, seed + 1)
        op = mrhs.Operator(Lb, BLOCK, BLOCK, torch.from_numpy(U), -0.3, CSW, prec=mrhs.PREC_F32, short_len=4)
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
    V = op.V
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
    zc = op.coarse_empty(n, n)

    def true_res(u):
        """the true relative residual ||b - D_c u|| / ||b|| per right-hand side, max"""
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
            "refine_site_rhs_per_s": op.V * n * N_SAP / (t_pass * 1e-3),
            "coarse_solve_mrhs_ms": round(t_cs, 4), "coarse_solve_srhs_looped_ms": round(t_cs1, 4),
            "coarse_solve_speedup": round(t_cs1 / t_cs, 2),
            "restrict_mrhs_ms": round(t_r, 4), "restrict_srhs_looped_ms": round(t_r1, 4),
            "restrict_speedup": round(t_r1 / t_r, 2)}


def coarse_grid_c5(mr, m=8, tol=0.05, reps=5):
    """The coarse grid of the headline workload (41472 coarse sites, 2 N_tv = 64 dof): the
    coarse-operator apply on the N_tv restricted test vectors and the low-accuracy coarse
    GMRES (m = 8, tolerance 0.05), with D_c (and the Krylov basis) in FP32 and in binary16
    (the half-precision coarse grid); the GMRES also replayed from a captured graph.
    Algorithmic bytes of an apply: D_c once plus the vectors of a site and its 8 neighbours
    (read once, written once: 2 x the coarse vectors, the neighbours' from cache)."""
    op, n = mr.op, mr.n
    nc = 2 * n
    bc, uc, zc = op.coarse_empty(n, n), op.coarse_empty(n, n), op.coarse_empty(n, n)
    mrhs.restrict_mrhs(op.handle, mr.Q, mrhs.DTYPE_F32, n, mr.x, op.dtype, bc, n)
    D16 = torch.empty(op.n_agg * 9 * nc * nc * 2, dtype=torch.float16, device="cuda")
    t_b16 = time_call(lambda: mrhs.coarse_op_build_f16(op.handle, mr.Q, mrhs.DTYPE_F32, n, D16), 2, warmup=1)
    cvb = bc.numel() * 4
    out = {"coarse_op_build_f16_ms": round(t_b16, 3)}
    for name, D, app, dcb in (("f32", mr.Dc, mrhs.coarse_apply_mrhs, mr.Dc.numel() * 4),
                              ("f16", D16, mrhs.coarse_apply_f16_mrhs, D16.numel() * 2)):
        ms = time_call(lambda: app(op.handle, D, n, bc, zc, n), reps)
        byts = dcb + 2 * cvb
        out["apply_" + name] = {"ms": round(ms, 4), "alg_bytes": byts, "alg_GBs": round(byts / ms / 1e6, 1),
                                "frac_hbm": round(byts / ms / 1e6 / HBM_PEAK_GBS, 4)}
    for name, D, solve, wsf in (("f32", mr.Dc, mrhs.coarse_solve_mrhs, mrhs.mrhs_coarse_solve_workspace_bytes),
                                ("f16", D16, mrhs.coarse_solve_f16_mrhs, mrhs.mrhs_coarse_solve_f16_workspace_bytes)):
        ws = torch.empty(wsf(op.handle, n, n, m), dtype=torch.uint8, device="cuda")
        res = torch.zeros(n, dtype=torch.float64, device="cuda")
        its = torch.zeros(n, dtype=torch.int32, device="cuda")
        fn = lambda stream=None: solve(op.handle, D, n, bc, uc, n, m, tol, ws, res, its, stream=stream)
        ms = time_call(fn, reps)
        fn()
        torch.cuda.synchronize()
        it = int(its.max().item())
        # the true relative residual ||b - D_c u|| / ||b|| with the FP32 operator
        mrhs.coarse_apply_mrhs(op.handle, mr.Dc, n, uc, zc, n)
        ldc = (n + 3) // 4 * 4
        r = (bc - zc).view(-1, ldc).double()
        true = float((r.pow(2).sum(0).sqrt() / bc.view(-1, ldc).double().pow(2).sum(0).sqrt())[:n].max().item())
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        g = torch.cuda.CUDAGraph()
        with torch.cuda.stream(s):
            with torch.cuda.graph(g, stream=s):
                fn(stream=s)
        torch.cuda.current_stream().wait_stream(s)
        ms_g = time_call(g.replay, reps)
        out["gmres_" + name] = {"ms": round(ms, 3), "graph_replay_ms": round(ms_g, 3), "iterations": it,
                                "ms_per_iteration": round(ms / max(it, 1), 3),
                                "workspace_bytes": ws.numel(), "residual_estimate_max": float(res.max().item()),
                                "true_residual_max": true}
        del ws, g
    del D16
    torch.cuda.empty_cache()
    return out


def extras_16(args):
    """The 16^4 workload (N_tv 20): its step, and the extras built on it."""
    cfg = C2
    U = inputs.gauge_field_device(cfg["L"], cfg["sigma"], cfg["seed_u"], "cuda")
    mr = Setup(cfg, U)
    autotune.autotune(mr.op, mr.n, N_SAP, N_MR, b=mr.b, x=mr.x)
    step_ms, _, per, _ = time_steps(mr, 10, 3)
    mr.resid()
    res_max = float(mr.res.max().item())
    out = {"workload": workload_name(cfg), "step_ms": round(step_ms, 4),
           "parts_ms": {k: round(v, 4) for k, v in per.items()},
           "value": mr.op.V * mr.n * N_SAP / (step_ms * 1e-3), "residual_max": res_max}
    log("16^4 step %.3f ms %s" % (step_ms, per))
    out["coarse_grid"] = coarse_grid_bench(mr)
    if not args.no_eo:
        out["even_odd_block_solver"] = eo_bench(U, cfg, per["sap"], res_max)
    if not args.no_refine:
        out["refinement"] = refinement_bench(mr)
    mr.close()
    del U
    if not args.no_batched:
        out["batched"] = batched_bench()
    torch.cuda.empty_cache()
    return out


# ------------------------------------------------------------------------------------------
# the FP64 single-RHS path (speedup reference) and FP16 storage
# ------------------------------------------------------------------------------------------

def srhs_bench(cfg, U, mrhs_fp32_ms, n_sub=8):
    """SAP through the same kernels one right-hand side per call in FP64 (S = 1, tile 1;
    timed on one vector, scaled by N_tv), MRHS in FP64 (tile 2; timed on n_sub vectors,
    scaled by N_tv / n_sub: right-hand-side tiles are independent workgroups, so the time
    is linear in their number at this size), and the step's MRHS FP32 SAP."""
    n = cfg["n_tv"]
    s1 = Setup(cfg, U, prec=mrhs.PREC_F64, n=1, short_len=1, gs=False)
    t1 = time_call(s1.sap, 3, warmup=1)
    s1.close()
    torch.cuda.empty_cache()
    m64 = Setup(cfg, U, prec=mrhs.PREC_F64, n=n_sub, short_len=S, gs=False)
    mrhs.mrhs_set_tiles(m64.op.handle, 2, 0)
    t64 = time_call(m64.sap, 3, warmup=1)
    m64.close()
    torch.cuda.empty_cache()
    srhs_ms = t1 * n
    m64_ms = t64 * n / n_sub
    return {"srhs_fp64_sap_ms": round(srhs_ms, 3), "mrhs_fp64_sap_ms": round(m64_ms, 3),
            "mrhs_fp32_sap_ms": round(mrhs_fp32_ms, 3),
            "speedup_equal_precision": round(srhs_ms / m64_ms, 2),
            "speedup_run_precision": round(srhs_ms / mrhs_fp32_ms, 2),
            "sample": "single-RHS FP64 timed on 1 vector x %d; MRHS FP64 (tile 2) timed on %d vectors x %g"
                      % (n, n_sub, n / n_sub)}


def fp16_bench(cfg, k_sample, reps=5):
    """SAP with FP16 (binary16) vector storage and FP32 arithmetic beside FP32 storage on the
    32^3 x 64 workload; returns timings and the sampled right-hand side of each result."""
    U = inputs.gauge_field_device(cfg["L"], cfg["sigma"], cfg["seed_u"], "cuda")
    out, sample = {}, {}
    V, n = int(np.prod(cfg["L"])), cfg["n_tv"]
    for name, prec in (("f16_storage", mrhs.PREC_F32_F16STORE), ("f32", mrhs.PREC_F32)):
        s = Setup(cfg, U, prec=prec, gs=False)
        autotune.autotune(s.op, n, N_SAP, N_MR, b=s.b, x=s.x)
        ms = time_call(s.sap, reps, warmup=1)
        s.sap()
        s.resid()
        torch.cuda.synchronize()
        sb = 2 if prec == mrhs.PREC_F32_F16STORE else 4
        byts = sap_bytes_per_call(V, n, N_SAP, sb, 4)
        flops = sap_flops_per_call(V, n, N_SAP, N_MR, BLOCK)
        out[name] = {"sap_ms": round(ms, 3), "site_rhs_per_s": V * n * N_SAP / (ms * 1e-3),
                     "alg_GBs": round(byts / ms / 1e6, 1), "alg_tflops": round(flops / ms / 1e9, 3),
                     "residual_max": float(s.res.max().item())}
        sample[name] = unpack_rhs(s.op, s.x, s.op.dtype, n, k_sample)
        s.close()
        torch.cuda.empty_cache()
    out["speedup_f16_storage"] = round(out["f32"]["sap_ms"] / out["f16_storage"]["sap_ms"], 3)
    Uh = U.cpu().numpy()
    del U
    torch.cuda.empty_cache()
    return out, sample, Uh


# ------------------------------------------------------------------------------------------
# the oracle: relative errors per result and the CPU baseline
# ------------------------------------------------------------------------------------------

def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def per_half_rel(got, ref):
    """relative error per spin half of one aggregate ([n][Va][4][3]); the max of the two"""
    n = ref.shape[0]
    g = got.reshape(n, -1, 2, 6)
    r = ref.reshape(n, -1, 2, 6)
    return max(rel(g[:, :, h], r[:, :, h]) for h in range(2))


def oracle_checks(cfg, host, fp16=None):
    """The FP64 oracle on the sampled outputs of the step: relative errors per result, and
    its run time on that sample scaled to the whole step (the CPU baseline)."""
    import oracle
    cores = min(len(os.sched_getaffinity(0)), int(os.environ.get("OMP_NUM_THREADS", "1000")))
    os.environ.setdefault("OMP_NUM_THREADS", str(cores))
    L, n, m0 = cfg["L"], cfg["n_tv"], cfg["m0"]
    V = int(np.prod(L))
    n_agg = oracle.n_aggregates(L, AGG)
    t = time.perf_counter()
    A = oracle.clover(L, host["U"], CSW, m0)
    t_clover = time.perf_counter() - t
    k = host["k"]
    log("oracle: SAP of test vector %d" % k)
    t = time.perf_counter()
    xs = oracle.sap(L, BLOCK, host["U"], A, host["b_k"][None], N_SAP, N_MR)
    t_sap = (time.perf_counter() - t) * n
    # the residual check runs on the b the GPU holds (rounded once to FP32) and its x
    b32 = host["b_k"].astype(np.complex64).astype(np.complex128)
    t = time.perf_counter()
    r_or = oracle.residual_norms(L, host["U"], A, b32[None], host["x_k"][None])
    t_res = (time.perf_counter() - t) * n
    del A
    acc = {"sap_fp32": {"rel_err": rel(host["x_k"], xs[0]), "tol": TOL["f32"], "sample": "test vector %d" % k},
           "residual_fp64": {"rel_err": abs(host["res_k"] - r_or[0]) / r_or[0], "tol": TOL["f64"],
                             "value": float(r_or[0]), "sample": "test vector %d, the GPU's x" % k}}
    del xs
    log("oracle: Gram-Schmidt of %d aggregates" % len(host["gs_aggs"]))
    t = time.perf_counter()
    errs = []
    for j, i in enumerate(host["gs_aggs"]):
        ref = oracle.block_gs(AGG, AGG, host["gs_V"][:, j])
        errs.append(per_half_rel(host["gs_Q"][:, j], ref))
    t_gs = (time.perf_counter() - t) * n_agg / len(host["gs_aggs"])
    acc["gs_fp64_to_fp32_q"] = {"rel_err": max(errs), "tol": 1e-6,
                                "sample": "%d aggregates, per spin half (FP32 storage of Q: 1e-6)" % len(errs)}
    log("oracle: D_c of %d coarse sites" % len(host["dc"]))
    t_dc = 0.0
    e_dc = []
    Lw = [3 * a for a in AGG]
    centre = 1 + 3 * (1 + 3 * (1 + 3 * 1))
    for (i, Uw, qw, got) in host["dc"]:
        Aw = oracle.clover(Lw, Uw, CSW, m0)
        t = time.perf_counter()
        ref = oracle.coarse_op(Lw, AGG, Uw, Aw, qw, agg_list=[centre])[centre]
        t_dc += time.perf_counter() - t
        e_dc.append(max(rel(got[d], ref[d]) for d in range(9)))
    t_dc *= n_agg / len(host["dc"])
    acc["dc_fp32"] = {"rel_err": max(e_dc), "tol": TOL["f32"],
                      "sample": "all 9 blocks of %d coarse sites (oracle on the 12^4 window around each)" % len(e_dc)}
    if fp16 is not None:
        c3, got, Uh = fp16
        log("oracle: SAP of one test vector of the 32^3 x 64 workload")
        A3 = oracle.clover(c3["L"], Uh, CSW, c3["m0"])
        b3 = inputs.test_vectors_device(c3["L"], 1, c3["seed_v"], "cuda", first=host["k"]).cpu().numpy()
        ref3 = oracle.sap(c3["L"], BLOCK, Uh, A3, b3, N_SAP, N_MR)[0]
        del A3
        acc["sap_c3_f16_storage"] = {"rel_err": rel(got["f16_storage"], ref3), "tol": TOL["f16_storage"],
                                     "sample": "32^3x64, test vector %d" % host["k"]}
        acc["sap_c3_fp32"] = {"rel_err": rel(got["f32"], ref3), "tol": TOL["f32"],
                              "sample": "32^3x64, test vector %d" % host["k"]}
    for v in acc.values():
        v["ok"] = bool(v["rel_err"] <= v["tol"])
    # one thread on the 16^4 workload: SAP from x = 0 on one of its 20 vectors, scaled x20
    log("oracle: one-thread SAP on 16^4")
    import ctypes
    gomp = ctypes.CDLL("libgomp.so.1")  # the OpenMP runtime the oracle library runs on
    L2 = C2["L"]
    U2 = inputs.gauge_field(L2, C2["sigma"], C2["seed_u"])
    A2 = oracle.clover(L2, U2, CSW, C2["m0"])
    b2 = inputs.test_vectors(L2, 1, C2["seed_v"])
    gomp.omp_set_num_threads(1)
    try:
        t = time.perf_counter()
        oracle.sap(L2, BLOCK, U2, A2, b2, N_SAP, N_MR)
        t_one = (time.perf_counter() - t) * C2["n_tv"]
    finally:
        gomp.omp_set_num_threads(cores)
    one = {"value": int(np.prod(L2)) * C2["n_tv"] * N_SAP / t_one, "unit": "site*RHS updates/s", "cores": 1,
           "sample": "16^4, SAP 3x4 from x = 0 on 1 of 20 test vectors (scaled x20)"}
    total = t_sap + t_res + t_gs + t_dc
    cpu = {"value": V * n * N_SAP / total, "unit": "site*RHS updates/s", "cores": cores, "kind": "oracle",
           "sample": ("48^3x96 step: SAP + residual on 1 of %d test vectors (scaled x%d), block GS on %d of %d "
                      "aggregates (scaled), D_c on %d of %d coarse sites (12^4 window each, scaled); clover "
                      "set-up (%.1f s) excluded; FP64 C, OpenMP"
                      % (n, n, len(host["gs_aggs"]), n_agg, len(host["dc"]), n_agg, t_clover)),
           "seconds_scaled": {"sap": round(t_sap, 2), "resid": round(t_res, 2), "gs": round(t_gs, 2),
                              "dc": round(t_dc, 2)},
           "one_thread_16x16x16x16_sap": one}
    return acc, cpu


def gather_for_oracle(st, U_dev, k=0, n_gs=64, dc_sites=(0, 12345)):
    """Copy to the host what the oracle needs to check the step's results on a sample."""
    op, n, L = st.op, st.n, st.cfg["L"]
    host = {"k": k, "x_k": unpack_rhs(op, st.x, op.dtype, n, k),
            "b_k": inputs.test_vectors_device(L, 1, st.cfg["seed_v"], "cuda", first=k).cpu().numpy()[0],
            "res_k": float(st.res[k].item())}
    aggs = list(np.linspace(0, op.n_agg - 1, n_gs).astype(int))
    sites = np.concatenate([agg_site_index(L, AGG, i) for i in aggs])
    Va = int(np.prod(AGG))
    host["gs_aggs"] = aggs
    host["gs_V"] = gather_sites(op, st.x, op.dtype, n, sites).reshape(n, n_gs, Va, 4, 3)
    host["gs_Q"] = gather_sites(op, st.Q, mrhs.DTYPE_F32, n, sites).reshape(n, n_gs, Va, 4, 3)
    nc = 2 * n
    host["dc"] = []
    for i in dc_sites:
        wsites = agg_site_index(L, AGG, i, window=3)
        Uw = U_dev[:, torch.as_tensor(wsites, device="cuda")].cpu().numpy()
        qw = gather_sites(op, st.Q, mrhs.DTYPE_F32, n, wsites)
        got = st.Dc.view(op.n_agg, 9, nc, nc, 2)[i].double().cpu().numpy()
        host["dc"].append((i, np.ascontiguousarray(Uw), qw, got[..., 0] + 1j * got[..., 1]))
    return host


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the oracle (errors and CPU baseline)")
    ap.add_argument("--no-srhs", action="store_true")
    ap.add_argument("--no-fp16", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the 16^4 extras and the batch")
    ap.add_argument("--no-coarse", action="store_true", help="skip the coarse grid of the headline workload")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-refine", action="store_true")
    ap.add_argument("--no-eo", action="store_true")
    ap.add_argument("--tiles", type=str, default=None, help="SAP,stencil tiles instead of the autotuner (e.g. 4,4)")
    ap.add_argument("--copy-calib", action="store_true", help="only run a plain 1 GiB device copy (counter scale)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (it would shard the "
              "lattice by domain decomposition, one halo exchange per SAP half-sweep)", file=sys.stderr)
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

    cfg = C5
    L, n = cfg["L"], cfg["n_tv"]
    V = int(np.prod(L))
    log("generating the %s inputs on the device" % "x".join(map(str, L)))
    U = inputs.gauge_field_device(L, cfg["sigma"], cfg["seed_u"], "cuda")
    plaq = average_plaquette(U, L)
    torch.cuda.empty_cache()
    log("average plaquette %.6f" % plaq)
    log("operator set-up")
    mr = Setup(cfg, U)
    if args.tiles:
        ts, td = (int(t) for t in args.tiles.split(","))
        mrhs.mrhs_set_tiles(mr.op.handle, ts, td)
        tiles = {"sap": ts, "dirac": td, "fixed": True}
    else:
        tiles = autotune.autotune(mr.op, n, N_SAP, N_MR, b=mr.b, x=mr.x)
    log("tiles: %s" % tiles)
    log("timing %d steps after %d warm-up" % (args.steps, args.warmup))
    step_ms, wall_ms, per, spread = time_steps(mr, args.steps, args.warmup)
    assert int(mr.status.item()) == 0
    res = mr.res.cpu().numpy()
    log("step %.3f ms (wall %.3f): %s; residuals %.4f..%.4f" % (step_ms, wall_ms, per, res.min(), res.max()))
    value = V * n * N_SAP / (step_ms * 1e-3)
    n_agg = V // int(np.prod(AGG))
    plat = platform()

    # dominant kernel: the SAP half-sweep (2 * N_SAP launches per call, nothing else)
    n_launch = 2 * N_SAP
    sap_launch_ms = per["sap"] / n_launch
    flops_launch = sap_flops_per_call(V, n, N_SAP, N_MR, BLOCK) / n_launch
    achieved = flops_launch / (sap_launch_ms * 1e-3) / 1e12
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved / FP32_VECTOR_PEAK_TFLOPS, 4), "traffic": sap_traffic_bytes(tiles["sap"]),
            "traffic_unit": "bytes per launch (HBM, counters)",
            "alg_bytes": round(sap_bytes_per_call(V, n, N_SAP, 4, 4) / n_launch),
            "kernel": "k_sap_batched (FP32, tile %d)" % tiles["sap"], "launch_ms": round(sap_launch_ms, 4),
            "frac_of_issue_peak": round(achieved / FP32_ISSUE_PEAK_TFLOPS, 4),
            "flops_per_launch": flops_launch}

    # stencil HBM roofline (the HBM-bound kernel of the path), and the copy ceiling
    y = mr.op.empty(n)
    d_ms = time_call(lambda: mrhs.dirac_apply_mrhs(mr.op.handle, mr.b, y, n), 10)
    del y
    d_bytes = V * n * pm.stencil_bytes_per_site_rhs(n, 4, 4)
    copy = copy_ceiling()
    # tile 4 on a short length of 4 runs two groups per workgroup
    dname = "k_dirac_2g" if tiles["dirac"] == 4 and S == 4 else "k_dirac"
    stencil = {"kernel": "%s (FP32, %d RHS, tile %d)" % (dname, n, tiles["dirac"]), "ms": round(d_ms, 4),
               "GBs": round(d_bytes / d_ms / 1e6, 1), "frac_hbm": round(d_bytes / d_ms / 1e6 / HBM_PEAK_GBS, 4),
               "frac_of_copy": round(d_bytes / d_ms / 1e6 / copy["GBs"], 4),
               "site_rhs_per_s": V * n / (d_ms * 1e-3)}
    roof["alg_GBs"] = round(roof["alg_bytes"] / (sap_launch_ms * 1e-3) / 1e9, 1)
    sap_bytes = sap_bytes_per_call(V, n, N_SAP, 4, 4)
    sap_info = {"ms_per_call": round(per["sap"], 4), "alg_GBs": round(sap_bytes / per["sap"] / 1e6, 1),
                "alg_tflops": round(sap_flops_per_call(V, n, N_SAP, N_MR, BLOCK) / per["sap"] / 1e9, 3)}
    log("roofline %s; stencil %s; copy %s" % (roof, stencil, copy))

    coarse5 = None
    if not args.no_coarse:
        log("coarse grid of the headline workload (FP32 and half precision)")
        coarse5 = coarse_grid_c5(mr)
        log("coarse %s" % coarse5)

    host = None
    if not args.no_cpu_baseline:
        log("copying the sampled results to the host")
        host = gather_for_oracle(mr, U)
        host["U"] = U.cpu().numpy()
    mr.close()
    torch.cuda.empty_cache()

    srhs = None
    if not args.no_srhs:
        log("single-RHS FP64 and MRHS FP64 paths")
        srhs = srhs_bench(cfg, U, per["sap"])
        log("srhs %s" % srhs)
    del U
    torch.cuda.empty_cache()

    fp16, fp16_data = None, None
    if not args.no_fp16:
        log("FP16 storage on 32^3x64")
        fp16, got16, U3 = fp16_bench(C3, 0)
        fp16_data = (C3, got16, U3)
        log("fp16 %s" % fp16)

    extras = None
    if not args.no_extras:
        log("16^4 extras")
        extras = extras_16(args)

    acc, cpu = None, None
    if host is not None:
        log("FP64 oracle on the sample")
        acc, cpu = oracle_checks(cfg, host, fp16_data)
        log("accuracy %s" % acc)
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
        "config": {"workload": workload_name(cfg), "lattice": L, "n_tv": n, "sap": [N_SAP, N_MR], "block": BLOCK,
                   "aggregate": AGG, "parallelism": "single GPU",
                   "tiles": {"sap": tiles["sap"], "dirac": tiles["dirac"]}},
        "parts_ms": {k: round(float(x), 4) for k, x in per.items()},
        "step_ms_spread": {k: round(x, 4) for k, x in spread.items()},
        "rates": {"sap_d_equivalents_per_s": V * n * N_SAP * (N_MR + 1) / (per["sap"] * 1e-3),
                  "gs_site_rhs_per_s": V * n / (per["gs"] * 1e-3),
                  "gs_aggregates_per_s": n_agg / (per["gs"] * 1e-3),
                  "dc_site_rhs_per_s": V * n / (per["dc"] * 1e-3),
                  "dc_aggregates_per_s": n_agg / (per["dc"] * 1e-3)},
        "average_plaquette": plaq,
        "platform": plat,
        "residual_max": float(res.max()),
        "roofline": roof,
        "stencil_roofline": stencil,
        "copy_ceiling": copy,
        "sap": sap_info,
        "coarse_grid": coarse5,
        "accuracy": acc,
        "srhs": srhs,
        "fp16_storage_32x32x32x64": fp16,
        "extras_16x16x16x16": extras,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
