"""Python binding of the C-ABI in include/mrhs.h (argument marshalling only).

Functions carry the C names; they take torch tensors that live on the GPU (device
memory and streams come from PyTorch) and raise MrhsError on a non-zero return
code.  Every step of the path runs in the HIP library; if libmrhs.so is missing
the first call raises -- there is no fallback.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libmrhs.so")

MRHS_OK, MRHS_EINVAL, MRHS_EUNSUPPORTED, MRHS_EHIP, MRHS_ERANK, MRHS_ERANGE = 0, -1, -2, -3, -4, -5
DTYPE_F64, DTYPE_F32, DTYPE_F16 = 0, 1, 2
PREC_F64, PREC_F32, PREC_F32_F16STORE = 0, 1, 2
BLOCK_MR, BLOCK_EO_MR = 0, 1
TORCH_DTYPE = {DTYPE_F64: torch.float64, DTYPE_F32: torch.float32, DTYPE_F16: torch.float16}


class MrhsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("mrhs error %d: %s" % (code, msg))
        self.code = code


class Geom(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32 * 4), ("block", ctypes.c_int32 * 4), ("agg", ctypes.c_int32 * 4)]


_lib = None


def lib():
    """Load libmrhs.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError("libmrhs.so not built: run python -m paper_1601_03184_amd.build")
        L = ctypes.CDLL(_LIB_PATH)
        p, i32, d, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double, ctypes.c_size_t
        sig = {
            "mrhs_op_create": (i32, [ctypes.POINTER(Geom), p, d, d, i32, i32, p, ctypes.POINTER(p)]),
            "mrhs_op_destroy": (i32, [p]),
            "mrhs_op_vector_dtype": (i32, [p]),
            "mrhs_op_short_len": (i32, [p]),
            "mrhs_vector_bytes": (sz, [p, i32, i32]),
            "mrhs_workspace_bytes": (sz, [p, i32]),
            "mrhs_pack": (i32, [p, p, p, i32, i32, p]),
            "mrhs_unpack": (i32, [p, p, i32, p, i32, p]),
            "dirac_apply_mrhs": (i32, [p, p, p, i32, p]),
            "sap_smooth_mrhs": (i32, [p, p, p, i32, i32, i32, p, sz, p]),
            "sap_smooth_mrhs_guess": (i32, [p, p, p, i32, i32, i32, p, sz, p]),
            "mrhs_residual_norms": (i32, [p, p, p, i32, p, p, sz, p]),
            "mrhs_residual_norms_noalloc": (i32, [p, p, p, i32, p, p]),
            "block_orthonormalize": (i32, [p, p, i32, p, i32, i32, p, p, sz, p]),
            "coarse_op_build": (i32, [p, p, i32, i32, p, p, sz, p]),
            "mrhs_set_tiles": (i32, [p, i32, i32]),
            "mrhs_set_block_solver": (i32, [p, i32, p]),
            "mrhs_op_block_solver": (i32, [p]),
            "sap_smooth_mrhs_batched": (i32, [p, i32, p, p, p, i32, i32, p, sz, p]),
            "mrhs_batched_workspace_bytes": (sz, [p, i32, p]),
            "mrhs_coarse_vector_bytes": (sz, [p, i32, i32]),
            "restrict_mrhs": (i32, [p, p, i32, i32, p, i32, p, i32, p]),
            "prolong_mrhs": (i32, [p, p, i32, i32, p, p, i32, i32, p]),
            "coarse_apply_mrhs": (i32, [p, p, i32, p, p, i32, p]),
            "mrhs_coarse_solve_workspace_bytes": (sz, [p, i32, i32, i32]),
            "coarse_solve_mrhs": (i32, [p, p, i32, p, p, i32, i32, d, p, p, p, sz, p]),
            "coarse_self_invert": (i32, [p, p, i32, p, p, p]),
            "coarse_op_build_f16": (i32, [p, p, i32, i32, p, p]),
            "coarse_apply_f16_mrhs": (i32, [p, p, i32, p, p, i32, p]),
            "mrhs_coarse_solve_f16_workspace_bytes": (sz, [p, i32, i32, i32]),
            "coarse_solve_f16_mrhs": (i32, [p, p, i32, p, p, i32, i32, d, p, p, p, sz, p]),
            "mrhs_coarse_solve_eo_workspace_bytes": (sz, [p, i32, i32, i32]),
            "coarse_solve_eo_mrhs": (i32, [p, p, p, i32, p, p, i32, i32, d, p, p, p, sz, p]),
            "mrhs_refine_workspace_bytes": (sz, [p, i32, i32]),
            "setup_refine_mrhs": (i32, [p, p, i32, p, i32, p, i32, i32, i32, d, p, sz, p]),
            "mrhs_last_error": (ctypes.c_char_p, []),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc):
    if rc != MRHS_OK:
        raise MrhsError(rc, lib().mrhs_last_error().decode())
    return rc


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    return ctypes.c_void_p(t.data_ptr())


def mrhs_last_error():
    return lib().mrhs_last_error().decode()


def mrhs_op_create(L, block, agg, links, m0, csw, prec, short_len, stream=None):
    """links: complex128 (or float64 view) GPU tensor [4][V][3][3].  Returns the handle."""
    g = Geom((ctypes.c_int32 * 4)(*L), (ctypes.c_int32 * 4)(*block), (ctypes.c_int32 * 4)(*agg))
    links = links.contiguous()
    out = ctypes.c_void_p()
    _check(lib().mrhs_op_create(ctypes.byref(g), _dptr(links), float(m0), float(csw), int(prec), int(short_len),
                                _stream(stream), ctypes.byref(out)))
    return out


def mrhs_op_destroy(op):
    _check(lib().mrhs_op_destroy(op))


def mrhs_op_vector_dtype(op):
    return lib().mrhs_op_vector_dtype(op)


def mrhs_op_short_len(op):
    return lib().mrhs_op_short_len(op)


def mrhs_vector_bytes(op, n_rhs, dtype):
    return lib().mrhs_vector_bytes(op, int(n_rhs), int(dtype))


def mrhs_workspace_bytes(op, n_rhs):
    return lib().mrhs_workspace_bytes(op, int(n_rhs))


def mrhs_pack(op, canon, native, dtype, n_rhs, stream=None):
    _check(lib().mrhs_pack(op, _dptr(canon), _dptr(native), int(dtype), int(n_rhs), _stream(stream)))


def mrhs_unpack(op, native, dtype, canon, n_rhs, stream=None):
    _check(lib().mrhs_unpack(op, _dptr(native), int(dtype), _dptr(canon), int(n_rhs), _stream(stream)))


def dirac_apply_mrhs(op, x, y, n_rhs, stream=None):
    _check(lib().dirac_apply_mrhs(op, _dptr(x), _dptr(y), int(n_rhs), _stream(stream)))


def sap_smooth_mrhs(op, b, x, n_rhs, n_sap, n_mr, ws, stream=None):
    nb = ws.numel() * ws.element_size() if ws is not None else 0
    _check(lib().sap_smooth_mrhs(op, _dptr(b), _dptr(x), int(n_rhs), int(n_sap), int(n_mr), _dptr(ws), nb,
                                 _stream(stream)))


def sap_smooth_mrhs_guess(op, b, x, n_rhs, n_sap, n_mr, ws, stream=None):
    nb = ws.numel() * ws.element_size() if ws is not None else 0
    _check(lib().sap_smooth_mrhs_guess(op, _dptr(b), _dptr(x), int(n_rhs), int(n_sap), int(n_mr), _dptr(ws), nb,
                                       _stream(stream)))


def mrhs_residual_norms(op, b, x, n_rhs, out, ws, stream=None):
    _check(lib().mrhs_residual_norms(op, _dptr(b), _dptr(x), int(n_rhs), _dptr(out), _dptr(ws),
                                     ws.numel() * ws.element_size(), _stream(stream)))


def mrhs_residual_norms_noalloc(op, b, x, n_rhs, out, stream=None):
    _check(lib().mrhs_residual_norms_noalloc(op, _dptr(b), _dptr(x), int(n_rhs), _dptr(out), _stream(stream)))


def block_orthonormalize(op, V, v_dtype, Q, q_dtype, n_tv, status, ws, stream=None):
    nb = ws.numel() * ws.element_size() if ws is not None else 0
    _check(lib().block_orthonormalize(op, _dptr(V), int(v_dtype), _dptr(Q), int(q_dtype), int(n_tv), _dptr(status),
                                      _dptr(ws), nb, _stream(stream)))


def coarse_op_build(op, Q, q_dtype, n_tv, Dc, ws, stream=None):
    nb = ws.numel() * ws.element_size() if ws is not None else 0
    _check(lib().coarse_op_build(op, _dptr(Q), int(q_dtype), int(n_tv), _dptr(Dc), _dptr(ws), nb, _stream(stream)))


def mrhs_coarse_vector_bytes(op, n_tv, n_rhs):
    return lib().mrhs_coarse_vector_bytes(op, int(n_tv), int(n_rhs))


def restrict_mrhs(op, Q, q_dtype, n_tv, y, y_dtype, yc, n_rhs, stream=None):
    _check(lib().restrict_mrhs(op, _dptr(Q), int(q_dtype), int(n_tv), _dptr(y), int(y_dtype), _dptr(yc), int(n_rhs),
                               _stream(stream)))


def prolong_mrhs(op, Q, q_dtype, n_tv, yc, y, y_dtype, n_rhs, stream=None):
    _check(lib().prolong_mrhs(op, _dptr(Q), int(q_dtype), int(n_tv), _dptr(yc), _dptr(y), int(y_dtype), int(n_rhs),
                              _stream(stream)))


def coarse_apply_mrhs(op, Dc, n_tv, yc, yc_out, n_rhs, stream=None):
    _check(lib().coarse_apply_mrhs(op, _dptr(Dc), int(n_tv), _dptr(yc), _dptr(yc_out), int(n_rhs), _stream(stream)))


def mrhs_coarse_solve_workspace_bytes(op, n_tv, n_rhs, m):
    return lib().mrhs_coarse_solve_workspace_bytes(op, int(n_tv), int(n_rhs), int(m))


def coarse_solve_mrhs(op, Dc, n_tv, bc, uc, n_rhs, m, tol, ws, res_out=None, iters_out=None, stream=None):
    nb = ws.numel() * ws.element_size() if ws is not None else 0
    _check(lib().coarse_solve_mrhs(op, _dptr(Dc), int(n_tv), _dptr(bc), _dptr(uc), int(n_rhs), int(m), float(tol),
                                   _dptr(res_out), _dptr(iters_out), _dptr(ws), nb, _stream(stream)))


def coarse_op_build_f16(op, Q, q_dtype, n_tv, Dc16, stream=None):
    _check(lib().coarse_op_build_f16(op, _dptr(Q), int(q_dtype), int(n_tv), _dptr(Dc16), _stream(stream)))


def coarse_apply_f16_mrhs(op, Dc16, n_tv, yc, yc_out, n_rhs, stream=None):
    _check(lib().coarse_apply_f16_mrhs(op, _dptr(Dc16), int(n_tv), _dptr(yc), _dptr(yc_out), int(n_rhs),
                                       _stream(stream)))


def mrhs_coarse_solve_f16_workspace_bytes(op, n_tv, n_rhs, m):
    return lib().mrhs_coarse_solve_f16_workspace_bytes(op, int(n_tv), int(n_rhs), int(m))


def coarse_solve_f16_mrhs(op, Dc16, n_tv, bc, uc, n_rhs, m, tol, ws, res_out=None, iters_out=None, stream=None):
    nb = ws.numel() * ws.element_size() if ws is not None else 0
    _check(lib().coarse_solve_f16_mrhs(op, _dptr(Dc16), int(n_tv), _dptr(bc), _dptr(uc), int(n_rhs), int(m), float(tol),
                                       _dptr(res_out), _dptr(iters_out), _dptr(ws), nb, _stream(stream)))


def coarse_self_invert(op, Dc, n_tv, Dinv, status=None, stream=None):
    _check(lib().coarse_self_invert(op, _dptr(Dc), int(n_tv), _dptr(Dinv), _dptr(status), _stream(stream)))


def mrhs_coarse_solve_eo_workspace_bytes(op, n_tv, n_rhs, m):
    return lib().mrhs_coarse_solve_eo_workspace_bytes(op, int(n_tv), int(n_rhs), int(m))


def coarse_solve_eo_mrhs(op, Dc, Dinv, n_tv, bc, uc, n_rhs, m, tol, ws, res_out=None, iters_out=None, stream=None):
    nb = ws.numel() * ws.element_size() if ws is not None else 0
    _check(lib().coarse_solve_eo_mrhs(op, _dptr(Dc), _dptr(Dinv), int(n_tv), _dptr(bc), _dptr(uc), int(n_rhs), int(m),
                                      float(tol), _dptr(res_out), _dptr(iters_out), _dptr(ws), nb, _stream(stream)))


def mrhs_refine_workspace_bytes(op, n_tv, m):
    return lib().mrhs_refine_workspace_bytes(op, int(n_tv), int(m))


def setup_refine_mrhs(op, V, n_tv, Q, q_dtype, Dc, n_sap, n_mr, m, tol, ws, stream=None):
    nb = ws.numel() * ws.element_size() if ws is not None else 0
    _check(lib().setup_refine_mrhs(op, _dptr(V), int(n_tv), _dptr(Q), int(q_dtype), _dptr(Dc), int(n_sap), int(n_mr),
                                   int(m), float(tol), _dptr(ws), nb, _stream(stream)))


def _arrays(ops, bs, xs, n_rhs):
    n = len(ops)
    OA = (ctypes.c_void_p * n)(*[h.value if isinstance(h, ctypes.c_void_p) else h for h in ops])
    NA = (ctypes.c_int32 * n)(*[int(k) for k in n_rhs])
    BA = (ctypes.c_void_p * n)(*[t.data_ptr() for t in bs]) if bs is not None else None
    XA = (ctypes.c_void_p * n)(*[t.data_ptr() for t in xs]) if xs is not None else None
    return n, OA, NA, BA, XA


def mrhs_batched_workspace_bytes(ops, n_rhs):
    n, OA, NA, _, _ = _arrays(ops, None, None, n_rhs)
    return lib().mrhs_batched_workspace_bytes(OA, n, NA)


def sap_smooth_mrhs_batched(ops, bs, xs, n_rhs, n_sap, n_mr, ws, stream=None):
    """ops: list of handles; bs, xs: lists of GPU native vectors; n_rhs: list of ints."""
    for t in list(bs) + list(xs):
        if not t.is_cuda:
            raise ValueError("tensor must live on the GPU")
    n, OA, NA, BA, XA = _arrays(ops, bs, xs, n_rhs)
    nb = ws.numel() * ws.element_size() if ws is not None else 0
    _check(lib().sap_smooth_mrhs_batched(OA, n, BA, XA, NA, int(n_sap), int(n_mr), _dptr(ws), nb, _stream(stream)))


def mrhs_set_tiles(op, sap_tile=0, dirac_tile=0):
    _check(lib().mrhs_set_tiles(op, int(sap_tile), int(dirac_tile)))


def mrhs_op_block_solver(op):
    return lib().mrhs_op_block_solver(op)


def mrhs_set_block_solver(op, solver, stream=None):
    """BLOCK_MR (plain MR on D_j) or BLOCK_EO_MR (MR on the block's even-site Schur complement)."""
    _check(lib().mrhs_set_block_solver(op, int(solver), _stream(stream)))


class Operator:
    """Owns an mrhs_op handle and allocates native vectors and workspace with torch."""

    def __init__(self, L, block, agg, links, m0, csw, prec=PREC_F32, short_len=4, device="cuda", stream=None):
        self.L, self.block, self.agg = list(L), list(block), list(agg)
        self.device = torch.device(device)
        if links.dtype == torch.complex128:
            links = torch.view_as_real(links)
        self.handle = mrhs_op_create(self.L, self.block, self.agg, links.to(self.device), m0, csw, prec, short_len,
                                     stream)
        self.prec = prec
        self.dtype = mrhs_op_vector_dtype(self.handle)
        self.S = mrhs_op_short_len(self.handle)
        self.V = L[0] * L[1] * L[2] * L[3]
        self.n_agg = 1
        for m in range(4):
            self.n_agg *= L[m] // agg[m]

    def close(self):
        if self.handle is not None:
            mrhs_op_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def empty(self, n_rhs, dtype=None):
        dt = self.dtype if dtype is None else dtype
        n = mrhs_vector_bytes(self.handle, n_rhs, dt) // torch.tensor([], dtype=TORCH_DTYPE[dt]).element_size()
        return torch.empty(n, dtype=TORCH_DTYPE[dt], device=self.device)

    def coarse_empty(self, n_tv, n_rhs):
        """FP32 coarse vectors (zeroed) for n_rhs right-hand sides of an n_tv-vector coarse grid."""
        return torch.zeros(mrhs_coarse_vector_bytes(self.handle, n_tv, n_rhs) // 4, dtype=torch.float32,
                           device=self.device)

    def workspace(self, n_rhs):
        return torch.empty(mrhs_workspace_bytes(self.handle, n_rhs), dtype=torch.uint8, device=self.device)

    def pack(self, canon, dtype=None):
        """canon: complex128 [n][V][4][3] (host or device) -> native vectors."""
        dt = self.dtype if dtype is None else dtype
        c = canon.to(self.device, torch.complex128).contiguous()
        n = c.shape[0]
        out = self.empty(n, dt)
        mrhs_pack(self.handle, torch.view_as_real(c), out, dt, n)
        return out

    def unpack(self, native, n_rhs, dtype=None):
        dt = self.dtype if dtype is None else dtype
        out = torch.zeros((n_rhs, self.V, 4, 3, 2), dtype=torch.float64, device=self.device)
        mrhs_unpack(self.handle, native, dt, out, n_rhs)
        return torch.view_as_complex(out)
