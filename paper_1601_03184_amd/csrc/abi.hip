// abi.hip -- the extern "C" entry points of include/mrhs.h: argument validation,
// operator construction, dispatch to the kernel launchers.
#include <cstdio>
#include <cstring>
#include <vector>

#include "launch.h"

namespace {
thread_local std::string g_last_error;
}

int set_error(int code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

int hip_check(hipError_t e, const char *what)
{
    if (e == hipSuccess) return MRHS_OK;
    return set_error(MRHS_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

int dtype_size(int dtype) { return dtype == MRHS_DTYPE_F64 ? 8 : dtype == MRHS_DTYPE_F32 ? 4 : 2; }

size_t native_elems(const mrhs_op *op, int n_rhs)
{
    const long ngrp = (n_rhs + op->k.S - 1) / op->k.S;
    return (size_t)ngrp * op->k.S * 24 * op->k.V;
}

namespace {

// [a, a + na) and [b, b + nb) intersect
bool ranges_overlap(const void *a, size_t na, const void *b, size_t nb)
{
    const char *pa = (const char *)a, *pb = (const char *)b;
    return pa < pb + nb && pb < pa + na;
}

bool ranges_overlap(const void *a, const void *b, size_t n) { return ranges_overlap(a, n, b, n); }

int check_op(const mrhs_op *op)
{
    if (!op) return set_error(MRHS_EINVAL, "null operator");
    return MRHS_OK;
}

int check_nrhs(int n_rhs)
{
    if (n_rhs <= 0) return set_error(MRHS_EINVAL, "n_rhs must be positive");
    return MRHS_OK;
}

int check_dtype(int dt)
{
    if (dt != MRHS_DTYPE_F64 && dt != MRHS_DTYPE_F32 && dt != MRHS_DTYPE_F16)
        return set_error(MRHS_EINVAL, "unknown dtype");
    return MRHS_OK;
}

size_t sap_lds_bytes(const mrhs_op *op, int T)
{
    const size_t esz = op->prec == MRHS_PREC_F64 ? 8 : 4;
    const size_t threads = (op->k.Vb * T + 63) / 64 * 64;
    return esz * (24 * (size_t)op->k.Vb * T + threads / 64 * T * 3);
}

// SAP and stencil tiles with FP64 arithmetic above 2 right-hand sides per site need more
// registers than a workgroup of that size may hold (the kernels would spill to scratch):
// they are not built
bool tile_built(const mrhs_op *op, int T) { return op->prec != MRHS_PREC_F64 || T <= 2; }

int pick_tile(const mrhs_op *op, int want, bool sap)
{
    int t = want;
    while (t > 1 && (op->k.S % t != 0 || op->k.Vb * t > 1024 || !tile_built(op, t) ||
                     (sap && sap_lds_bytes(op, t) > op->max_lds)))
        t >>= 1;
    return t;
}

void free_op(mrhs_op *op)
{
    if (!op) return;
    void *ptrs[] = {op->links64, op->clover64, op->links32, op->clover32, op->blk_coords, op->loc_coords,
                    op->colour_blocks, op->agg_sites, op->cloverinv64, op->cloverinv32, op->eo_sites,
                    op->status};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    delete op;
}

}  // namespace

extern "C" {

const char *mrhs_last_error(void) { return g_last_error.c_str(); }

int mrhs_op_create(const mrhs_geom *geom, const double *links, double m0, double csw, int32_t prec, int32_t short_len,
                   void *stream, mrhs_op **out)
{
    if (!geom || !links || !out) return set_error(MRHS_EINVAL, "null argument");
    *out = nullptr;
    if (prec < MRHS_PREC_F64 || prec > MRHS_PREC_F32_F16STORE) return set_error(MRHS_EINVAL, "unknown precision");
    if (short_len != 1 && short_len != 2 && short_len != 4 && short_len != 8)
        return set_error(MRHS_EINVAL, "short_len must be 1, 2, 4 or 8");
    long V = 1, Vb = 1, Va = 1;
    for (int mu = 0; mu < 4; ++mu) {
        const int L = geom->L[mu], b = geom->block[mu], a = geom->agg[mu];
        if (L < 1 || b < 1 || a < 1 || L % b != 0 || L % a != 0)
            return set_error(MRHS_EINVAL, "block and aggregate extents must divide the lattice");
        if (L / b > 255 || b > 255 || L / a > 255 || a > 255)
            return set_error(MRHS_EUNSUPPORTED, "more than 255 blocks or sites per block in a direction");
        V *= L;
        Vb *= b;
        Va *= a;
    }
    if (Vb > 256) return set_error(MRHS_EUNSUPPORTED, "SAP block volume above 256");
    // kernels address a group of S right-hand sides with 32-bit element offsets
    if (24.0 * (double)V * short_len >= 2147483648.0)
        return set_error(MRHS_EUNSUPPORTED, "lattice too large for the 32-bit in-group offsets");
    if (6 * Va > (1 << 20)) return set_error(MRHS_EUNSUPPORTED, "aggregate too large");

    mrhs_op *op = new mrhs_op();
    op->g = *geom;
    op->prec = prec;
    op->dtype = prec == MRHS_PREC_F64 ? MRHS_DTYPE_F64 : prec == MRHS_PREC_F32 ? MRHS_DTYPE_F32 : MRHS_DTYPE_F16;
    KGeo &k = op->k;
    int nblk = 1;
    for (int mu = 0; mu < 4; ++mu) {
        k.L[mu] = geom->L[mu];
        k.b[mu] = geom->block[mu];
        k.nb[mu] = geom->L[mu] / geom->block[mu];
        op->na[mu] = geom->L[mu] / geom->agg[mu];
        nblk *= k.nb[mu];
    }
    k.ostr[0] = 1;
    k.bstr[0] = 1;
    for (int mu = 1; mu < 4; ++mu) {
        k.ostr[mu] = k.ostr[mu - 1] * k.b[mu - 1];
        k.bstr[mu] = k.bstr[mu - 1] * k.nb[mu - 1];
    }
    k.Vb = (int)Vb;
    k.nblk = nblk;
    k.V = V;
    k.S = short_len;
    op->Va = (int)Va;
    op->n_agg = op->na[0] * op->na[1] * op->na[2] * op->na[3];
    op->odd_blocks = false;
    for (int mu = 0; mu < 4; ++mu)
        if (k.nb[mu] > 1 && (k.nb[mu] % 2)) op->odd_blocks = true;

    int rc = hip_check(hipGetDevice(&op->device), "hipGetDevice");
    int lds = 0;
    if (!rc) rc = hip_check(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, op->device),
                            "hipDeviceGetAttribute");
    op->max_lds = (size_t)lds;

    // host tables
    std::vector<uint32_t> bcoords(nblk), lcoords(Vb);
    std::vector<int32_t> colours;
    for (int j = 0; j < nblk; ++j) {
        int r = j;
        uint32_t p = 0;
        for (int mu = 0; mu < 4; ++mu) {
            p |= (uint32_t)(r % k.nb[mu]) << (8 * mu);
            r /= k.nb[mu];
        }
        bcoords[j] = p;
    }
    for (int o = 0; o < Vb; ++o) {
        int r = o;
        uint32_t p = 0;
        for (int mu = 0; mu < 4; ++mu) {
            p |= (uint32_t)(r % k.b[mu]) << (8 * mu);
            r /= k.b[mu];
        }
        lcoords[o] = p;
    }
    op->n_colour[0] = op->n_colour[1] = 0;
    for (int c = 0; c < 2; ++c)
        for (int j = 0; j < nblk; ++j) {
            uint32_t p = bcoords[j];
            int col = (unpack_coord(p, 0) + unpack_coord(p, 1) + unpack_coord(p, 2) + unpack_coord(p, 3)) & 1;
            if (col == c) {
                colours.push_back(j);
                op->n_colour[c]++;
            }
        }
    // native site of every aggregate site: [n_agg][Va], local sites lexicographic
    std::vector<int32_t> asites((size_t)op->n_agg * Va);
    for (int i = 0; i < op->n_agg; ++i) {
        int ac[4], r = i;
        for (int mu = 0; mu < 4; ++mu) {
            ac[mu] = r % op->na[mu];
            r /= op->na[mu];
        }
        for (int ls = 0; ls < Va; ++ls) {
            int lc[4], q = ls;
            for (int mu = 0; mu < 4; ++mu) {
                lc[mu] = q % geom->agg[mu];
                q /= geom->agg[mu];
            }
            long blk = 0, off = 0;
            for (int mu = 3; mu >= 0; --mu) {
                const int x = ac[mu] * geom->agg[mu] + lc[mu];
                blk = blk * k.nb[mu] + x / k.b[mu];
                off = off * k.b[mu] + x % k.b[mu];
            }
            asites[(size_t)i * Va + ls] = (int32_t)(blk * Vb + off);
        }
    }

    auto alloc = [&](void **p, size_t bytes, const char *what) {
        if (!rc) rc = hip_check(hipMalloc(p, bytes), what);
    };
    alloc((void **)&op->links64, sizeof(double) * 4 * 18 * V, "hipMalloc links64");
    alloc((void **)&op->clover64, sizeof(double) * 72 * V, "hipMalloc clover64");
    if (prec != MRHS_PREC_F64) {
        alloc((void **)&op->links32, sizeof(float) * 4 * 18 * V, "hipMalloc links32");
        alloc((void **)&op->clover32, sizeof(float) * 72 * V, "hipMalloc clover32");
    }
    alloc((void **)&op->blk_coords, sizeof(uint32_t) * nblk, "hipMalloc blk_coords");
    alloc((void **)&op->loc_coords, sizeof(uint32_t) * Vb, "hipMalloc loc_coords");
    alloc((void **)&op->colour_blocks, sizeof(int32_t) * nblk, "hipMalloc colour_blocks");
    alloc((void **)&op->agg_sites, sizeof(int32_t) * asites.size(), "hipMalloc agg_sites");
    alloc((void **)&op->status, sizeof(int), "hipMalloc status");
    hipStream_t st = (hipStream_t)stream;
    if (!rc) rc = hip_check(hipMemcpyAsync(op->blk_coords, bcoords.data(), sizeof(uint32_t) * nblk, hipMemcpyHostToDevice, st), "copy");
    if (!rc) rc = hip_check(hipMemcpyAsync(op->loc_coords, lcoords.data(), sizeof(uint32_t) * Vb, hipMemcpyHostToDevice, st), "copy");
    if (!rc) rc = hip_check(hipMemcpyAsync(op->colour_blocks, colours.data(), sizeof(int32_t) * nblk, hipMemcpyHostToDevice, st), "copy");
    if (!rc) rc = hip_check(hipMemcpyAsync(op->agg_sites, asites.data(), sizeof(int32_t) * asites.size(), hipMemcpyHostToDevice, st), "copy");
    if (!rc) rc = launch_build_fields(op, links, m0, csw, st);
    if (!rc) rc = hip_check(hipStreamSynchronize(st), "hipStreamSynchronize(op_create)");
    op->sap_tile = pick_tile(op, prec == MRHS_PREC_F64 ? 1 : 2, true);
    op->dirac_tile = pick_tile(op, prec == MRHS_PREC_F64 ? 1 : 4, false);
    if (rc) {
        free_op(op);
        return rc;
    }
    *out = op;
    return MRHS_OK;
}

int mrhs_op_destroy(mrhs_op *op)
{
    if (!op) return set_error(MRHS_EINVAL, "null operator");
    int rc = hip_check(hipDeviceSynchronize(), "hipDeviceSynchronize(op_destroy)");
    free_op(op);
    return rc;
}

int mrhs_op_vector_dtype(const mrhs_op *op) { return op ? op->dtype : MRHS_EINVAL; }
int mrhs_op_short_len(const mrhs_op *op) { return op ? op->k.S : MRHS_EINVAL; }

size_t mrhs_vector_bytes(const mrhs_op *op, int32_t n_rhs, int32_t dtype)
{
    if (!op || n_rhs <= 0 || check_dtype(dtype)) return 0;
    return native_elems(op, n_rhs) * dtype_size(dtype);
}

size_t mrhs_workspace_bytes(const mrhs_op *op, int32_t n_rhs)
{
    if (!op || n_rhs <= 0) return 0;
    size_t w = ws_bytes_sap(op, n_rhs);
    w = std::max(w, ws_bytes_residual(op, n_rhs));
    w = std::max(w, ws_bytes_gs(op, n_rhs));
    w = std::max(w, ws_bytes_coarse(op, n_rhs));
    return std::max(w, (size_t)256);
}

int mrhs_pack(const mrhs_op *op, const double *canon, void *native, int32_t dtype, int32_t n_rhs, void *stream)
{
    if (int rc = check_op(op)) return rc;
    if (int rc = check_nrhs(n_rhs)) return rc;
    if (int rc = check_dtype(dtype)) return rc;
    if (!canon || !native) return set_error(MRHS_EINVAL, "null vector");
    hipStream_t st = (hipStream_t)stream;
    // the op's status word carries the FP16 range flag (the call synchronises, so it is
    // never part of a captured graph)
    int *flag = dtype == MRHS_DTYPE_F16 ? op->status : nullptr;
    int rc = MRHS_OK;
    if (flag) rc = hip_check(hipMemsetAsync(flag, 0, sizeof(int), st), "hipMemsetAsync(flag)");
    if (!rc) rc = launch_pack(op, canon, native, dtype, n_rhs, flag, st);
    int host_flag = 0;
    if (flag && !rc)
        rc = hip_check(hipMemcpyAsync(&host_flag, flag, sizeof(int), hipMemcpyDeviceToHost, st), "copy flag");
    if (!rc) rc = hip_check(hipStreamSynchronize(st), "hipStreamSynchronize(pack)");
    if (!rc && host_flag) return set_error(MRHS_ERANGE, "value outside the FP16 range");
    return rc;
}

int mrhs_unpack(const mrhs_op *op, const void *native, int32_t dtype, double *canon, int32_t n_rhs, void *stream)
{
    if (int rc = check_op(op)) return rc;
    if (int rc = check_nrhs(n_rhs)) return rc;
    if (int rc = check_dtype(dtype)) return rc;
    if (!canon || !native) return set_error(MRHS_EINVAL, "null vector");
    return launch_unpack(op, native, dtype, canon, n_rhs, (hipStream_t)stream);
}

int dirac_apply_mrhs(const mrhs_op *op, const void *x, void *y, int32_t n_rhs, void *stream)
{
    if (int rc = check_op(op)) return rc;
    if (int rc = check_nrhs(n_rhs)) return rc;
    if (!x || !y) return set_error(MRHS_EINVAL, "null vector");
    const size_t bytes = native_elems(op, n_rhs) * dtype_size(op->dtype);
    if (ranges_overlap(x, y, bytes)) return set_error(MRHS_EINVAL, "x and y overlap");
    return launch_dirac(op, x, y, n_rhs, (hipStream_t)stream);
}

namespace {

int sap_common(const mrhs_op *op, const void *b, void *x, int32_t n_rhs, int32_t n_sap, int32_t n_mr, void *ws,
               size_t ws_bytes, void *stream, bool guess)
{
    if (int rc = check_op(op)) return rc;
    if (int rc = check_nrhs(n_rhs)) return rc;
    if (!b || !x) return set_error(MRHS_EINVAL, "null vector");
    if (n_sap < 0 || n_mr < 0) return set_error(MRHS_EINVAL, "negative iteration count");
    const size_t bytes = native_elems(op, n_rhs) * dtype_size(op->dtype);
    if (ranges_overlap(b, x, bytes)) return set_error(MRHS_EINVAL, "b and x overlap");
    const size_t need = ws_bytes_sap(op, n_rhs);
    if (need && (!ws || ws_bytes < need)) return set_error(MRHS_EINVAL, "workspace too small");
    if (need && (ranges_overlap(ws, need, x, bytes) || ranges_overlap(ws, need, b, bytes)))
        return set_error(MRHS_EINVAL, "workspace overlaps a vector");
    return launch_sap(op, b, x, n_rhs, n_sap, n_mr, ws, (hipStream_t)stream, guess);
}

}  // namespace

int sap_smooth_mrhs(const mrhs_op *op, const void *b, void *x, int32_t n_rhs, int32_t n_sap, int32_t n_mr, void *ws,
                    size_t ws_bytes, void *stream)
{
    return sap_common(op, b, x, n_rhs, n_sap, n_mr, ws, ws_bytes, stream, false);
}

int sap_smooth_mrhs_guess(const mrhs_op *op, const void *b, void *x, int32_t n_rhs, int32_t n_sap, int32_t n_mr,
                          void *ws, size_t ws_bytes, void *stream)
{
    return sap_common(op, b, x, n_rhs, n_sap, n_mr, ws, ws_bytes, stream, true);
}

int mrhs_residual_norms(const mrhs_op *op, const void *b, const void *x, int32_t n_rhs, double *out, void *ws,
                        size_t ws_bytes, void *stream)
{
    if (int rc = check_op(op)) return rc;
    if (int rc = check_nrhs(n_rhs)) return rc;
    if (!b || !x || !out || !ws) return set_error(MRHS_EINVAL, "null argument");
    if (ws_bytes < ws_bytes_residual(op, n_rhs)) return set_error(MRHS_EINVAL, "workspace too small");
    return launch_residual(op, b, x, n_rhs, out, ws, (hipStream_t)stream);
}

int mrhs_residual_norms_noalloc(const mrhs_op *op, const void *b, const void *x, int32_t n_rhs, double *out,
                                void *stream)
{
    if (int rc = check_op(op)) return rc;
    if (int rc = check_nrhs(n_rhs)) return rc;
    if (!b || !x || !out) return set_error(MRHS_EINVAL, "null argument");
    return launch_residual_noalloc(op, b, x, n_rhs, out, (hipStream_t)stream);
}

int block_orthonormalize(const mrhs_op *op, const void *V, int32_t v_dtype, void *Q, int32_t q_dtype, int32_t n_tv,
                         int32_t *status, void *ws, size_t ws_bytes, void *stream)
{
    if (int rc = check_op(op)) return rc;
    if (int rc = check_nrhs(n_tv)) return rc;
    if (int rc = check_dtype(v_dtype)) return rc;
    if (int rc = check_dtype(q_dtype)) return rc;
    if (!V || !Q) return set_error(MRHS_EINVAL, "null vector");
    if (n_tv > 6 * op->Va) return set_error(MRHS_EINVAL, "more test vectors than rows of an aggregate half");
    const size_t ne = native_elems(op, n_tv);
    const bool same = V == Q && v_dtype == q_dtype;  // in place
    if (!same && ranges_overlap(V, ne * dtype_size(v_dtype), Q, ne * dtype_size(q_dtype)))
        return set_error(MRHS_EINVAL, "V and Q overlap (only exact in-place use with equal types is allowed)");
    if (ws_bytes < ws_bytes_gs(op, n_tv) || (!ws && ws_bytes_gs(op, n_tv)))
        return set_error(MRHS_EINVAL, "workspace too small");
    return launch_gs(op, V, v_dtype, Q, q_dtype, n_tv, status, ws, (hipStream_t)stream);
}

int coarse_op_build(const mrhs_op *op, const void *Q, int32_t q_dtype, int32_t n_tv, void *Dc, void *ws,
                    size_t ws_bytes, void *stream)
{
    if (int rc = check_op(op)) return rc;
    if (int rc = check_nrhs(n_tv)) return rc;
    if (!Q || !Dc) return set_error(MRHS_EINVAL, "null argument");
    if (int rc = check_dtype(q_dtype)) return rc;
    (void)ws;
    (void)ws_bytes;
    return launch_coarse(op, Q, q_dtype, n_tv, Dc, MRHS_DTYPE_F32, (hipStream_t)stream);
}

int coarse_op_build_f16(const mrhs_op *op, const void *Q, int32_t q_dtype, int32_t n_tv, void *Dc16, void *stream)
{
    if (int rc = check_op(op)) return rc;
    if (int rc = check_nrhs(n_tv)) return rc;
    if (!Q || !Dc16) return set_error(MRHS_EINVAL, "null argument");
    if (int rc = check_dtype(q_dtype)) return rc;
    return launch_coarse(op, Q, q_dtype, n_tv, Dc16, MRHS_DTYPE_F16, (hipStream_t)stream);
}

size_t mrhs_coarse_vector_bytes(const mrhs_op *op, int32_t n_tv, int32_t n_rhs)
{
    if (!op || n_tv <= 0 || n_rhs <= 0) return 0;
    return (size_t)op->n_agg * 2 * n_tv * 2 * ((n_rhs + 3) / 4 * 4) * sizeof(float);
}

namespace {

int check_transfer(const mrhs_op *op, int n_tv, int n_rhs, int q_dtype)
{
    if (int rc = check_op(op)) return rc;
    if (int rc = check_nrhs(n_tv)) return rc;
    if (int rc = check_nrhs(n_rhs)) return rc;
    if (n_tv > 32 || n_rhs > 32) return set_error(MRHS_EUNSUPPORTED, "at most 32 test vectors and 32 right-hand sides");
    if (n_tv > 6 * op->Va) return set_error(MRHS_EINVAL, "more test vectors than rows of an aggregate half");
    if (int rc = check_dtype(q_dtype)) return rc;
    if (transfer_lds_bytes(op) > op->max_lds) return set_error(MRHS_EUNSUPPORTED, "aggregate too large for the LDS");
    return MRHS_OK;
}

}  // namespace

int restrict_mrhs(const mrhs_op *op, const void *Q, int32_t q_dtype, int32_t n_tv, const void *y, int32_t y_dtype,
                  float *yc, int32_t n_rhs, void *stream)
{
    if (int rc = check_transfer(op, n_tv, n_rhs, q_dtype)) return rc;
    if (int rc = check_dtype(y_dtype)) return rc;
    if (!Q || !y || !yc) return set_error(MRHS_EINVAL, "null argument");
    const size_t cb = mrhs_coarse_vector_bytes(op, n_tv, n_rhs);
    if (ranges_overlap(yc, cb, y, native_elems(op, n_rhs) * dtype_size(y_dtype)) ||
        ranges_overlap(yc, cb, Q, native_elems(op, n_tv) * dtype_size(q_dtype)))
        return set_error(MRHS_EINVAL, "coarse output overlaps an input");
    return launch_restrict(op, Q, q_dtype, n_tv, y, y_dtype, yc, n_rhs, (hipStream_t)stream);
}

int prolong_mrhs(const mrhs_op *op, const void *Q, int32_t q_dtype, int32_t n_tv, const float *yc, void *y,
                 int32_t y_dtype, int32_t n_rhs, void *stream)
{
    if (int rc = check_transfer(op, n_tv, n_rhs, q_dtype)) return rc;
    if (int rc = check_dtype(y_dtype)) return rc;
    if (!Q || !y || !yc) return set_error(MRHS_EINVAL, "null argument");
    const size_t yb = native_elems(op, n_rhs) * dtype_size(y_dtype);
    if (ranges_overlap(y, yb, yc, mrhs_coarse_vector_bytes(op, n_tv, n_rhs)) ||
        ranges_overlap(y, yb, Q, native_elems(op, n_tv) * dtype_size(q_dtype)))
        return set_error(MRHS_EINVAL, "fine output overlaps an input");
    return launch_prolong(op, Q, q_dtype, n_tv, yc, y, y_dtype, n_rhs, (hipStream_t)stream);
}

int coarse_apply_mrhs(const mrhs_op *op, const float *Dc, int32_t n_tv, const float *yc, float *yc_out,
                      int32_t n_rhs, void *stream)
{
    if (int rc = check_transfer(op, n_tv, n_rhs, MRHS_DTYPE_F32)) return rc;
    if (!Dc || !yc || !yc_out) return set_error(MRHS_EINVAL, "null argument");
    const size_t cb = mrhs_coarse_vector_bytes(op, n_tv, n_rhs);
    if (ranges_overlap(yc_out, cb, yc, cb) ||
        ranges_overlap(yc_out, cb, Dc, (size_t)op->n_agg * 9 * 4 * n_tv * n_tv * 2 * sizeof(float)))
        return set_error(MRHS_EINVAL, "coarse output overlaps an input");
    return launch_coarse_apply(op, Dc, n_tv, yc, yc_out, n_rhs, (hipStream_t)stream);
}

int coarse_apply_f16_mrhs(const mrhs_op *op, const void *Dc16, int32_t n_tv, const float *yc, float *yc_out,
                          int32_t n_rhs, void *stream)
{
    if (int rc = check_transfer(op, n_tv, n_rhs, MRHS_DTYPE_F32)) return rc;
    if (!Dc16 || !yc || !yc_out) return set_error(MRHS_EINVAL, "null argument");
    const size_t cb = mrhs_coarse_vector_bytes(op, n_tv, n_rhs);
    if (ranges_overlap(yc_out, cb, yc, cb) ||
        ranges_overlap(yc_out, cb, Dc16, (size_t)op->n_agg * 9 * 4 * n_tv * n_tv * 2 * sizeof(__half)))
        return set_error(MRHS_EINVAL, "coarse output overlaps an input");
    return launch_coarse_apply_f16(op, (const __half *)Dc16, n_tv, yc, yc_out, n_rhs, (hipStream_t)stream);
}

size_t mrhs_coarse_solve_f16_workspace_bytes(const mrhs_op *op, int32_t n_tv, int32_t n_rhs, int32_t m)
{
    if (!op || n_tv <= 0 || n_rhs <= 0 || m <= 0) return 0;
    return ws_bytes_coarse_solve_f16(op, n_tv, n_rhs, m);
}

int coarse_solve_f16_mrhs(const mrhs_op *op, const void *Dc16, int32_t n_tv, const float *bc, float *uc, int32_t n_rhs,
                          int32_t m, double tol, double *res_out, int32_t *iters_out, void *ws, size_t ws_bytes,
                          void *stream)
{
    if (int rc = check_transfer(op, n_tv, n_rhs, MRHS_DTYPE_F32)) return rc;
    if (!Dc16 || !bc || !uc) return set_error(MRHS_EINVAL, "null argument");
    if (m < 1 || m > 64) return set_error(MRHS_EINVAL, "iteration count must be 1..64");
    if (!(tol >= 0.0)) return set_error(MRHS_EINVAL, "tolerance must be >= 0");
    const size_t need = ws_bytes_coarse_solve_f16(op, n_tv, n_rhs, m);
    if (!ws || ws_bytes < need) return set_error(MRHS_EINVAL, "workspace too small");
    const size_t cb = mrhs_coarse_vector_bytes(op, n_tv, n_rhs);
    if (ranges_overlap(uc, cb, bc, cb) || ranges_overlap(uc, cb, ws, need) || ranges_overlap(bc, cb, ws, need) ||
        ranges_overlap(uc, cb, Dc16, (size_t)op->n_agg * 9 * 4 * n_tv * n_tv * 2 * sizeof(__half)))
        return set_error(MRHS_EINVAL, "coarse vectors overlap each other, D_c or the workspace");
    return launch_coarse_solve_f16(op, (const __half *)Dc16, n_tv, bc, uc, n_rhs, m, tol, res_out, iters_out, ws,
                                   (hipStream_t)stream);
}

size_t mrhs_coarse_solve_workspace_bytes(const mrhs_op *op, int32_t n_tv, int32_t n_rhs, int32_t m)
{
    if (!op || n_tv <= 0 || n_rhs <= 0 || m <= 0) return 0;
    return ws_bytes_coarse_solve(op, n_tv, n_rhs, m);
}

int coarse_solve_mrhs(const mrhs_op *op, const float *Dc, int32_t n_tv, const float *bc, float *uc, int32_t n_rhs,
                      int32_t m, double tol, double *res_out, int32_t *iters_out, void *ws, size_t ws_bytes,
                      void *stream)
{
    if (int rc = check_transfer(op, n_tv, n_rhs, MRHS_DTYPE_F32)) return rc;
    if (!Dc || !bc || !uc) return set_error(MRHS_EINVAL, "null argument");
    if (m < 1 || m > 64) return set_error(MRHS_EINVAL, "iteration count must be 1..64");
    if (!(tol >= 0.0)) return set_error(MRHS_EINVAL, "tolerance must be >= 0");
    const size_t need = ws_bytes_coarse_solve(op, n_tv, n_rhs, m);
    if (!ws || ws_bytes < need) return set_error(MRHS_EINVAL, "workspace too small");
    const size_t cb = mrhs_coarse_vector_bytes(op, n_tv, n_rhs);
    if (ranges_overlap(uc, cb, bc, cb) || ranges_overlap(uc, cb, ws, need) || ranges_overlap(bc, cb, ws, need) ||
        ranges_overlap(uc, cb, Dc, (size_t)op->n_agg * 9 * 4 * n_tv * n_tv * 2 * sizeof(float)))
        return set_error(MRHS_EINVAL, "coarse vectors overlap each other, D_c or the workspace");
    return launch_coarse_solve(op, Dc, n_tv, bc, uc, n_rhs, m, tol, res_out, iters_out, ws, (hipStream_t)stream);
}

int coarse_self_invert(const mrhs_op *op, const float *Dc, int32_t n_tv, float *Dinv, int32_t *status, void *stream)
{
    if (int rc = check_op(op)) return rc;
    if (n_tv < 1 || n_tv > 32) return set_error(MRHS_EUNSUPPORTED, "n_tv must be 1..32");
    if (!Dc || !Dinv) return set_error(MRHS_EINVAL, "null argument");
    const size_t n2 = (size_t)4 * n_tv * n_tv;
    if (ranges_overlap(Dinv, (size_t)op->n_agg * n2 * 2 * sizeof(float), Dc, (size_t)op->n_agg * 9 * n2 * 2 * sizeof(float)))
        return set_error(MRHS_EINVAL, "Dinv overlaps D_c");
    return launch_coarse_self_inverse(op, Dc, n_tv, Dinv, status, (hipStream_t)stream);
}

size_t mrhs_coarse_solve_eo_workspace_bytes(const mrhs_op *op, int32_t n_tv, int32_t n_rhs, int32_t m)
{
    if (!op || n_tv <= 0 || n_rhs <= 0 || m <= 0) return 0;
    return ws_bytes_coarse_solve_eo(op, n_tv, n_rhs, m);
}

int coarse_solve_eo_mrhs(const mrhs_op *op, const float *Dc, const float *Dinv, int32_t n_tv, const float *bc, float *uc,
                         int32_t n_rhs, int32_t m, double tol, double *res_out, int32_t *iters_out, void *ws,
                         size_t ws_bytes, void *stream)
{
    if (int rc = check_transfer(op, n_tv, n_rhs, MRHS_DTYPE_F32)) return rc;
    if (!Dc || !Dinv || !bc || !uc) return set_error(MRHS_EINVAL, "null argument");
    for (int mu = 0; mu < 4; ++mu)
        if (op->na[mu] % 2)
            return set_error(MRHS_EUNSUPPORTED, "the even-odd coarse solve needs an even coarse extent in every direction");
    if (m < 1 || m > 64) return set_error(MRHS_EINVAL, "iteration count must be 1..64");
    if (!(tol >= 0.0)) return set_error(MRHS_EINVAL, "tolerance must be >= 0");
    const size_t need = ws_bytes_coarse_solve_eo(op, n_tv, n_rhs, m);
    if (!ws || ws_bytes < need) return set_error(MRHS_EINVAL, "workspace too small");
    const size_t cb = mrhs_coarse_vector_bytes(op, n_tv, n_rhs);
    const size_t n2 = (size_t)4 * n_tv * n_tv;
    if (ranges_overlap(uc, cb, bc, cb) || ranges_overlap(uc, cb, ws, need) || ranges_overlap(bc, cb, ws, need) ||
        ranges_overlap(uc, cb, Dc, (size_t)op->n_agg * 9 * n2 * 2 * sizeof(float)) ||
        ranges_overlap(uc, cb, Dinv, (size_t)op->n_agg * n2 * 2 * sizeof(float)))
        return set_error(MRHS_EINVAL, "coarse vectors overlap each other, D_c, Dinv or the workspace");
    return launch_coarse_solve_eo(op, Dc, Dinv, n_tv, bc, uc, n_rhs, m, tol, res_out, iters_out, ws,
                                  (hipStream_t)stream);
}

size_t mrhs_refine_workspace_bytes(const mrhs_op *op, int32_t n_tv, int32_t m)
{
    if (!op || n_tv <= 0 || m <= 0) return 0;
    return ws_bytes_refine(op, n_tv, m);
}

int setup_refine_mrhs(const mrhs_op *op, void *V, int32_t n_tv, const void *Q, int32_t q_dtype, const float *Dc,
                      int32_t n_sap, int32_t n_mr, int32_t m, double tol, void *ws, size_t ws_bytes, void *stream)
{
    if (int rc = check_transfer(op, n_tv, n_tv, q_dtype)) return rc;
    if (!V || !Q || !Dc) return set_error(MRHS_EINVAL, "null argument");
    if (n_sap < 0 || n_mr < 0) return set_error(MRHS_EINVAL, "negative iteration count");
    if (m < 1 || m > 64) return set_error(MRHS_EINVAL, "iteration count must be 1..64");
    if (!(tol >= 0.0)) return set_error(MRHS_EINVAL, "tolerance must be >= 0");
    const size_t need = ws_bytes_refine(op, n_tv, m);
    if (!ws || ws_bytes < need) return set_error(MRHS_EINVAL, "workspace too small");
    const size_t vb = native_elems(op, n_tv) * dtype_size(op->dtype);
    const size_t qb = native_elems(op, n_tv) * dtype_size(q_dtype);
    if (ranges_overlap(V, vb, Q, qb) || ranges_overlap(ws, need, V, vb) || ranges_overlap(ws, need, Q, qb) ||
        ranges_overlap(ws, need, Dc, (size_t)op->n_agg * 9 * 4 * n_tv * n_tv * 2 * sizeof(float)))
        return set_error(MRHS_EINVAL, "test vectors, Q, D_c and the workspace must not overlap");
    return launch_refine(op, V, n_tv, Q, q_dtype, Dc, n_sap, n_mr, m, tol, ws, (hipStream_t)stream);
}

size_t mrhs_batched_workspace_bytes(mrhs_op *const *ops, int32_t n_inst, const int32_t *n_rhs)
{
    if (!ops || !n_rhs || n_inst <= 0) return 0;
    for (int k = 0; k < n_inst; ++k)
        if (!ops[k] || n_rhs[k] <= 0) return 0;
    return std::max(ws_bytes_sap_batched(ops, n_inst, n_rhs), (size_t)256);
}

int sap_smooth_mrhs_batched(mrhs_op *const *ops, int32_t n_inst, const void *const *b, void *const *x,
                            const int32_t *n_rhs, int32_t n_sap, int32_t n_mr, void *ws, size_t ws_bytes,
                            void *stream)
{
    if (!ops || !b || !x || !n_rhs) return set_error(MRHS_EINVAL, "null argument");
    if (n_inst <= 0 || n_inst > 8) return set_error(MRHS_EINVAL, "n_inst must be 1..8");
    if (n_sap < 0 || n_mr < 0) return set_error(MRHS_EINVAL, "negative iteration count");
    for (int k = 0; k < n_inst; ++k) {
        if (int rc = check_op(ops[k])) return rc;
        if (int rc = check_nrhs(n_rhs[k])) return rc;
        if (!b[k] || !x[k]) return set_error(MRHS_EINVAL, "null vector");
        if (ops[k]->prec != ops[0]->prec || ops[k]->k.S != ops[0]->k.S)
            return set_error(MRHS_EINVAL, "all operators of a batch need the same precision and short length");
        const size_t bytes = native_elems(ops[k], n_rhs[k]) * dtype_size(ops[k]->dtype);
        for (int j = 0; j <= k; ++j) {
            const size_t bj = native_elems(ops[j], n_rhs[j]) * dtype_size(ops[j]->dtype);
            if (ranges_overlap(b[k], bytes, x[j], bj) || (j < k && ranges_overlap(x[k], bytes, x[j], bj)))
                return set_error(MRHS_EINVAL, "vectors of the batch overlap");
        }
    }
    const size_t need = ws_bytes_sap_batched(ops, n_inst, n_rhs);
    if (need && (!ws || ws_bytes < need)) return set_error(MRHS_EINVAL, "workspace too small");
    return launch_sap_batched(ops, n_inst, b, x, n_rhs, n_sap, n_mr, ws, (hipStream_t)stream);
}

int mrhs_set_tiles(mrhs_op *op, int32_t sap_tile, int32_t dirac_tile)
{
    if (int rc = check_op(op)) return rc;
    auto ok = [&](int t) { return t == 1 || t == 2 || t == 4; };
    if (sap_tile) {
        if (!ok(sap_tile) || op->k.S % sap_tile || op->k.Vb * sap_tile > 1024)
            return set_error(MRHS_EINVAL, "SAP tile must be 1, 2 or 4, divide S and fit the block");
        if (sap_lds_bytes(op, sap_tile) > op->max_lds)
            return set_error(MRHS_EUNSUPPORTED, "SAP tile exceeds the LDS of a workgroup");
        if (!tile_built(op, sap_tile))
            return set_error(MRHS_EUNSUPPORTED, "SAP tiles above 2 are not built for FP64 arithmetic");
        op->sap_tile = sap_tile;
    }
    if (dirac_tile) {
        if (!ok(dirac_tile) || op->k.S % dirac_tile || op->k.Vb * dirac_tile > 1024)
            return set_error(MRHS_EINVAL, "stencil tile must be 1, 2 or 4, divide S and fit the block");
        if (!tile_built(op, dirac_tile))
            return set_error(MRHS_EUNSUPPORTED, "stencil tiles above 2 are not built for FP64 arithmetic");
        op->dirac_tile = dirac_tile;
    }
    return MRHS_OK;
}

int mrhs_op_block_solver(const mrhs_op *op) { return op ? op->block_solver : MRHS_EINVAL; }

int mrhs_set_block_solver(mrhs_op *op, int32_t solver, void *stream)
{
    if (int rc = check_op(op)) return rc;
    if (solver == MRHS_BLOCK_MR) {
        op->block_solver = MRHS_BLOCK_MR;
        return MRHS_OK;
    }
    if (solver != MRHS_BLOCK_EO_MR) return set_error(MRHS_EINVAL, "unknown block solver");
    for (int mu = 0; mu < 4; ++mu)
        if (op->k.b[mu] % 2) return set_error(MRHS_EUNSUPPORTED, "the even-odd block solver needs even block extents");
    if (!op->cloverinv64) {
        const long V = op->k.V;
        const int Vb = op->k.Vb;
        std::vector<int32_t> order;
        for (int p = 0; p < 2; ++p)
            for (int off = 0; off < Vb; ++off) {
                int q = off, par = 0;
                for (int mu = 0; mu < 4; ++mu) {
                    par += q % op->k.b[mu];
                    q /= op->k.b[mu];
                }
                if ((par & 1) == p) order.push_back(off);
            }
        hipStream_t st = (hipStream_t)stream;
        double *inv64 = nullptr;
        float *inv32 = nullptr;
        int32_t *eo = nullptr;
        int *bad = nullptr;
        int rc = hip_check(hipMalloc((void **)&inv64, sizeof(double) * 72 * V), "hipMalloc cloverinv64");
        if (!rc && op->clover32) rc = hip_check(hipMalloc((void **)&inv32, sizeof(float) * 72 * V), "hipMalloc cloverinv32");
        if (!rc) rc = hip_check(hipMalloc((void **)&eo, sizeof(int32_t) * Vb), "hipMalloc eo_sites");
        if (!rc) rc = hip_check(hipMalloc((void **)&bad, sizeof(int)), "hipMalloc flag");
        if (!rc) rc = hip_check(hipMemcpyAsync(eo, order.data(), sizeof(int32_t) * Vb, hipMemcpyHostToDevice, st), "copy");
        if (!rc) rc = hip_check(hipMemsetAsync(bad, 0, sizeof(int), st), "hipMemsetAsync flag");
        if (!rc) {
            op->cloverinv64 = inv64;
            op->cloverinv32 = inv32;
            rc = launch_clover_inverse(op, bad, st);
        }
        int hbad = 0;
        if (!rc) rc = hip_check(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, st), "copy flag");
        if (!rc) rc = hip_check(hipStreamSynchronize(st), "hipStreamSynchronize(set_block_solver)");
        if (bad) (void)hipFree(bad);
        if (!rc && hbad) rc = set_error(MRHS_EINVAL, "the clover term has a singular 6x6 block");
        if (rc) {
            (void)hipStreamSynchronize(st);
            if (inv64) (void)hipFree(inv64);
            if (inv32) (void)hipFree(inv32);
            if (eo) (void)hipFree(eo);
            op->cloverinv64 = nullptr;
            op->cloverinv32 = nullptr;
            return rc;
        }
        op->eo_sites = eo;
    }
    op->block_solver = MRHS_BLOCK_EO_MR;
    return MRHS_OK;
}

}  // extern "C"
