// launch.h -- host-side launchers and workspace sizes of the library's kernels (one per
// source file), used by the C-ABI in abi.hip.
#pragma once

#include "internal.h"

// A^-1 of the op's clover term per site (FP64, and FP32 when the op has FP32 fields);
// *bad (device) is set to 1 where a 6x6 block has no usable pivot
int launch_clover_inverse(mrhs_op *op, int *bad, hipStream_t st);
int launch_build_fields(mrhs_op *op, const double *links_canon, double m0, double csw, hipStream_t st);
int launch_pack(const mrhs_op *op, const double *canon, void *native, int dtype, int n_rhs, int *flag, hipStream_t st);
int launch_unpack(const mrhs_op *op, const void *native, int dtype, double *canon, int n_rhs, hipStream_t st);
int launch_dirac(const mrhs_op *op, const void *x, void *y, int n_rhs, hipStream_t st);
int launch_sap(const mrhs_op *op, const void *b, void *x, int n_rhs, int n_sap, int n_mr, void *ws, hipStream_t st,
               bool guess = false);
int launch_residual(const mrhs_op *op, const void *b, const void *x, int n_rhs, double *out, void *ws, hipStream_t st);
// the same with the library's static per-device scratch instead of a workspace (no allocation)
int launch_residual_noalloc(const mrhs_op *op, const void *b, const void *x, int n_rhs, double *out, hipStream_t st);
int launch_gs(const mrhs_op *op, const void *V, int vdt, void *Q, int qdt, int n_tv, int32_t *status, void *ws,
              hipStream_t st);
// D_c into Dc as complex64 (dcdt MRHS_DTYPE_F32) or as binary16 pairs (MRHS_DTYPE_F16)
int launch_coarse(const mrhs_op *op, const void *Q, int qdt, int n_tv, void *Dc, int dcdt, hipStream_t st);
size_t ws_bytes_sap(const mrhs_op *op, int n_rhs);
size_t ws_bytes_sap_batched(const mrhs_op *const *ops, int n, const int32_t *n_rhs);
int launch_sap_batched(const mrhs_op *const *ops, int n, const void *const *b, void *const *x, const int32_t *n_rhs,
                       int n_sap, int n_mr, void *ws, hipStream_t st, bool guess = false);
size_t ws_bytes_residual(const mrhs_op *op, int n_rhs);
size_t ws_bytes_gs(const mrhs_op *op, int n_tv);
size_t ws_bytes_coarse(const mrhs_op *op, int n_tv);
size_t native_elems(const mrhs_op *op, int n_rhs);
int dtype_size(int dtype);
int launch_restrict(const mrhs_op *op, const void *Q, int qdt, int n_tv, const void *y, int ydt, float *yc, int n,
                    hipStream_t st);
int launch_prolong(const mrhs_op *op, const void *Q, int qdt, int n_tv, const float *yc, void *y, int ydt, int n,
                   hipStream_t st);
int launch_coarse_apply(const mrhs_op *op, const float *Dc, int n_tv, const float *yc, float *yco, int n,
                        hipStream_t st);
// the general form: yco = y0 + D_self yself + s_hop * sum_d D_d yhop(nbr_d) with D = Dc[site][0..nblk),
// on every coarse site (parity -1) or those of one parity (the others zeroed or left untouched);
// null inputs drop their terms
// gate (nullable, gate_n flags): the launch does nothing when every flag is zero
int launch_coarse_apply_ex(const mrhs_op *op, const float *Dc, int nblk, int n_tv, const float *y0, const float *yself,
                           const float *yhop, float s_hop, int parity, bool zero_other, float *yco, int n,
                           hipStream_t st, const int *gate = nullptr, int gate_n = 0);
// yco = D_c yc with D_c stored in binary16 (as written by launch_coarse with MRHS_DTYPE_F16)
int launch_coarse_apply_f16(const mrhs_op *op, const __half *Dc16, int n_tv, const float *yc, float *yco, int n,
                            hipStream_t st, const int *gate = nullptr, int gate_n = 0);
size_t transfer_lds_bytes(const mrhs_op *op);
// even-odd preconditioned coarse solve and the self-block inverses it uses
size_t ws_bytes_coarse_solve_eo(const mrhs_op *op, int n_tv, int n, int m);
int launch_coarse_self_inverse(const mrhs_op *op, const float *Dc, int n_tv, float *Dinv, int32_t *status,
                               hipStream_t st);
int launch_coarse_solve_eo(const mrhs_op *op, const float *Dc, const float *Dinv, int n_tv, const float *b, float *u,
                           int n, int m, double tol, double *res_out, int32_t *iters_out, void *ws, hipStream_t st);
size_t ws_bytes_coarse_solve(const mrhs_op *op, int n_tv, int n, int m);
// the half-precision coarse grid: D_c and the Krylov basis in binary16, FP32 arithmetic
size_t ws_bytes_coarse_solve_f16(const mrhs_op *op, int n_tv, int n, int m);
int launch_coarse_solve_f16(const mrhs_op *op, const __half *Dc16, int n_tv, const float *b, float *u, int n, int m,
                            double tol, double *res_out, int32_t *iters_out, void *ws, hipStream_t st);
int launch_coarse_solve(const mrhs_op *op, const float *Dc, int n_tv, const float *b, float *u, int n, int m, double tol,
                        double *res_out, int32_t *iters_out, void *ws, hipStream_t st);
size_t ws_bytes_refine(const mrhs_op *op, int n_tv, int m);
int launch_refine(const mrhs_op *op, void *V, int n_tv, const void *Q, int qdt, const float *Dc, int n_sap, int n_mr,
                  int m, double tol, void *ws, hipStream_t st);
