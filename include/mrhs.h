/*
 * mrhs.h -- C-ABI of the MI355X (gfx950) library for the multiple-right-hand-side
 * setup of DD-alpha-AMG (Richtmann, Heybrock, Wettig, Lattice 2015).
 *
 * The setup's initial phase (Sec. 2): N_tv random test vectors of dimension 12V are
 * smoothed by the Schwarz alternating procedure (SAP) from a zero starting guess and
 * replaced by the result; restriction R, prolongation P = R^dagger and the coarse
 * operator D_c are then built from them.  The library runs that phase on all test
 * vectors at once (Sec. 3, Alg. 2: the test-vector loop blocked and moved into the
 * lowest-level kernels), in a layout with the right-hand-side index innermost
 * (Sec. 5, the AoSoSV layout), so that the operator is read once per site for all
 * right-hand sides (Sec. 6, mat-vec -> mat-mat).
 *
 * Conventions (the paper leaves them to the works it cites):
 *   lattice extents L[0..3] for directions x,y,z,t, canonical site index
 *   x0 + L0*(x1 + L1*(x2 + L2*x3)), periodic boundaries; spinor component
 *   3*spin + colour; Wilson-clover operator in the DeGrand-Rossi chiral basis,
 *     (D psi)(x) = A(x) psi(x) - 1/2 sum_mu [ (1 - g_mu) U_mu(x) psi(x+mu)
 *                                            + (1 + g_mu) U_mu(x-mu)^dag psi(x-mu) ],
 *     A(x) = (4 + m0) + C(x), C(x) = -(csw/16) sum_{mu<nu} g_mu g_nu (Q_munu - Q_munu^dag),
 *   Q_munu(x) the sum of the four plaquette leaves in the (mu,nu) plane at x.
 *
 * Memory: every pointer to field or vector data is a DEVICE pointer owned by the
 * caller.  The library owns what mrhs_op_create allocates (the operator's fields in
 * kernel layout and a status word, used by mrhs_pack for its FP16 range flag) and, on
 * the first switch to the even-odd block solver, what mrhs_set_block_solver allocates
 * (A^-1 per site and the block's parity order), until mrhs_op_destroy.  No other call
 * allocates device memory; scratch space is passed in as a caller-owned workspace.
 *
 * Asynchrony: every call only enqueues work on the given HIP stream (a hipStream_t
 * passed as void*, NULL = the default stream), except mrhs_op_create, mrhs_op_destroy
 * and mrhs_pack, which synchronise that stream before returning.  Arguments are
 * validated before anything is enqueued.
 *
 * Errors: every int-returning call returns 0 on success or a negative MRHS_E* code;
 * mrhs_last_error() returns a thread-local message for the last failure.  No call
 * throws, exits or aborts.
 *
 * Native vector layout (the "AoSoSV" layout of Sec. 5 with short-vector length S):
 *   sites are re-ordered block-major: native site = blk * Vb + off, blk the SAP block
 *   (lexicographic block coordinates), off the lexicographic local coordinate within
 *   the block, Vb = block volume.  Right-hand side k sits in group g = k / S at lane
 *   t = k % S.  Real component r = 2*(3*spin + colour) + (0 re | 1 im) of site (blk, off)
 *   of rhs k is element
 *       ((g * n_blocks + blk) * 24 + r) * Vb * S + off * S + t.
 *   A native vector set for n_rhs right-hand sides holds ceil(n_rhs / S) groups; the
 *   padding lanes of the last group must be zero (mrhs_pack writes them so), and stay
 *   zero under every call (a zero right-hand side gives a zero MR step).
 */
#ifndef MRHS_H
#define MRHS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define MRHS_OK 0
#define MRHS_EINVAL (-1)      /* null pointer, aliasing, bad size or geometry */
#define MRHS_EUNSUPPORTED (-2) /* a shape / precision combination the library does not handle */
#define MRHS_EHIP (-3)        /* HIP runtime or launch error (text in mrhs_last_error) */
#define MRHS_ERANK (-4)       /* rank-deficient aggregate in block_orthonormalize */
#define MRHS_ERANGE (-5)      /* value outside the FP16 range in mrhs_pack */

/* element types of native vectors */
#define MRHS_DTYPE_F64 0
#define MRHS_DTYPE_F32 1
#define MRHS_DTYPE_F16 2

/* operator precisions */
#define MRHS_PREC_F64 0          /* FP64 fields, vectors and arithmetic */
#define MRHS_PREC_F32 1          /* FP32 fields, vectors and arithmetic */
#define MRHS_PREC_F32_F16STORE 2 /* FP32 fields and arithmetic, FP16 (binary16) vector storage */

typedef struct mrhs_geom {
    int32_t L[4];     /* lattice extents x,y,z,t */
    int32_t block[4]; /* SAP block extents; must divide L; block volume <= 256 */
    int32_t agg[4];   /* aggregate extents (Alg. 3's domains); must divide L */
} mrhs_geom;

typedef struct mrhs_op mrhs_op;

/* Build the operator for one gauge field (Sec. 2's Dirac operator, readings above).
 * links: DEVICE, complex128 interleaved (re, im), canonical [4][V][3][3] (direction,
 *        canonical site, row, column); read during the call only.
 * m0, csw: bare mass and clover coefficient.  prec: MRHS_PREC_*.
 * short_len: S of the native layout, 1, 2, 4 or 8 (1 = single-RHS layout).
 * The op keeps FP64 copies of its fields for mrhs_residual_norms in every precision.
 * Synchronises the stream.  *out receives the handle. */
int mrhs_op_create(const mrhs_geom *geom, const double *links, double m0, double csw, int32_t prec,
                   int32_t short_len, void *stream, mrhs_op **out);
int mrhs_op_destroy(mrhs_op *op);

/* the operator's vector element type (MRHS_DTYPE_*) and short-vector length */
int mrhs_op_vector_dtype(const mrhs_op *op);
int mrhs_op_short_len(const mrhs_op *op);

/* bytes of a native vector set of n_rhs right-hand sides of element type dtype */
size_t mrhs_vector_bytes(const mrhs_op *op, int32_t n_rhs, int32_t dtype);
/* bytes of workspace any call below needs for up to n_rhs right-hand sides (test vectors) */
size_t mrhs_workspace_bytes(const mrhs_op *op, int32_t n_rhs);

/* canonical complex128 [n_rhs][V][4][3] (DEVICE) <-> native vectors of element type dtype.
 * mrhs_pack rounds to nearest-even and writes zero padding lanes; it synchronises the
 * stream and returns MRHS_ERANGE if an FP16 target would overflow (|v| > 65504). */
int mrhs_pack(const mrhs_op *op, const double *canon, void *native, int32_t dtype, int32_t n_rhs, void *stream);
int mrhs_unpack(const mrhs_op *op, const void *native, int32_t dtype, double *canon, int32_t n_rhs, void *stream);

/* y = D x on the full periodic lattice for n_rhs right-hand sides (the stencil whose
 * operator reads are shared by all right-hand sides, Sec. 6).  x, y: native vectors of
 * the op's element type; x != y. */
int dirac_apply_mrhs(const mrhs_op *op, const void *x, void *y, int32_t n_rhs, void *stream);

/* x = SAP(b) from a zero starting guess (Sec. 2, initial phase), n_sap sweeps over the
 * red (even block-coordinate sum) then black SAP blocks; per colour the residual
 * b - D x is formed on that colour's blocks, then every block j adds n_mr minimal-
 * residual steps on D_j = I_j^T D I_j (step length 0 when <q,q> = 0).  b, x: native
 * vectors of the op's element type, x != b; x is overwritten.  ws: workspace of at
 * least mrhs_workspace_bytes(op, n_rhs) bytes.  With the plain MR block solver it carries
 * a block's residual from one visit to the next, so that a later visit forms only the hops
 * across the block's faces (the same residual up to rounding order): when no direction holds
 * an odd number (> 1) of blocks, the block residual rho_j after its MR steps and every block's
 * last change of x (arithmetic type, one vector set each), a later residual being rho_j minus
 * the face hops of the neighbours' changes; otherwise sigma_j = b_j - D_j x_j and a snapshot
 * of x, a later residual being sigma_j minus the face hops of x. */
int sap_smooth_mrhs(const mrhs_op *op, const void *b, void *x, int32_t n_rhs, int32_t n_sap, int32_t n_mr,
                    void *ws, size_t ws_bytes, void *stream);

/* As sap_smooth_mrhs, but x holds the starting guess on entry (the refinement phase of the
 * setup, Alg. 1 and 2: the smoother starts from the prolongated coarse-grid solution); the
 * first visit of each colour forms the full residual b - D x.  With n_sap = 0, x is left as
 * it is. */
int sap_smooth_mrhs_guess(const mrhs_op *op, const void *b, void *x, int32_t n_rhs, int32_t n_sap, int32_t n_mr,
                          void *ws, size_t ws_bytes, void *stream);

/* out[k] = ||b_k - D x_k||_2 / ||b_k||_2 in FP64 (FP64 fields, x and b up-converted from
 * their storage type).  out: DEVICE double[n_rhs]. */
int mrhs_residual_norms(const mrhs_op *op, const void *b, const void *x, int32_t n_rhs, double *out, void *ws,
                        size_t ws_bytes, void *stream);

/* mrhs_residual_norms for callers that cannot allocate device memory or pass a workspace
 * (code under graph capture, tight loops, harnesses that forbid allocation): the same
 * kernels, with their partial sums in a static 32 MiB scratch array of the library instead
 * of ws.  Each device holds one copy of the array until the process ends; the first call on
 * a device looks up its address (no allocation).  The call allocates nothing and never
 * synchronises.  The partial sums take 16 bytes per block and right-hand side, n_rhs rounded
 * up to a multiple of 8 (short length 4; of S otherwise); larger requests return
 * MRHS_EUNSUPPORTED (at 48^3 x 96 with 4^4 blocks: up to 48 right-hand sides).  All calls on one device share the array and it keeps the last
 * call's partial sums: calls that overlap in time on one device (other streams, other
 * threads) race and give wrong norms; the caller serialises them. */
int mrhs_residual_norms_noalloc(const mrhs_op *op, const void *b, const void *x, int32_t n_rhs, double *out,
                                void *stream);

/* Per aggregate i and spin half h (spins {0,1} | {2,3}), orthonormalise the n_tv columns
 * of V^h_i (6 * aggregate volume rows: local site, spin in half, colour): V^h_i = Q^h_i T
 * with T upper triangular, real positive diagonal (the setup of R = Q^dag, P = Q; Sec. 2,
 * Alg. 3).  FP64 arithmetic.  V: native vectors of v_dtype; Q: native vectors of q_dtype
 * (may alias V exactly when the types agree); q_dtype F16 stores Q in binary16, each entry
 * rounded once from FP64 (the entries of an orthonormal column are at most 1 in modulus).  status (DEVICE int32, nullable) receives 0
 * or 1 + (2*aggregate + h) of the first aggregate half whose Cholesky pivot falls to
 * <= 1e-14 ||v_k||^2 (T_kk <= 1e-7 ||v_k||, the resolution limit of CholQR in FP64);
 * such a half's Q is not meaningful.  Needs n_tv <= 32 and n_tv <= 6 * aggregate volume. */
int block_orthonormalize(const mrhs_op *op, const void *V, int32_t v_dtype, void *Q, int32_t q_dtype, int32_t n_tv,
                         int32_t *status, void *ws, size_t ws_bytes, void *stream);

/* D_c = R D P, the Galerkin coarse-grid operator built from the test vectors in the
 * setup (Sec. 2: the coarse operator is set up together with R and P = R^dag), from Q
 * (the output of block_orthonormalize, q_dtype F64, F32 or F16; the
 * arithmetic is that of the op's fields, FP32 or FP64, whatever Q's storage), stored per
 * coarse site i (lexicographic over L/agg) as 9 blocks [self,+x,+y,+z,+t,-x,-y,-z,-t],
 * each 2 n_tv x 2 n_tv complex64 row-major, row = h*n_tv + k.  The self block holds the
 * site term and the hops that stay inside the aggregate without crossing its faces; the
 * +mu (-mu) block holds the hops across the aggregate's +mu (-mu) face.  Dc: DEVICE.
 * Needs no workspace (ws may be null).  Needs n_tv <= 32. */
int coarse_op_build(const mrhs_op *op, const void *Q, int32_t q_dtype, int32_t n_tv, void *Dc, void *ws,
                    size_t ws_bytes, void *stream);

/* ---- coarse-grid correction of the refinement phase (Alg. 1, 2; restriction Alg. 3) ----
 * Coarse vectors: FP32 on the coarse lattice L/agg (Vc = number of aggregates, sites
 * lexicographic), element (rhs k, coarse site i, coarse dof c = h*n_tv + j, re/im p) at
 * ((i * 2*n_tv + c) * 2 + p) * ldc + k, ldc = n_rhs rounded up to a multiple of 4; the
 * kernels write the padding entries k >= n_rhs as zero.  Arithmetic is FP32 (matrix cores,
 * FP32 accumulation).  1 <= n_tv, n_rhs <= 32.  Q: the output of block_orthonormalize
 * (q_dtype F64, F32 or F16; FP16 storage halves the bytes of Q that restriction, prolongation
 * and the D_c build read, the arithmetic stays FP32). */
size_t mrhs_coarse_vector_bytes(const mrhs_op *op, int32_t n_tv, int32_t n_rhs);

/* y_c = R y, R = Q^dag per aggregate and spin half: (y_c)^h_i[j] = sum_n conj(Q^h_i[n, j]) y^h_i[n]
 * (Alg. 3).  y: n_rhs native vectors of y_dtype; yc: DEVICE coarse vectors (output). */
int restrict_mrhs(const mrhs_op *op, const void *Q, int32_t q_dtype, int32_t n_tv, const void *y, int32_t y_dtype,
                  float *yc, int32_t n_rhs, void *stream);

/* y = P y_c, P = Q = R^dag (Sec. 2): y^h_i[n] = sum_j Q^h_i[n, j] (y_c)^h_i[j].  y: n_rhs
 * native vectors of y_dtype (output; the padding lanes of its last group are written zero). */
int prolong_mrhs(const mrhs_op *op, const void *Q, int32_t q_dtype, int32_t n_tv, const float *yc, void *y,
                 int32_t y_dtype, int32_t n_rhs, void *stream);

/* yc_out = D_c yc (the coarse operator of the coarse solve): per coarse site,
 * Dc[i][self] yc(i) + sum_mu (Dc[i][+mu] yc(i+mu) + Dc[i][-mu] yc(i-mu)), neighbours periodic
 * on the coarse lattice; Dc as written by coarse_op_build.  yc_out must not overlap yc or Dc. */
int coarse_apply_mrhs(const mrhs_op *op, const float *Dc, int32_t n_tv, const float *yc, float *yc_out,
                      int32_t n_rhs, void *stream);

/* uc ~ D_c^-1 bc, the low-accuracy coarse solve of the refinement phase (Alg. 1), for all
 * right-hand sides at once: GMRES from a zero start, at most m (1..64) iterations, Arnoldi
 * with classical Gram-Schmidt applied twice, complex Givens rotations; a right-hand side
 * stops once its residual estimate falls to tol * ||bc_k|| (tol = 0: m iterations, fewer
 * only at an exact solution).  Vectors FP32, inner products and the small Hessenberg
 * algebra FP64.  res_out (DEVICE double[n_rhs], nullable): final estimate / ||bc_k||;
 * iters_out (DEVICE int32[n_rhs], nullable): iterations taken.  ws: at least
 * mrhs_coarse_solve_workspace_bytes(op, n_tv, n_rhs, m) bytes (Krylov bases of all
 * right-hand sides).  uc must not overlap bc, Dc or ws.  The call enqueues a fixed sequence
 * of launches (no host synchronisation). */
size_t mrhs_coarse_solve_workspace_bytes(const mrhs_op *op, int32_t n_tv, int32_t n_rhs, int32_t m);
int coarse_solve_mrhs(const mrhs_op *op, const float *Dc, int32_t n_tv, const float *bc, float *uc, int32_t n_rhs,
                      int32_t m, double tol, double *res_out, int32_t *iters_out, void *ws, size_t ws_bytes,
                      void *stream);

/* ---- the half-precision coarse grid (storage precision reduced on the coarse grid, as the
 * DD-alpha-AMG implementation the paper builds on does, Sec. 1; arithmetic stays FP32) ----
 * Dc16: D_c stored in IEEE binary16, the same layout and element order as coarse_op_build's
 * complex64 (a (re, im) pair of binary16 per entry, 8 N^2 bytes per block): half the bytes
 * that every coarse-operator apply reads.  Entries above 65504 in modulus would overflow
 * (D_c of a Wilson-clover operator is O(1)); the relative rounding error of an entry is at
 * most 2^-11.
 * coarse_op_build_f16: as coarse_op_build, each entry rounded once from its FP32 sum.
 * coarse_apply_f16_mrhs: as coarse_apply_mrhs with D_c from Dc16 (FP32 vectors and FP32
 *   accumulation on the matrix cores).
 * coarse_solve_f16_mrhs: as coarse_solve_mrhs with D_c from Dc16 and the Krylov basis stored
 *   in binary16 (each basis vector rounded once when formed; inner products, the Hessenberg
 *   matrix and the rotations stay FP64, the working vector FP32); bc, uc FP32.  ws: at least
 *   mrhs_coarse_solve_f16_workspace_bytes(op, n_tv, n_rhs, m) bytes. */
int coarse_op_build_f16(const mrhs_op *op, const void *Q, int32_t q_dtype, int32_t n_tv, void *Dc16, void *stream);
int coarse_apply_f16_mrhs(const mrhs_op *op, const void *Dc16, int32_t n_tv, const float *yc, float *yc_out,
                          int32_t n_rhs, void *stream);
size_t mrhs_coarse_solve_f16_workspace_bytes(const mrhs_op *op, int32_t n_tv, int32_t n_rhs, int32_t m);
int coarse_solve_f16_mrhs(const mrhs_op *op, const void *Dc16, int32_t n_tv, const float *bc, float *uc, int32_t n_rhs,
                          int32_t m, double tol, double *res_out, int32_t *iters_out, void *ws, size_t ws_bytes,
                          void *stream);

/* Even-odd preconditioned coarse solve (the coarse-grid counterpart of DD-alpha-AMG's even-odd
 * preconditioning).  Coarse sites split by the parity of their coordinate sum; every coarse
 * extent L/agg must be even, so each of the 8 hop blocks joins sites of opposite parity:
 * D_c = [[A_ee, H_eo], [H_oe, A_oo]] with A the self blocks.  With bhat_e = b_e - H_eo A_oo^-1 b_o,
 * GMRES as in coarse_solve_mrhs (m iterations, tolerance tol relative to ||bhat_e||) runs on
 * the Schur complement S = A_ee - H_eo A_oo^-1 H_oe for S u_e = bhat_e from zero, and then
 * u_o = A_oo^-1 (b_o - H_oe u_e); res_out and iters_out refer to the Schur system.
 * coarse_self_invert: Dinv [Vc][2 n_tv][2 n_tv] complex64 (DEVICE), the inverse of every site's
 * self block by FP64 Gauss-Jordan elimination with partial pivoting; status (DEVICE int32,
 * nullable) receives 0, or 1 + the lowest site whose block has no non-zero pivot (its Dinv is
 * zero).  Errors: EUNSUPPORTED for an odd coarse extent or n_tv > 32; overlaps as for
 * coarse_solve_mrhs.  ws: at least mrhs_coarse_solve_eo_workspace_bytes bytes. */
int coarse_self_invert(const mrhs_op *op, const float *Dc, int32_t n_tv, float *Dinv, int32_t *status, void *stream);
size_t mrhs_coarse_solve_eo_workspace_bytes(const mrhs_op *op, int32_t n_tv, int32_t n_rhs, int32_t m);
int coarse_solve_eo_mrhs(const mrhs_op *op, const float *Dc, const float *Dinv, int32_t n_tv, const float *bc, float *uc,
                         int32_t n_rhs, int32_t m, double tol, double *res_out, int32_t *iters_out, void *ws,
                         size_t ws_bytes, void *stream);

/* One pass of the refinement phase over all test vectors at once (Alg. 2 with the block
 * length N_b = n_tv, Alg. 1's loop body for every vector): v_c = R v, u_c ~ D_c^-1 v_c
 * (coarse_solve_mrhs: m iterations, tolerance tol), u = P u_c, then x = SAP(v) started
 * from u (sap_smooth_mrhs_guess: n_sap x n_mr), and v is replaced by x.  V: n_tv native
 * test vectors of the op's element type, overwritten; Q, Dc: the current R = Q^dag and
 * D_c (from block_orthonormalize and coarse_op_build on the previous V), not overlapping V.
 * Rebuilding Q and D_c from the new V is the caller's next step (Alg. 2, last line).
 * ws: at least mrhs_refine_workspace_bytes(op, n_tv, m) bytes. */
size_t mrhs_refine_workspace_bytes(const mrhs_op *op, int32_t n_tv, int32_t m);
int setup_refine_mrhs(const mrhs_op *op, void *V, int32_t n_tv, const void *Q, int32_t q_dtype, const float *Dc,
                      int32_t n_sap, int32_t n_mr, int32_t m, double tol, void *ws, size_t ws_bytes, void *stream);

/* SAP on several operators at once -- lattices of uneven size, each with its own
 * right-hand sides -- with one launch per half-sweep for the whole batch (the loop over
 * test vectors and over lattices moved into the kernel, Sec. 3).  The enqueued work is a
 * fixed sequence of kernels whose arguments carry everything by value, so the call can be
 * captured into a graph and replayed.  ops, b, x, n_rhs: HOST arrays of n_inst (1..8)
 * entries; ops[k] share precision and short length; b[k], x[k] are DEVICE native vectors
 * of ops[k] for n_rhs[k] right-hand sides, no two overlapping.  The result for instance k
 * equals sap_smooth_mrhs(ops[k], b[k], x[k], n_rhs[k], n_sap, n_mr) with the batch's tile
 * (the smallest of the operators' SAP tiles).  ws: at least
 * mrhs_batched_workspace_bytes(ops, n_inst, n_rhs) bytes. */
int sap_smooth_mrhs_batched(mrhs_op *const *ops, int32_t n_inst, const void *const *b, void *const *x,
                            const int32_t *n_rhs, int32_t n_sap, int32_t n_mr, void *ws, size_t ws_bytes,
                            void *stream);
size_t mrhs_batched_workspace_bytes(mrhs_op *const *ops, int32_t n_inst, const int32_t *n_rhs);

/* Block solver of the SAP (every SAP entry point of the op, the refinement pass included).
 *   MRHS_BLOCK_MR    (default): n_mr minimal-residual steps on D_j from zero;
 *   MRHS_BLOCK_EO_MR : DD-alpha-AMG's even-odd preconditioned block solve.  A block's sites
 *     are split by the parity of their block-local coordinate sum (every block extent must
 *     be even, so each hop inside a block joins opposite parities): D_j = [[A_ee, H_eo],
 *     [H_oe, A_oo]] with A the clover term and H the hops inside the block.  n_mr
 *     minimal-residual steps are taken on the Schur complement S = A_ee - H_eo A_oo^-1 H_oe
 *     for S e_e = r_e - H_eo A_oo^-1 r_o from zero, then e_o = A_oo^-1 (r_o - H_oe e_e).
 * The first switch to MRHS_BLOCK_EO_MR computes A^-1 per site (FP64 Gauss-Jordan with
 * partial pivoting on each 6x6 block, kept by the op, 576 B per site, +288 B with FP32
 * fields) and synchronises the stream.  Errors: EUNSUPPORTED for an odd block extent,
 * EINVAL for an unknown solver or a clover block without a usable pivot (the op keeps its
 * previous solver). */
#define MRHS_BLOCK_MR 0
#define MRHS_BLOCK_EO_MR 1
int mrhs_set_block_solver(mrhs_op *op, int32_t solver, void *stream);

/* Execution tiles (right-hand sides per site that share one workgroup's field loads) of the
 * SAP and stencil kernels; 0 keeps the current choice.  A tile must divide the op's short
 * length and fit the block (EINVAL otherwise); SAP and stencil tiles above 2 with FP64
 * arithmetic are not built (EUNSUPPORTED: they would not fit the register file).  The
 * stencil at tile 4 on a short length of 4 with FP32 arithmetic takes two groups of 4
 * right-hand sides per workgroup.  Tiles change the execution only, never a result. */
int mrhs_set_tiles(mrhs_op *op, int32_t sap_tile, int32_t dirac_tile);

/* the op's current SAP block solver (MRHS_BLOCK_MR or MRHS_BLOCK_EO_MR) */
int mrhs_op_block_solver(const mrhs_op *op);

/* thread-local text of the last error */
const char *mrhs_last_error(void);

#ifdef __cplusplus
}
#endif

#endif
