// gs.hip -- block Gram-Schmidt of the test vectors per aggregate and spin half (the
// setup of R = Q^dag and P = Q, Sec. 2; the blocks R^h_i of Alg. 3), in FP64 on the
// matrix cores.
//
// One workgroup (4 wavefronts) per (aggregate i, half h).  V^h_i has 6 Va rows (local site,
// spin in the half, colour) and n_tv <= 32 columns, padded to NP = 16 or 32.  CholQR2:
//   G1 = V^dag V = R1^dag R1,  Q1 = V R1^-1,  G2 = Q1^dag Q1 = R2^dag R2,  Q = V (R1^-1 R2^-1),
// the thin QR factor with a real positive triangular diagonal (the Q that Gram-Schmidt
// with re-orthogonalisation produces).  The products V^dag V, V M and Q1^dag Q1 run on
// v_mfma_f64_16x16x4f64 (16x16 output tiles, complex = 4 real products); the Cholesky
// factorisations and triangular inverses of the n_tv x n_tv matrices run on the vector
// units in LDS.
//
// MFMA lane layout of v_mfma_f64_16x16x4f64 (measured on gfx950): lane l supplies A[l%16][l/16]
// and B[l/16][l%16] and holds D[l/16 + 4r][l%16] in accumulator register r.  A Gram matrix
// is a sum over rows, so the accumulator of a 16-row transform (rows l/16 + 4r) is used
// directly as the operand of the next Gram product, with register r as the K step.
#include <climits>

#include "internal.h"

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
constexpr int NTHR = 256;  // 4 wavefronts
constexpr int NW = NTHR / 64;

struct GsArgs {
    KGeo g;
    int Va, n_tv, NT;  // NT = NP / 16 column tiles
    const int32_t *agg_sites;
    const void *V;
    int vdt;
    void *Q;
    int qdt;
    int32_t *status;
};

struct Cplx {
    double re, im;
};

__device__ inline double load_elem(const void *p, int dt, size_t i)
{
    if (dt == MRHS_DTYPE_F64) return ((const double *)p)[i];
    if (dt == MRHS_DTYPE_F32) return (double)((const float *)p)[i];
    return (double)__half2float(((const __half *)p)[i]);
}

__device__ inline void store_elem(void *p, int dt, size_t i, double v)
{
    if (dt == MRHS_DTYPE_F64) ((double *)p)[i] = v;
    else ((float *)p)[i] = (float)v;
}

// native element offset of row n of half h of aggregate i (column part excluded), real part
__device__ inline size_t row_offset(const GsArgs &a, int i, int h, int n)
{
    const KGeo &g = a.g;
    const int ls = n / 6, sp = (n % 6) / 3, c = n % 3;
    const int ns = a.agg_sites[(size_t)i * a.Va + ls];
    const int blk = ns / g.Vb, off = ns - blk * g.Vb;
    const int r = 2 * (3 * (2 * h + sp) + c);
    return (((size_t)blk * 24 + r) * g.Vb + off) * g.S;
}

// native element offset of column k (test vector), row part excluded
__device__ inline size_t col_offset(const GsArgs &a, int k)
{
    const int grp = k / a.g.S, t = k - grp * a.g.S;
    return (size_t)grp * a.g.nblk * 24 * a.g.Vb * a.g.S + t;
}

__device__ inline d4 mfma(double x, double y, d4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, c, 0, 0, 0); }

// G (NP x NP, upper triangle, in place) -> R with G = R^dag R.  Flags a pivot that falls to
// <= 1e-14 of the column's original squared norm, i.e. T_kk <= 1e-7 ||v_k||: the Gram
// matrix squares the condition number, so below that level CholQR cannot resolve the
// column (an exactly dependent column leaves a pivot of order eps ||v_k||^2, of either
// sign).  A flagged pivot is replaced by 1 so that no NaN or Inf is produced.  Padding
// columns (beyond n_tv) get R = 1 on the diagonal and 0 elsewhere.
__device__ void cholesky_inplace(Cplx *G, const double *diag0, int N, int NP, int *bad)
{
    for (int j = 0; j < NP; ++j) {
        __syncthreads();
        const double piv = G[j * NP + j].re;
        const bool pad = j >= N;
        const bool deficient = !pad && !(piv > 1e-14 * diag0[j]);
        const double d = (deficient || pad) ? 1.0 : sqrt(piv);
        if (threadIdx.x == 0 && deficient) *bad = 1;
        __syncthreads();
        for (int l = j + threadIdx.x; l < NP; l += blockDim.x) {
            Cplx v = G[j * NP + l];
            if (l == j) v = {d, 0.0};
            else v = pad ? Cplx{0.0, 0.0} : Cplx{v.re / d, v.im / d};
            G[j * NP + l] = v;
        }
        __syncthreads();
        const int m = NP - j - 1;
        for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
            const int k = j + 1 + e / m, l = j + 1 + e % m;
            if (l < k) continue;
            const Cplx rk = G[j * NP + k], rl = G[j * NP + l];
            // G[k][l] -= conj(R[j][k]) R[j][l]
            G[k * NP + l].re -= rk.re * rl.re + rk.im * rl.im;
            G[k * NP + l].im -= rk.re * rl.im - rk.im * rl.re;
        }
    }
    __syncthreads();
}

// X = R^-1 for upper-triangular R (NP x NP in LDS); one thread per column.
__device__ void tri_inverse(const Cplx *R, Cplx *X, int NP)
{
    for (int e = threadIdx.x; e < NP * NP; e += blockDim.x) X[e] = {0.0, 0.0};
    __syncthreads();
    for (int l = threadIdx.x; l < NP; l += blockDim.x) {
        X[l * NP + l] = {1.0 / R[l * NP + l].re, 0.0};
        for (int k = l - 1; k >= 0; --k) {
            double sr = 0, si = 0;
            for (int j = k + 1; j <= l; ++j) {
                const Cplx r = R[k * NP + j], x = X[j * NP + l];
                sr += r.re * x.re - r.im * x.im;
                si += r.re * x.im + r.im * x.re;
            }
            const double d = R[k * NP + k].re;
            X[k * NP + l] = {-sr / d, -si / d};
        }
    }
    __syncthreads();
}

// C = A B for upper-triangular A, B (NP x NP in LDS)
__device__ void tri_product(const Cplx *A, const Cplx *B, Cplx *C, int NP)
{
    for (int e = threadIdx.x; e < NP * NP; e += blockDim.x) {
        const int k = e / NP, l = e % NP;
        double sr = 0, si = 0;
        for (int j = k; j <= l; ++j) {
            const Cplx x = A[k * NP + j], y = B[j * NP + l];
            sr += x.re * y.re - x.im * y.im;
            si += x.re * y.im + x.im * y.re;
        }
        C[e] = {sr, si};
    }
    __syncthreads();
}

// Gram accumulators of the tile pairs (0,0), (0,1), (1,1), real and imaginary part
struct GramAcc {
    d4 re[3], im[3];
};

__device__ inline int pair_index(int ti, int tj) { return ti == 0 ? tj : 2; }

// G += x^dag y for one K step, x the operands of the NT column tiles (x = y)
template <int NT> __device__ inline void gram_step(const double (&xr)[2], const double (&xi)[2], GramAcc &acc)
{
#pragma unroll
    for (int ti = 0; ti < NT; ++ti)
#pragma unroll
        for (int tj = ti; tj < NT; ++tj) {
            const int p = pair_index(ti, tj);
            acc.re[p] = mfma(xr[ti], xr[tj], acc.re[p]);
            acc.re[p] = mfma(xi[ti], xi[tj], acc.re[p]);
            acc.im[p] = mfma(xr[ti], xi[tj], acc.im[p]);
            acc.im[p] = mfma(-xi[ti], xr[tj], acc.im[p]);
        }
}

// write this wavefront's Gram tiles (upper triangle of tiles) to Gw (NP x NP complex)
template <int NT> __device__ inline void gram_store(const GramAcc &acc, Cplx *Gw, int NP, int lane)
{
#pragma unroll
    for (int ti = 0; ti < NT; ++ti)
#pragma unroll
        for (int tj = ti; tj < NT; ++tj) {
            const int p = pair_index(ti, tj);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = ti * 16 + (lane >> 4) + 4 * r, col = tj * 16 + (lane & 15);
                Gw[row * NP + col] = {acc.re[p][r], acc.im[p][r]};
            }
        }
}

// 16-row block transform: tile tj of (rows b0..b0+15 of V) M for upper-triangular M
// (NP x NP in LDS).  Lane l supplies V[b0 + l%16][4 ks + l/16] and M[4 ks + l/16][16 tj + l%16].
template <int NT>
__device__ inline void transform_block(const GsArgs &a, int i, int h, int b0, int rows, const Cplx *M, int NP, int lane,
                                       d4 (&dr)[2], d4 (&di)[2])
{
    const int N = a.n_tv;
    const int rr = b0 + (lane & 15);
    const size_t cstr = (size_t)a.g.Vb * a.g.S;
    const size_t ro = rr < rows ? row_offset(a, i, h, rr) : 0;
#pragma unroll
    for (int tj = 0; tj < 2; ++tj) dr[tj] = di[tj] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int ks = 0; ks < NT * 4; ++ks) {
        const int k = ks * 4 + (lane >> 4);  // column of V = row of M
        double vr = 0.0, vi = 0.0;
        if (rr < rows && k < N) {
            const size_t idx = ro + col_offset(a, k);
            vr = load_elem(a.V, a.vdt, idx);
            vi = load_elem(a.V, a.vdt, idx + cstr);
        }
#pragma unroll
        for (int tj = 0; tj < NT; ++tj) {
            if (ks * 4 >= (tj + 1) * 16) continue;  // M is upper triangular
            const Cplx m = M[k * NP + tj * 16 + (lane & 15)];
            dr[tj] = mfma(vr, m.re, dr[tj]);
            dr[tj] = mfma(-vi, m.im, dr[tj]);
            di[tj] = mfma(vr, m.im, di[tj]);
            di[tj] = mfma(vi, m.re, di[tj]);
        }
    }
}

template <int NT> __global__ void __launch_bounds__(NTHR) k_block_gs(GsArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int NP = NT * 16;
    const int N = a.n_tv;
    Cplx *Gp = reinterpret_cast<Cplx *>(smem);  // [NW][NP*NP] partial Gram matrices
    Cplx *G = Gp + NW * NP * NP;                // reduced Gram matrix / Cholesky factor / M
    Cplx *X1 = G + NP * NP;                     // R1^-1
    Cplx *X2 = X1 + NP * NP;                    // R2^-1
    double *diag0 = reinterpret_cast<double *>(X2 + NP * NP);
    __shared__ int bad;

    const int i = blockIdx.x >> 1, h = blockIdx.x & 1;
    const int rows = 6 * a.Va;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const size_t cstr = (size_t)a.g.Vb * a.g.S;
    if (threadIdx.x == 0) bad = 0;

    for (int pass = 0; pass < 2; ++pass) {
        GramAcc acc;
#pragma unroll
        for (int p = 0; p < 3; ++p) acc.re[p] = acc.im[p] = d4{0.0, 0.0, 0.0, 0.0};
        if (pass == 0) {
            // G1 = V^dag V: K steps of 4 rows, spread over the wavefronts
            size_t co[2] = {0, 0};
#pragma unroll
            for (int t = 0; t < NT; ++t) co[t] = col_offset(a, t * 16 + (lane & 15));
            const int nsteps = (rows + 3) / 4;
            for (int s = wave; s < nsteps; s += NW) {
                const int n = s * 4 + (lane >> 4);
                double xr[2] = {0.0, 0.0}, xi[2] = {0.0, 0.0};
                if (n < rows) {
                    const size_t ro = row_offset(a, i, h, n);
#pragma unroll
                    for (int t = 0; t < NT; ++t)
                        if (t * 16 + (lane & 15) < N) {
                            xr[t] = load_elem(a.V, a.vdt, ro + co[t]);
                            xi[t] = load_elem(a.V, a.vdt, ro + co[t] + cstr);
                        }
                }
                gram_step<NT>(xr, xi, acc);
            }
        } else {
            // G2 = Q1^dag Q1, Q1 = V R1^-1 formed 16 rows at a time on the matrix cores
            for (int b0 = wave * 16; b0 < rows; b0 += NW * 16) {
                d4 dr[2], di[2];
                transform_block<NT>(a, i, h, b0, rows, X1, NP, lane, dr, di);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const double xr[2] = {dr[0][r], dr[1][r]};
                    const double xi[2] = {di[0][r], di[1][r]};
                    gram_step<NT>(xr, xi, acc);
                }
            }
        }
        gram_store<NT>(acc, Gp + wave * NP * NP, NP, lane);
        __syncthreads();
        // reduce the wavefronts' partial Gram matrices (upper triangle)
        for (int e = threadIdx.x; e < NP * NP; e += blockDim.x) {
            const int k = e / NP, l = e % NP;
            if (l < k) continue;
            Cplx s = Gp[e];
            for (int w = 1; w < NW; ++w) {
                s.re += Gp[w * NP * NP + e].re;
                s.im += Gp[w * NP * NP + e].im;
            }
            G[e] = s;
        }
        __syncthreads();
        for (int k = threadIdx.x; k < NP; k += blockDim.x) diag0[k] = pass == 0 ? G[k * NP + k].re : 1.0;
        cholesky_inplace(G, diag0, N, NP, &bad);
        tri_inverse(G, pass == 0 ? X1 : X2, NP);
    }
    tri_product(X1, X2, G, NP);  // G <- R1^-1 R2^-1
    // Q = V (R1^-1 R2^-1), 16-row blocks spread over the wavefronts
    for (int b0 = wave * 16; b0 < rows; b0 += NW * 16) {
        d4 dr[2], di[2];
        transform_block<NT>(a, i, h, b0, rows, G, NP, lane, dr, di);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int n = b0 + (lane >> 4) + 4 * r;
            if (n >= rows) continue;
            const size_t ro = row_offset(a, i, h, n);
#pragma unroll
            for (int tj = 0; tj < NT; ++tj) {
                const int k = tj * 16 + (lane & 15);
                if (k >= N) continue;
                const size_t idx = ro + col_offset(a, k);
                store_elem(a.Q, a.qdt, idx, dr[tj][r]);
                store_elem(a.Q, a.qdt, idx + cstr, di[tj][r]);
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0 && bad && a.status) atomicMin(a.status, 1 + (int)blockIdx.x);
}

__global__ void k_status_init(int32_t *s) { *s = INT_MAX; }
__global__ void k_status_final(int32_t *s)
{
    if (*s == INT_MAX) *s = 0;
}

size_t gs_lds(int NP) { return sizeof(Cplx) * (size_t)(NW + 3) * NP * NP + sizeof(double) * NP; }

template <int NT> int launch_nt(const GsArgs &a, int n_agg, size_t max_lds, hipStream_t st)
{
    const size_t lds = gs_lds(NT * 16);
    if (lds > max_lds) return set_error(MRHS_EUNSUPPORTED, "Gram-Schmidt LDS exceeds the workgroup limit");
    static size_t done = 0;
    if (lds > 65536 && lds > done) {
        if (int rc = hip_check(hipFuncSetAttribute((const void *)k_block_gs<NT>,
                                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds),
                               "hipFuncSetAttribute(gs LDS)"))
            return rc;
        done = lds;
    }
    hipLaunchKernelGGL(k_block_gs<NT>, dim3(2 * n_agg), dim3(NTHR), lds, st, a);
    return hip_check(hipGetLastError(), "k_block_gs launch");
}

}  // namespace

size_t ws_bytes_gs(const mrhs_op *, int) { return 0; }

int launch_gs(const mrhs_op *op, const void *V, int vdt, void *Q, int qdt, int n_tv, int32_t *status, void *,
              hipStream_t st)
{
    if (n_tv > 32) return set_error(MRHS_EUNSUPPORTED, "Gram-Schmidt handles at most 32 test vectors");
    GsArgs a{};
    a.g = op->k;
    a.Va = op->Va;
    a.n_tv = n_tv;
    a.NT = n_tv > 16 ? 2 : 1;
    a.agg_sites = op->agg_sites;
    a.V = V;
    a.vdt = vdt;
    a.Q = Q;
    a.qdt = qdt;
    a.status = status;
    if (!a.agg_sites || !a.V || !a.Q) return set_error(MRHS_EINVAL, "block_orthonormalize: missing buffer");
    if (status) {
        hipLaunchKernelGGL(k_status_init, dim3(1), dim3(1), 0, st, status);
        if (int rc = hip_check(hipGetLastError(), "k_status_init launch")) return rc;
    }
    int rc = a.NT == 2 ? launch_nt<2>(a, op->n_agg, op->max_lds, st) : launch_nt<1>(a, op->n_agg, op->max_lds, st);
    if (rc) return rc;
    if (status) {
        hipLaunchKernelGGL(k_status_final, dim3(1), dim3(1), 0, st, status);
        if (int rc2 = hip_check(hipGetLastError(), "k_status_final launch")) return rc2;
    }
    return MRHS_OK;
}
