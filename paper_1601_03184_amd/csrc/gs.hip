// gs.hip -- block Gram-Schmidt of the test vectors per aggregate and spin half (the
// setup of R = Q^dag and P = Q, Sec. 2; the blocks R^h_i of Alg. 3), in FP64.
//
// One workgroup per (aggregate i, half h).  V^h_i has 6 Va rows (local site, spin in the
// half, colour) and n_tv columns.  CholQR2: G = V^dag V, G = R1^dag R1 (Cholesky),
// Q1 = V R1^-1; G2 = Q1^dag Q1 = R2^dag R2; Q = V (R1^-1 R2^-1).  The result is the thin
// QR factor with a real positive triangular diagonal, the same Q that Gram-Schmidt with
// re-orthogonalisation produces.  Rows stream through LDS in chunks of CH rows; the
// n_tv x n_tv matrices stay in LDS.  The three passes read V three times.
#include <climits>

#include "internal.h"

namespace {

constexpr int CH = 16;     // rows per chunk
constexpr int NTHR = 256;

struct GsArgs {
    KGeo g;
    int Va, n_tv;
    const int32_t *agg_sites;
    const void *V;
    int vdt;
    void *Q;
    int qdt;
    int32_t *status;
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

// native element index of (row n of half h of aggregate i, column k), real part;
// the imaginary part is one component stride further
__device__ inline size_t row_index(const GsArgs &a, int i, int h, int n, int k)
{
    const KGeo &g = a.g;
    const int ls = n / 6, sp = (n % 6) / 3, c = n % 3;
    const int ns = a.agg_sites[(size_t)i * a.Va + ls];
    const int blk = ns / g.Vb, off = ns - blk * g.Vb;
    const int r = 2 * (3 * (2 * h + sp) + c);
    const int grp = k / g.S, t = k - grp * g.S;
    return ((((size_t)grp * g.nblk + blk) * 24 + r) * g.Vb + off) * g.S + t;
}

struct Cplx {
    double re, im;
};

// G (upper triangle, in place) -> R with G = R^dag R.  Flags a pivot that falls to
// <= 1e-14 of the column's original squared norm, i.e. T_kk <= 1e-7 ||v_k||: the Gram
// matrix squares the condition number, so below that level CholQR cannot resolve the
// column (an exactly dependent column leaves a pivot of order eps ||v_k||^2, of either
// sign).  A flagged pivot is replaced by 1 so that no NaN or Inf is produced.
__device__ void cholesky_inplace(Cplx *G, const double *diag0, int N, int *bad)
{
    for (int j = 0; j < N; ++j) {
        __syncthreads();
        const double piv = G[j * N + j].re;
        const bool deficient = !(piv > 1e-14 * diag0[j]);
        const double d = deficient ? 1.0 : sqrt(piv);
        if (threadIdx.x == 0 && deficient) *bad = 1;
        __syncthreads();
        for (int l = j + threadIdx.x; l < N; l += blockDim.x) {
            Cplx v = G[j * N + l];
            if (l == j) v = {d, 0.0};
            else v = {v.re / d, v.im / d};
            G[j * N + l] = v;
        }
        __syncthreads();
        const int m = N - j - 1;
        for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
            const int k = j + 1 + e / m, l = j + 1 + e % m;
            if (l < k) continue;
            const Cplx rk = G[j * N + k], rl = G[j * N + l];
            // G[k][l] -= conj(R[j][k]) R[j][l]
            G[k * N + l].re -= rk.re * rl.re + rk.im * rl.im;
            G[k * N + l].im -= rk.re * rl.im - rk.im * rl.re;
        }
    }
    __syncthreads();
}

// X = R^-1 for upper-triangular R (both N x N in LDS); one thread per column.
__device__ void tri_inverse(const Cplx *R, Cplx *X, int N)
{
    for (int e = threadIdx.x; e < N * N; e += blockDim.x) X[e] = {0.0, 0.0};
    __syncthreads();
    for (int l = threadIdx.x; l < N; l += blockDim.x) {
        const Cplx rll = R[l * N + l];
        X[l * N + l] = {1.0 / rll.re, 0.0};
        for (int k = l - 1; k >= 0; --k) {
            double sr = 0, si = 0;
            for (int j = k + 1; j <= l; ++j) {
                const Cplx r = R[k * N + j], x = X[j * N + l];
                sr += r.re * x.re - r.im * x.im;
                si += r.re * x.im + r.im * x.re;
            }
            const double d = R[k * N + k].re;
            X[k * N + l] = {-sr / d, -si / d};
        }
    }
    __syncthreads();
}

// C = A B for upper-triangular A, B (N x N in LDS)
__device__ void tri_product(const Cplx *A, const Cplx *B, Cplx *C, int N)
{
    for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
        const int k = e / N, l = e % N;
        double sr = 0, si = 0;
        for (int j = k; j <= l; ++j) {
            const Cplx x = A[k * N + j], y = B[j * N + l];
            sr += x.re * y.re - x.im * y.im;
            si += x.re * y.im + x.im * y.re;
        }
        C[e] = {sr, si};
    }
    __syncthreads();
}

// Load rows [r0, r0+CH) of V^h_i into raw[CH][N] (zero beyond the last row)
__device__ void load_chunk(const GsArgs &a, int i, int h, int r0, int rows, Cplx *raw)
{
    const int N = a.n_tv;
    const size_t cstr = (size_t)a.g.Vb * a.g.S;
    for (int e = threadIdx.x; e < CH * N; e += blockDim.x) {
        const int rr = e / N, k = e % N, n = r0 + rr;
        Cplx v = {0.0, 0.0};
        if (n < rows) {
            const size_t idx = row_index(a, i, h, n, k);
            v = {load_elem(a.V, a.vdt, idx), load_elem(a.V, a.vdt, idx + cstr)};
        }
        raw[e] = v;
    }
}

// out[CH][N] = raw[CH][N] M, M upper triangular
__device__ void transform_chunk(const Cplx *raw, const Cplx *M, Cplx *out, int N)
{
    for (int e = threadIdx.x; e < CH * N; e += blockDim.x) {
        const int rr = e / N, l = e % N;
        double sr = 0, si = 0;
        for (int j = 0; j <= l; ++j) {
            const Cplx v = raw[rr * N + j], m = M[j * N + l];
            sr += v.re * m.re - v.im * m.im;
            si += v.re * m.im + v.im * m.re;
        }
        out[e] = {sr, si};
    }
}

// G[k][l] += sum_rows conj(C[r][k]) C[r][l] for k <= l
__device__ void gram_accumulate(const Cplx *C, Cplx *G, int N)
{
    for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
        const int k = e / N, l = e % N;
        if (l < k) continue;
        double sr = 0, si = 0;
#pragma unroll 4
        for (int rr = 0; rr < CH; ++rr) {
            const Cplx x = C[rr * N + k], y = C[rr * N + l];
            sr += x.re * y.re + x.im * y.im;
            si += x.re * y.im - x.im * y.re;
        }
        G[e].re += sr;
        G[e].im += si;
    }
}

__global__ void __launch_bounds__(NTHR) k_block_gs(GsArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int N = a.n_tv;
    Cplx *G = reinterpret_cast<Cplx *>(smem);  // N*N
    Cplx *X1 = G + N * N;                      // R1^-1, later R1^-1 R2^-1
    Cplx *X2 = X1 + N * N;                     // R2^-1
    Cplx *raw = X2 + N * N;                    // CH*N
    Cplx *tr = raw + CH * N;                   // CH*N
    double *diag0 = reinterpret_cast<double *>(tr + CH * N);  // N
    __shared__ int bad;

    const int i = blockIdx.x >> 1, h = blockIdx.x & 1;
    const int rows = 6 * a.Va;
    const size_t cstr = (size_t)a.g.Vb * a.g.S;
    if (threadIdx.x == 0) bad = 0;

    for (int pass = 0; pass < 2; ++pass) {
        for (int e = threadIdx.x; e < N * N; e += blockDim.x) G[e] = {0.0, 0.0};
        for (int r0 = 0; r0 < rows; r0 += CH) {
            __syncthreads();
            load_chunk(a, i, h, r0, rows, raw);
            __syncthreads();
            if (pass == 0) {
                gram_accumulate(raw, G, N);
            } else {
                transform_chunk(raw, X1, tr, N);
                __syncthreads();
                gram_accumulate(tr, G, N);
            }
        }
        __syncthreads();
        if (pass == 0)
            for (int k = threadIdx.x; k < N; k += blockDim.x) diag0[k] = G[k * N + k].re;
        else
            for (int k = threadIdx.x; k < N; k += blockDim.x) diag0[k] = 1.0;
        cholesky_inplace(G, diag0, N, &bad);
        if (pass == 0) {
            tri_inverse(G, X1, N);
        } else {
            tri_inverse(G, X2, N);
            tri_product(X1, X2, G, N);  // G <- R1^-1 R2^-1
        }
    }
    // Q = V (R1^-1 R2^-1)
    for (int r0 = 0; r0 < rows; r0 += CH) {
        __syncthreads();
        load_chunk(a, i, h, r0, rows, raw);
        __syncthreads();
        transform_chunk(raw, G, tr, N);
        __syncthreads();
        for (int e = threadIdx.x; e < CH * N; e += blockDim.x) {
            const int rr = e / N, k = e % N, n = r0 + rr;
            if (n >= rows) continue;
            const size_t idx = row_index(a, i, h, n, k);
            store_elem(a.Q, a.qdt, idx, tr[e].re);
            store_elem(a.Q, a.qdt, idx + cstr, tr[e].im);
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

size_t gs_lds(int N) { return sizeof(Cplx) * (3 * (size_t)N * N + 2 * (size_t)CH * N) + sizeof(double) * N; }

}  // namespace

size_t ws_bytes_gs(const mrhs_op *, int) { return 0; }

int launch_gs(const mrhs_op *op, const void *V, int vdt, void *Q, int qdt, int n_tv, int32_t *status, void *,
              hipStream_t st)
{
    const size_t lds = gs_lds(n_tv);
    if (lds > op->max_lds) return set_error(MRHS_EUNSUPPORTED, "too many test vectors for the Gram-Schmidt LDS");
    static size_t done = 0;
    if (lds > 65536 && lds > done) {
        if (int rc = hip_check(hipFuncSetAttribute((const void *)k_block_gs, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                   (int)lds), "hipFuncSetAttribute(gs LDS)"))
            return rc;
        done = lds;
    }
    GsArgs a{};
    a.g = op->k;
    a.Va = op->Va;
    a.n_tv = n_tv;
    a.agg_sites = op->agg_sites;
    a.V = V;
    a.vdt = vdt;
    a.Q = Q;
    a.qdt = qdt;
    a.status = status;
    if (status) {
        hipLaunchKernelGGL(k_status_init, dim3(1), dim3(1), 0, st, status);
        if (int rc = hip_check(hipGetLastError(), "k_status_init launch")) return rc;
    }
    hipLaunchKernelGGL(k_block_gs, dim3(2 * op->n_agg), dim3(NTHR), lds, st, a);
    if (int rc = hip_check(hipGetLastError(), "k_block_gs launch")) return rc;
    if (status) {
        hipLaunchKernelGGL(k_status_final, dim3(1), dim3(1), 0, st, status);
        if (int rc = hip_check(hipGetLastError(), "k_status_final launch")) return rc;
    }
    return MRHS_OK;
}
