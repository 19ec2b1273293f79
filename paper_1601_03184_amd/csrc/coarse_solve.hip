// coarse_solve.hip -- the low-accuracy coarse solve of the refinement phase (Alg. 1, 2:
// u_c ~ D_c^-1 v_c) on all right-hand sides at once: GMRES from a zero start, Arnoldi
// with classical Gram-Schmidt applied twice, complex Givens rotations.  Every right-hand
// side has its own Krylov basis; one launch of each step serves all of them, and the
// operator is applied to all of them in one coarse_apply (the mat-mat form of Sec. 6).
//
// Vectors are FP32 (coarse layout of transfer.hip); inner products, norms, the Hessenberg
// matrix, the rotations and the small triangular solve are FP64.  The half-precision coarse
// grid keeps the Krylov basis in binary16 (each basis vector rounded once when it is formed;
// a FP32 copy of the newest one feeds the operator) and D_c in binary16.  A right-hand side whose
// residual estimate has reached tol * ||b|| stops taking part (its later basis vectors are
// zero and its Hessenberg matrix is frozen), so the host issues a fixed sequence of
// launches without reading anything back; once no right-hand side takes part, the
// remaining launches return at once.
#include <algorithm>
#include <climits>
#include <type_traits>

#include "launch.h"

namespace {

struct Z {
    double re, im;
};
__device__ inline Z zmul(Z a, Z b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ inline Z zconjmul(Z a, Z b) { return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re}; }  // conj(a) b

constexpr int GTHR = 256;
constexpr int DTHR = 512;
constexpr int DROWS = DTHR / 32;  // element rows per block pass of the inner products (32 right-hand-side lanes)

struct GmArgs {
    int n, ldc, m;
    long dim;     // complex entries per right-hand side (coarse sites x 2 n_tv)
    long cvlen;   // floats of one coarse vector
    double tol;
    void *V;      // (m + 1) coarse vectors, FP32 or binary16 (the basis type of gmres_run)
    float *v32;   // binary16 basis: the newest basis vector as FP32 (input of the operator)
    float *w;
    Z *part;      // [vectors][G][ldc] partial inner products, G x vectors <= GPART
    Z *hcur;      // [ldc][m + 1]: the current inner products, then y
    Z *H;         // [ldc][m + 1][m]
    Z *g;         // [ldc][m + 1]
    Z *sn;        // [ldc][m]
    double *cs;   // [ldc][m]
    double *beta, *est, *scale;  // [ldc]
    int *J, *active;             // [ldc]
};

// whether any right-hand side still iterates: the kernels of an Arnoldi step return at once
// when none does, so that the fixed launch sequence costs only the launches after the last
// right-hand side has stopped
__device__ inline bool gm_running(const GmArgs &a)
{
    // one flag per lane (at most 32 right-hand sides), combined over the wavefront; called
    // first thing, with every lane of the wavefront active
    const int l = threadIdx.x & 63;
    const int f = l < a.n ? a.active[l] : 0;
    return __ballot(f != 0) != 0;
}

// element of thread t of an elementwise launch: entry e = t / ldc, right-hand side k; its real
// part at cre(e, k) (a coarse vector has fewer than 2^31 floats, checked on the host)
__device__ inline bool gm_elem(const GmArgs &a, uint32_t &o, int &k)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x, ldc = (uint32_t)a.ldc;
    if (t >= (uint32_t)a.dim * ldc) return false;
    const uint32_t e = t / ldc;
    k = (int)(t - e * ldc);
    o = 2 * e * ldc + (uint32_t)k;
    return true;
}

constexpr int GU = 8;  // basis vectors whose loads an elementwise kernel issues together

// element (e, k) of a coarse vector: entry e = site * 2 n_tv + dof, right-hand side k
__device__ inline long cre(const GmArgs &a, long e, int k) { return (2 * e) * a.ldc + k; }

constexpr int GPART = 512;  // partial-sum blocks per inner-product launch (all vectors together)

// start: beta = ||b|| (from ||b||^2), g = (beta, 0, ...), H = 0, scale = 1 / beta
__device__ void gm_start(const GmArgs &a, int k, double b2)
{
    const double b = sqrt(b2);
    a.beta[k] = b;
    a.est[k] = b;
    a.J[k] = 0;
    a.active[k] = k < a.n && b > 0.0 && b > a.tol * b;
    a.scale[k] = b > 0.0 ? 1.0 / b : 0.0;
    for (int i = 0; i <= a.m; ++i) a.g[(long)k * (a.m + 1) + i] = {i == 0 ? b : 0.0, 0.0};
    for (long e = 0; e < (long)(a.m + 1) * a.m; ++e) a.H[(long)k * (a.m + 1) * a.m + e] = {0.0, 0.0};
}

// iteration j: ||w|| -> H[j+1][j], the earlier rotations on column j, a new rotation, g,
// the residual estimate and whether the right-hand side continues; scale = 1 / ||w||
__device__ void gm_givens(const GmArgs &a, int k, int j, double nw2)
{
    if (!a.active[k]) {
        a.scale[k] = 0.0;
        return;
    }
    const int m = a.m;
    Z *H = a.H + (long)k * (m + 1) * m;
    Z *g = a.g + (long)k * (m + 1);
    double *cs = a.cs + (long)k * m;
    Z *sn = a.sn + (long)k * m;
    const double nw = sqrt(nw2);
    for (int i = 0; i < j; ++i) {
        const Z x0 = H[i * m + j], x1 = H[(i + 1) * m + j];
        const Z s1 = zmul(sn[i], x1), s0 = zmul({sn[i].re, -sn[i].im}, x0);
        H[i * m + j] = {cs[i] * x0.re + s1.re, cs[i] * x0.im + s1.im};
        H[(i + 1) * m + j] = {-s0.re + cs[i] * x1.re, -s0.im + cs[i] * x1.im};
    }
    const Z hj = H[j * m + j];
    const double ah = sqrt(hj.re * hj.re + hj.im * hj.im), rho = sqrt(ah * ah + nw * nw);
    if (ah == 0.0) {
        cs[j] = 0.0;
        sn[j] = {1.0, 0.0};
    } else {
        cs[j] = ah / rho;
        sn[j] = {hj.re / ah * nw / rho, hj.im / ah * nw / rho};
    }
    H[j * m + j] = {cs[j] * hj.re + sn[j].re * nw, cs[j] * hj.im + sn[j].im * nw};
    H[(j + 1) * m + j] = {0.0, 0.0};
    const Z gj = g[j];
    const Z t = zmul({sn[j].re, -sn[j].im}, gj);
    g[j + 1] = {-t.re, -t.im};
    g[j] = {cs[j] * gj.re, cs[j] * gj.im};
    const double est = sqrt(g[j + 1].re * g[j + 1].re + g[j + 1].im * g[j + 1].im);
    a.est[k] = est;
    a.J[k] = j + 1;
    a.active[k] = nw > 0.0 && est > a.tol * a.beta[k];
    a.scale[k] = nw > 0.0 ? 1.0 / nw : 0.0;
}

// part[i][blk][k] = sum over this block's chunk of entries of conj(X_i) y, for the vectors
// X_i = X + i * xstride (i = blockIdx.y) and every right-hand side k
template <typename TX>
__global__ void __launch_bounds__(DTHR) k_gm_dots(GmArgs a, const TX *X, long xstride, const float *y, int gated)
{
    __shared__ Z red[DROWS][32];
    if (gated && !gm_running(a)) return;
    const int G = gridDim.x, i = blockIdx.y;
    const int k = threadIdx.x & 31, row = threadIdx.x >> 5;
    const long chunk = (a.dim + G - 1) / G, e0 = blockIdx.x * chunk, e1 = e0 + chunk < a.dim ? e0 + chunk : a.dim;
    const TX *xi = X + i * xstride;
    Z s = {0.0, 0.0};
    if (k < a.ldc)
        for (long e = e0 + row; e < e1; e += DROWS) {
            const long o = cre(a, e, k);
            const Z xv = {load_as<double>(xi + o), load_as<double>(xi + o + a.ldc)}, yv = {y[o], y[o + a.ldc]};
            const Z p = zconjmul(xv, yv);
            s.re += p.re;
            s.im += p.im;
        }
    red[row][k] = s;
    __syncthreads();
    if (row == 0 && k < a.ldc) {
        Z t = red[0][k];
        for (int r = 1; r < DROWS; ++r) {
            t.re += red[r][k].re;
            t.im += red[r][k].im;
        }
        a.part[((long)i * G + blockIdx.x) * a.ldc + k] = t;
    }
}

enum GmStep { GM_PROJECT = 1, GM_NORM = 2, GM_START = 3 };

constexpr int FR = 16;  // threads per inner product in k_gm_finish

// h_i[k] = the G partial sums of k_gm_dots added up (thread r of an output's FR threads takes
// blocks r, r + FR, ... in order; the FR sums are combined by a fixed shuffle tree), then the
// step that needs them:
//   GM_PROJECT: hcur[k][i] = h_i, and H[k][i][col] += h_i for the right-hand sides still active
//   GM_NORM   : (X = y = w) the Givens step of iteration col with ||w||^2
//   GM_START  : (X = y = b) the start of the iteration with ||b||^2
__global__ void __launch_bounds__(256) k_gm_finish(GmArgs a, int G, int nvec, int col, int step)
{
    if (step != GM_START && !gm_running(a)) return;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int o = t / FR, r = t - o * FR;
    const bool ok = o < nvec * a.ldc;
    const int i = ok ? o / a.ldc : 0, k = ok ? o - i * a.ldc : 0;
    const Z *pp = a.part + (long)i * G * a.ldc + k;
    Z s = {0.0, 0.0};
    if (ok) {
#pragma unroll 8
        for (int b = r; b < G; b += FR) {
            const Z p = pp[(long)b * a.ldc];
            s.re += p.re;
            s.im += p.im;
        }
    }
    for (int off = 1; off < FR; off *= 2) {
        s.re += __shfl_down(s.re, off, FR);
        s.im += __shfl_down(s.im, off, FR);
    }
    if (!ok || r != 0) return;
    a.hcur[(long)k * (a.m + 1) + i] = s;
    if (step == GM_PROJECT) {
        if (a.active[k]) {
            Z &h = a.H[((long)k * (a.m + 1) + i) * a.m + col];
            h.re += s.re;
            h.im += s.im;
        }
    } else if (step == GM_NORM) {
        gm_givens(a, k, col, s.re);
    } else {
        gm_start(a, k, s.re);
    }
}

// blocks per vector of an inner-product launch over nvec vectors
int gm_blocks(const GmArgs &a, int nvec)
{
    const long want = (a.dim + 4 * DROWS - 1) / (4 * DROWS);  // at least 4 entries per thread
    return (int)std::max<long>(1, std::min<long>(want, GPART / nvec));
}

// w -= sum_i hcur[k][i] V_i   (i < nvec)
template <typename TV> __global__ void __launch_bounds__(GTHR) k_gm_axpy(GmArgs a, int nvec)
{
    if (!gm_running(a)) return;
    uint32_t o;
    int k;
    if (!gm_elem(a, o, k)) return;
    double wr = a.w[o], wi = a.w[o + a.ldc];
    for (int i0 = 0; i0 < nvec; i0 += GU) {
        Z h[GU], v[GU];
#pragma unroll
        for (int u = 0; u < GU; ++u) {
            h[u] = v[u] = {0.0, 0.0};
            if (i0 + u < nvec) {
                const TV *vi = (const TV *)a.V + (long)(i0 + u) * a.cvlen;
                h[u] = a.hcur[(long)k * (a.m + 1) + i0 + u];
                v[u] = {load_as<double>(vi + o), load_as<double>(vi + o + a.ldc)};
            }
        }
#pragma unroll
        for (int u = 0; u < GU; ++u) {
            const Z p = zmul(h[u], v[u]);
            wr -= p.re;
            wi -= p.im;
        }
    }
    a.w[o] = (float)wr;
    a.w[o + a.ldc] = (float)wi;
}

// V_dst = src * scale[k] (rounded to the basis type); dst32 (nullable): the same values as FP32
template <typename TV>
__global__ void __launch_bounds__(GTHR) k_gm_scale(GmArgs a, const float *src, TV *dst, float *dst32, int gated)
{
    if (gated && !gm_running(a)) return;
    uint32_t o;
    int k;
    if (!gm_elem(a, o, k)) return;
    const double s = a.scale[k];
    const TV re = store_as<TV>((float)(src[o] * s)), im = store_as<TV>((float)(src[o + a.ldc] * s));
    dst[o] = re;
    dst[o + a.ldc] = im;
    if (dst32) {
        dst32[o] = load_as<float>(&re);
        dst32[o + a.ldc] = load_as<float>(&im);
    }
}

// y = H^-1 g (back substitution over the J[k] iterations taken), into hcur
__global__ void k_gm_solve(GmArgs a, double *res_out, int32_t *iters_out)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.ldc) return;
    const int m = a.m, J = a.J[k];
    const Z *H = a.H + (long)k * (m + 1) * m;
    const Z *g = a.g + (long)k * (m + 1);
    Z *y = a.hcur + (long)k * (m + 1);
    for (int i = 0; i <= m; ++i) y[i] = {0.0, 0.0};
    for (int i = J - 1; i >= 0; --i) {
        Z s = g[i];
        for (int l = i + 1; l < J; ++l) {
            const Z p = zmul(H[i * m + l], y[l]);
            s.re -= p.re;
            s.im -= p.im;
        }
        const Z d = H[i * m + i];
        const double dd = d.re * d.re + d.im * d.im;
        y[i] = {(s.re * d.re + s.im * d.im) / dd, (s.im * d.re - s.re * d.im) / dd};
    }
    if (k < a.n) {
        if (res_out) res_out[k] = a.beta[k] > 0.0 ? a.est[k] / a.beta[k] : 0.0;
        if (iters_out) iters_out[k] = J;
    }
}

// u = sum_i y_i V_i
template <typename TV> __global__ void __launch_bounds__(GTHR) k_gm_combine(GmArgs a, float *u)
{
    uint32_t o;
    int k;
    if (!gm_elem(a, o, k)) return;
    double ur = 0.0, ui = 0.0;
    const int J = a.J[k];
    for (int i0 = 0; i0 < J; i0 += GU) {
        Z y[GU], v[GU];
#pragma unroll
        for (int q = 0; q < GU; ++q) {
            y[q] = v[q] = {0.0, 0.0};
            if (i0 + q < J) {
                const TV *vi = (const TV *)a.V + (long)(i0 + q) * a.cvlen;
                y[q] = a.hcur[(long)k * (a.m + 1) + i0 + q];
                v[q] = {load_as<double>(vi + o), load_as<double>(vi + o + a.ldc)};
            }
        }
#pragma unroll
        for (int q = 0; q < GU; ++q) {
            const Z p = zmul(y[q], v[q]);
            ur += p.re;
            ui += p.im;
        }
    }
    u[o] = k < a.n ? (float)ur : 0.f;
    u[o + a.ldc] = k < a.n ? (float)ui : 0.f;
}

size_t align256(size_t n) { return (n + 255) / 256 * 256; }

// workspace layout for (op, n_tv, n, m); fills the pointers when base != nullptr.  vsz: bytes
// of a basis element (4, or 2 for a binary16 basis, which also takes a FP32 vector v32)
size_t gm_layout(const mrhs_op *op, int n_tv, int n, int m, char *base, GmArgs *a, int vsz = 4)
{
    const int ldc = (n + 3) / 4 * 4;
    const long dim = (long)op->n_agg * 2 * n_tv;
    const long cvlen = dim * 2 * ldc;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *p = base ? base + off : nullptr;
        off += align256(bytes);
        return p;
    };
    char *V = take((size_t)vsz * cvlen * (m + 1));
    char *v32 = vsz == 4 ? nullptr : take(sizeof(float) * cvlen);
    char *w = take(sizeof(float) * cvlen);
    char *part = take(sizeof(Z) * (size_t)GPART * ldc);
    char *hcur = take(sizeof(Z) * (size_t)ldc * (m + 1));
    char *H = take(sizeof(Z) * (size_t)ldc * (m + 1) * m);
    char *g = take(sizeof(Z) * (size_t)ldc * (m + 1));
    char *sn = take(sizeof(Z) * (size_t)ldc * m);
    char *cs = take(sizeof(double) * (size_t)ldc * m);
    char *beta = take(sizeof(double) * ldc);
    char *est = take(sizeof(double) * ldc);
    char *scale = take(sizeof(double) * ldc);
    char *J = take(sizeof(int) * ldc);
    char *act = take(sizeof(int) * ldc);
    if (a) {
        a->n = n;
        a->ldc = ldc;
        a->m = m;
        a->dim = dim;
        a->cvlen = cvlen;
        a->V = V;
        a->v32 = (float *)v32;
        a->w = (float *)w;
        a->part = (Z *)part;
        a->hcur = (Z *)hcur;
        a->H = (Z *)H;
        a->g = (Z *)g;
        a->sn = (Z *)sn;
        a->cs = (double *)cs;
        a->beta = (double *)beta;
        a->est = (double *)est;
        a->scale = (double *)scale;
        a->J = (int *)J;
        a->active = (int *)act;
    }
    return off;
}

// Inverse of every coarse site's self block (2N x 2N complex): Gauss-Jordan elimination with
// partial (row) pivoting, in place in LDS in FP64, one workgroup per coarse site; the row
// exchanges are undone as column exchanges at the end.  A block without a non-zero pivot gives
// zeros and status = 1 + the lowest such site (status preset to INT_MAX, mapped to 0 after).
__global__ void __launch_bounds__(256) k_coarse_self_inverse(const float *__restrict__ Dc, float *__restrict__ Dinv,
                                                             int N2, int *status)
{
    extern __shared__ __align__(16) unsigned char smem[];
    double2 *M = reinterpret_cast<double2 *>(smem);  // [N2][N2]
    double2 *f = M + N2 * N2;                          // column factors [N2]
    int *perm = reinterpret_cast<int *>(f + N2);       // [N2]
    __shared__ int piv, singular;
    const int i = blockIdx.x, tid = threadIdx.x, bd = blockDim.x, n2 = N2 * N2;
    const float *blk = Dc + (size_t)i * 9 * n2 * 2;  // block 0: self
    for (int e = tid; e < n2; e += bd) M[e] = make_double2(blk[2 * e], blk[2 * e + 1]);
    if (tid == 0) singular = 0;
    __syncthreads();
    for (int k = 0; k < N2; ++k) {
        if (tid == 0) {
            int p = k;
            double best = M[k * N2 + k].x * M[k * N2 + k].x + M[k * N2 + k].y * M[k * N2 + k].y;
            for (int r = k + 1; r < N2; ++r) {
                const double2 v = M[r * N2 + k];
                const double mg = v.x * v.x + v.y * v.y;
                if (mg > best) {
                    best = mg;
                    p = r;
                }
            }
            perm[k] = p;
            piv = p;
            if (!(best > 0.0) || !isfinite(best)) singular = 1;
        }
        __syncthreads();
        if (singular) break;  // shared: every thread leaves together
        const int p = piv;
        if (p != k)
            for (int j = tid; j < N2; j += bd) {
                const double2 t = M[k * N2 + j];
                M[k * N2 + j] = M[p * N2 + j];
                M[p * N2 + j] = t;
            }
        __syncthreads();
        const double2 pv = M[k * N2 + k];
        const double den = pv.x * pv.x + pv.y * pv.y, ir = pv.x / den, ii = -pv.y / den;  // 1 / pivot
        for (int r = tid; r < N2; r += bd) f[r] = M[r * N2 + k];
        __syncthreads();
        // row k: (row k with a_kk = 1) / pivot
        for (int j = tid; j < N2; j += bd) {
            const double2 x = j == k ? make_double2(1.0, 0.0) : M[k * N2 + j];
            M[k * N2 + j] = make_double2(x.x * ir - x.y * ii, x.x * ii + x.y * ir);
        }
        __syncthreads();
        // other rows: (row r with a_rk = 0) - f_r row k
        for (int e = tid; e < n2; e += bd) {
            const int r = e / N2, j = e - r * N2;
            if (r == k) continue;
            double2 x = j == k ? make_double2(0.0, 0.0) : M[e];
            const double2 fr = f[r], y = M[k * N2 + j];
            x.x -= fr.x * y.x - fr.y * y.y;
            x.y -= fr.x * y.y + fr.y * y.x;
            M[e] = x;
        }
        __syncthreads();
    }
    float *out = Dinv + (size_t)i * n2 * 2;
    if (singular) {
        for (int e = tid; e < 2 * n2; e += bd) out[e] = 0.f;
        if (tid == 0 && status) atomicMin(status, i + 1);
        return;
    }
    for (int k = N2 - 1; k >= 0; --k) {
        const int p = perm[k];
        if (p != k)
            for (int r = tid; r < N2; r += bd) {
                const double2 t = M[r * N2 + k];
                M[r * N2 + k] = M[r * N2 + p];
                M[r * N2 + p] = t;
            }
        __syncthreads();
    }
    for (int e = tid; e < n2; e += bd) {
        out[2 * e] = (float)M[e].x;
        out[2 * e + 1] = (float)M[e].y;
    }
}

__global__ void k_inv_status_init(int *s) { *s = INT_MAX; }
__global__ void k_inv_status_final(int *s)
{
    if (*s == INT_MAX) *s = 0;
}

// GMRES on all right-hand sides for the operator apply(in, out) (coarse vectors), from b into u;
// TV: the basis type (float, or __half for the half-precision coarse grid)
template <typename TV, typename Apply>
int gmres_run(GmArgs &a, const float *b, float *u, int m, double *res_out, int32_t *iters_out, Apply apply,
              hipStream_t st)
{
    const long nel = a.dim * a.ldc;
    if (a.cvlen >= (1L << 31)) return set_error(MRHS_EUNSUPPORTED, "coarse solve: a coarse vector above 2^31 floats");
    const int eb = (int)((nel + GTHR - 1) / GTHR);
    const int kb = (a.ldc + 63) / 64;
    TV *V = (TV *)a.V;
#define GM_CHECK(what) \
    if (int rc = hip_check(hipGetLastError(), what)) return rc
    auto dots = [&](auto X, long xstride, int nvec, const float *y, int col, int step) {
        using TX = std::remove_const_t<std::remove_pointer_t<decltype(X)>>;
        const int G = gm_blocks(a, nvec);
        hipLaunchKernelGGL(k_gm_dots<TX>, dim3(G, nvec), dim3(DTHR), 0, st, a, X, xstride, y, step != GM_START ? 1 : 0);
        if (int rc = hip_check(hipGetLastError(), "k_gm_dots launch")) return rc;
        hipLaunchKernelGGL(k_gm_finish, dim3((nvec * a.ldc * FR + 255) / 256), dim3(256), 0, st, a, G, nvec, col, step);
        return hip_check(hipGetLastError(), "k_gm_finish launch");
    };
    // beta, V_0
    if (int rc = dots(b, 0L, 1, b, 0, GM_START)) return rc;
    hipLaunchKernelGGL(k_gm_scale<TV>, dim3(eb), dim3(GTHR), 0, st, a, b, V, a.v32, 0);
    GM_CHECK("k_gm_scale launch");
    // every launch of an iteration (the operator's included) returns at once when no
    // right-hand side iterates any more
    for (int j = 0; j < m; ++j) {
        // the operator's input: the basis vector itself, or its FP32 copy for a binary16 basis
        const float *vj = a.v32 ? a.v32 : (const float *)(V + (long)j * a.cvlen);
        if (int rc = apply(vj, a.w)) return rc;
        for (int pass = 0; pass < 2; ++pass) {
            if (int rc = dots((const TV *)V, a.cvlen, j + 1, a.w, j, GM_PROJECT)) return rc;
            hipLaunchKernelGGL(k_gm_axpy<TV>, dim3(eb), dim3(GTHR), 0, st, a, j + 1);
            GM_CHECK("k_gm_axpy launch");
        }
        if (int rc = dots((const float *)a.w, 0L, 1, a.w, j, GM_NORM)) return rc;
        hipLaunchKernelGGL(k_gm_scale<TV>, dim3(eb), dim3(GTHR), 0, st, a, (const float *)a.w, V + (long)(j + 1) * a.cvlen,
                           a.v32, 1);
        GM_CHECK("k_gm_scale launch");
    }
    hipLaunchKernelGGL(k_gm_solve, dim3(kb), dim3(64), 0, st, a, res_out, iters_out);
    GM_CHECK("k_gm_solve launch");
    hipLaunchKernelGGL(k_gm_combine<TV>, dim3(eb), dim3(GTHR), 0, st, a, u);
    GM_CHECK("k_gm_combine launch");
#undef GM_CHECK
    return MRHS_OK;
}

size_t cvec_bytes(const mrhs_op *op, int n_tv, int n)
{
    return align256((size_t)op->n_agg * 2 * n_tv * 2 * ((n + 3) / 4 * 4) * sizeof(float));
}

}  // namespace

size_t ws_bytes_coarse_solve(const mrhs_op *op, int n_tv, int n, int m) { return gm_layout(op, n_tv, n, m, nullptr, nullptr); }

int launch_coarse_solve(const mrhs_op *op, const float *Dc, int n_tv, const float *b, float *u, int n, int m, double tol,
                        double *res_out, int32_t *iters_out, void *ws, hipStream_t st)
{
    GmArgs a{};
    gm_layout(op, n_tv, n, m, (char *)ws, &a);
    a.tol = tol;
    auto apply = [&](const float *in, float *out) {
        return launch_coarse_apply_ex(op, Dc, 9, n_tv, nullptr, in, in, 1.f, -1, false, out, n, st, a.active, n);
    };
    return gmres_run<float>(a, b, u, m, res_out, iters_out, apply, st);
}

size_t ws_bytes_coarse_solve_f16(const mrhs_op *op, int n_tv, int n, int m)
{
    return gm_layout(op, n_tv, n, m, nullptr, nullptr, 2);
}

int launch_coarse_solve_f16(const mrhs_op *op, const __half *Dc16, int n_tv, const float *b, float *u, int n, int m,
                            double tol, double *res_out, int32_t *iters_out, void *ws, hipStream_t st)
{
    GmArgs a{};
    gm_layout(op, n_tv, n, m, (char *)ws, &a, 2);
    a.tol = tol;
    auto apply = [&](const float *in, float *out) {
        return launch_coarse_apply_f16(op, Dc16, n_tv, in, out, n, st, a.active, n);
    };
    return gmres_run<__half>(a, b, u, m, res_out, iters_out, apply, st);
}

size_t ws_bytes_coarse_solve_eo(const mrhs_op *op, int n_tv, int n, int m)
{
    return gm_layout(op, n_tv, n, m, nullptr, nullptr) + 3 * cvec_bytes(op, n_tv, n);
}

size_t coarse_inverse_lds_bytes(int n_tv)
{
    const size_t N2 = 2 * (size_t)n_tv;
    return N2 * N2 * sizeof(double2) + N2 * sizeof(double2) + N2 * sizeof(int);
}

int launch_coarse_self_inverse(const mrhs_op *op, const float *Dc, int n_tv, float *Dinv, int32_t *status,
                               hipStream_t st)
{
    const size_t lds = coarse_inverse_lds_bytes(n_tv);
    static size_t done = 0;
    if (lds > 65536 && lds > done) {
        if (int rc = hip_check(hipFuncSetAttribute((const void *)k_coarse_self_inverse,
                                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds),
                               "hipFuncSetAttribute(coarse self inverse LDS)"))
            return rc;
        done = lds;
    }
    if (status) {
        hipLaunchKernelGGL(k_inv_status_init, dim3(1), dim3(1), 0, st, status);
        if (int rc = hip_check(hipGetLastError(), "k_inv_status_init launch")) return rc;
    }
    hipLaunchKernelGGL(k_coarse_self_inverse, dim3(op->n_agg), dim3(256), lds, st, Dc, Dinv, 2 * n_tv, status);
    if (int rc = hip_check(hipGetLastError(), "k_coarse_self_inverse launch")) return rc;
    if (status) {
        hipLaunchKernelGGL(k_inv_status_final, dim3(1), dim3(1), 0, st, status);
        if (int rc = hip_check(hipGetLastError(), "k_inv_status_final launch")) return rc;
    }
    return MRHS_OK;
}

// The even-odd preconditioned coarse solve.  Coarse sites split by the parity of their
// coordinate sum (every coarse extent even, so each hop block joins opposite parities):
// D_c = [[A_ee, H_eo], [H_oe, A_oo]] with A the self blocks.  bhat_e = b_e - H_eo A_oo^-1 b_o;
// GMRES on S u_e = bhat_e, S = A_ee - H_eo A_oo^-1 H_oe (coarse vectors whose odd sites stay
// zero); u_o = A_oo^-1 (b_o - H_oe u_e).  Dinv: the self-block inverses (launch_coarse_self_inverse).
int launch_coarse_solve_eo(const mrhs_op *op, const float *Dc, const float *Dinv, int n_tv, const float *b, float *u,
                           int n, int m, double tol, double *res_out, int32_t *iters_out, void *ws, hipStream_t st)
{
    GmArgs a{};
    const size_t gmb = gm_layout(op, n_tv, n, m, (char *)ws, &a);
    a.tol = tol;
    const size_t cb = cvec_bytes(op, n_tv, n);
    float *bh = (float *)((char *)ws + gmb), *t1 = (float *)((char *)ws + gmb + cb), *t2 = (float *)((char *)ws + gmb + 2 * cb);
    auto ap = [&](const float *D, int nblk, const float *y0, const float *ys, const float *yh, float sh, int par, bool zero,
                  float *out, const int *gate = nullptr) {
        return launch_coarse_apply_ex(op, D, nblk, n_tv, y0, ys, yh, sh, par, zero, out, n, st, gate, gate ? n : 0);
    };
    // bhat = b - H (A_oo^-1 b_o) on the even sites, 0 on the odd ones
    if (int rc = ap(Dinv, 1, nullptr, b, nullptr, 1.f, 1, true, t1)) return rc;
    if (int rc = ap(Dc, 9, b, nullptr, t1, -1.f, 0, true, bh)) return rc;
    // S v = A v - H (A_oo^-1 (H v)_o) on the even sites
    auto schur = [&](const float *in, float *out) {
        if (int rc = ap(Dc, 9, nullptr, nullptr, in, 1.f, 1, true, t1, a.active)) return rc;
        if (int rc = ap(Dinv, 1, nullptr, t1, nullptr, 1.f, 1, true, t2, a.active)) return rc;
        return ap(Dc, 9, nullptr, in, t2, -1.f, 0, true, out, a.active);
    };
    if (int rc = gmres_run<float>(a, bh, u, m, res_out, iters_out, schur, st)) return rc;
    // u_o = A_oo^-1 (b - H u)_o, the even sites of u kept
    if (int rc = ap(Dc, 9, b, nullptr, u, -1.f, 1, true, t1)) return rc;
    return ap(Dinv, 1, nullptr, t1, nullptr, 1.f, 1, false, u);
}
