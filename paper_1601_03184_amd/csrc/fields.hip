// fields.hip -- operator set-up on the GPU: re-lay the gauge links out in block-major
// site order (the 4 forward links of a site side by side, scaled by -1/2) and build the
// site term A(x) = (4 + m0) + C(x) as two Hermitian 6x6 blocks (chiral halves), in FP64;
// FP32 copies for the FP32 operators.
#include "launch.h"

namespace {

struct M3 {
    double re[9], im[9];
};

__device__ inline M3 load_canon(const double *__restrict__ U, long V, int mu, long x)
{
    M3 m;
    const double *p = U + ((long)mu * V + x) * 18;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        m.re[i] = p[2 * i];
        m.im[i] = p[2 * i + 1];
    }
    return m;
}

__device__ inline M3 dag(const M3 &a)
{
    M3 c;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            c.re[3 * r + k] = a.re[3 * k + r];
            c.im[3 * r + k] = -a.im[3 * k + r];
        }
    return c;
}

__device__ inline M3 mul(const M3 &a, const M3 &b)
{
    M3 c;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            double sr = 0, si = 0;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                sr += a.re[3 * r + j] * b.re[3 * j + k] - a.im[3 * r + j] * b.im[3 * j + k];
                si += a.re[3 * r + j] * b.im[3 * j + k] + a.im[3 * r + j] * b.re[3 * j + k];
            }
            c.re[3 * r + k] = sr;
            c.im[3 * r + k] = si;
        }
    return c;
}

__device__ inline long canon_index(const int (&L)[4], const int (&x)[4])
{
    return x[0] + (long)L[0] * (x[1] + (long)L[1] * (x[2] + (long)L[2] * x[3]));
}

__device__ inline long shifted(const int (&L)[4], const int (&x)[4], int mu, int dmu, int nu, int dnu)
{
    int y[4] = {x[0], x[1], x[2], x[3]};
    y[mu] = (y[mu] + dmu + L[mu]) % L[mu];
    y[nu] = (y[nu] + dnu + L[nu]) % L[nu];
    return canon_index(L, y);
}

// Sum of the four plaquettes in the (mu,nu) plane that start and end at x, each
// traversed mu-first (counter-clockwise in the mu-nu plane).
__device__ M3 plaquette_sum(const double *__restrict__ U, long V, const int (&L)[4], const int (&x)[4], int mu, int nu)
{
    const long x0 = canon_index(L, x);
    const long xm = shifted(L, x, mu, -1, nu, 0), xp = shifted(L, x, mu, 1, nu, 0);
    const long yn = shifted(L, x, mu, 0, nu, -1), yp = shifted(L, x, mu, 0, nu, 1);
    const long xm_yp = shifted(L, x, mu, -1, nu, 1), xm_yn = shifted(L, x, mu, -1, nu, -1);
    const long xp_yn = shifted(L, x, mu, 1, nu, -1);
    M3 s, t;
    // x -> x+mu -> x+mu+nu -> x+nu -> x
    s = mul(mul(load_canon(U, V, mu, x0), load_canon(U, V, nu, xp)),
            mul(dag(load_canon(U, V, mu, yp)), dag(load_canon(U, V, nu, x0))));
    // x -> x+nu -> x-mu+nu -> x-mu -> x
    t = mul(mul(load_canon(U, V, nu, x0), dag(load_canon(U, V, mu, xm_yp))),
            mul(dag(load_canon(U, V, nu, xm)), load_canon(U, V, mu, xm)));
#pragma unroll
    for (int i = 0; i < 9; ++i) { s.re[i] += t.re[i]; s.im[i] += t.im[i]; }
    // x -> x-mu -> x-mu-nu -> x-nu -> x
    t = mul(mul(dag(load_canon(U, V, mu, xm)), dag(load_canon(U, V, nu, xm_yn))),
            mul(load_canon(U, V, mu, xm_yn), load_canon(U, V, nu, yn)));
#pragma unroll
    for (int i = 0; i < 9; ++i) { s.re[i] += t.re[i]; s.im[i] += t.im[i]; }
    // x -> x-nu -> x+mu-nu -> x+mu -> x
    t = mul(mul(dag(load_canon(U, V, nu, yn)), load_canon(U, V, mu, yn)),
            mul(load_canon(U, V, nu, xp_yn), dag(load_canon(U, V, mu, x0))));
#pragma unroll
    for (int i = 0; i < 9; ++i) { s.re[i] += t.re[i]; s.im[i] += t.im[i]; }
    return s;
}

// (launched with 128 threads: the bound lets the plaquette products use 232 registers
// instead of spilling at the default 128)
__global__ void __launch_bounds__(128)
    k_build_fields(KGeo g, const double *__restrict__ Ucanon, const uint32_t *__restrict__ blk_coords,
                   const uint32_t *__restrict__ loc_coords, double m0, double csw, double *__restrict__ links,
                   double *__restrict__ clover)
{
    const long ns = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (ns >= g.V) return;
    const int blk = (int)(ns / g.Vb), off = (int)(ns % g.Vb);
    const uint32_t pb = blk_coords[blk], pl = loc_coords[off];
    int x[4];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) x[mu] = unpack_coord(pb, mu) * g.b[mu] + unpack_coord(pl, mu);
    const long cx = canon_index(g.L, x);
    for (int mu = 0; mu < 4; ++mu) {
        // kernel layout stores W = -U/2 (exact), the hop coefficient folded in
        const double *p = Ucanon + ((long)mu * g.V + cx) * 18;
        for (int c = 0; c < 18; ++c) links[(ns * 4 + mu) * 18 + c] = -0.5 * p[c];
    }
    // F_munu = Q_munu - Q_munu^dag for the 6 planes
    M3 F[6];
    int pl_i = 0;
    for (int mu = 0; mu < 4; ++mu)
        for (int nu = mu + 1; nu < 4; ++nu) {
            M3 Q = plaquette_sum(Ucanon, g.V, g.L, x, mu, nu);
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c) {
                    F[pl_i].re[3 * r + c] = Q.re[3 * r + c] - Q.re[3 * c + r];
                    F[pl_i].im[3 * r + c] = Q.im[3 * r + c] + Q.im[3 * c + r];
                }
            ++pl_i;
        }
    // C = -(csw/16) sum_{mu<nu} (g_mu g_nu) (x) F_munu.  g_mu g_nu maps spin row r to
    // column gperm(nu, gperm(mu, r)) with phase i^(gphase(mu,r) + gphase(nu, gperm(mu,r))),
    // and stays inside a chiral half.
    const double cf = -csw / 16.0;
    for (int hf = 0; hf < 2; ++hf) {
        double out[36];
        int kk = 0;
        for (int i = 0; i < 6; ++i) {
            const int ri = 2 * hf + i / 3, ai = i % 3;
            for (int j = i; j < 6; ++j) {
                const int rj = 2 * hf + j / 3, bj = j % 3;
                double sr = 0, si = 0;
                int p = 0;
                for (int mu = 0; mu < 4; ++mu)
                    for (int nu = mu + 1; nu < 4; ++nu, ++p) {
                        const int mid = gperm(mu, ri);
                        if (gperm(nu, mid) != rj) continue;
                        const int ph = (gphase(mu, ri) + gphase(nu, mid)) & 3;
                        double fr = F[p].re[3 * ai + bj], fi = F[p].im[3 * ai + bj];
                        double tr = ph == 0 ? fr : ph == 1 ? -fi : ph == 2 ? -fr : fi;
                        double ti = ph == 0 ? fi : ph == 1 ? fr : ph == 2 ? -fi : -fr;
                        sr += tr;
                        si += ti;
                    }
                sr *= cf;
                si *= cf;
                if (i == j) {
                    out[i] = sr + 4.0 + m0;  // the diagonal of a Hermitian block is real
                } else {
                    out[6 + 2 * kk] = sr;
                    out[7 + 2 * kk] = si;
                    ++kk;
                }
            }
        }
        for (int c = 0; c < 36; ++c) clover[ns * 72 + 36 * hf + c] = out[c];
    }
}

__global__ void k_to_f32(const double *__restrict__ in, float *__restrict__ out, long n)
{
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        out[i] = (float)in[i];
}

template <typename Ts>
__global__ void k_pack(KGeo g, const double *__restrict__ canon, Ts *__restrict__ nat, int n_rhs, long total,
                       const uint32_t *__restrict__ blk_coords, const uint32_t *__restrict__ loc_coords,
                       int *__restrict__ overflow)
{
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
        const int t = (int)(e % g.S);
        long rest = e / g.S;
        const int off = (int)(rest % g.Vb);
        rest /= g.Vb;
        const int r = (int)(rest % 24);
        rest /= 24;
        const int blk = (int)(rest % g.nblk);
        const int grp = (int)(rest / g.nblk);
        const int k = grp * g.S + t;
        double v = 0.0;
        if (k < n_rhs) {
            const uint32_t pb = blk_coords[blk], pl = loc_coords[off];
            long cx = 0, stride = 1;
            for (int mu = 0; mu < 4; ++mu) {
                cx += (long)(unpack_coord(pb, mu) * g.b[mu] + unpack_coord(pl, mu)) * stride;
                stride *= g.L[mu];
            }
            v = canon[((long)k * g.V + cx) * 24 + r];
        }
        if constexpr (sizeof(Ts) == 2) {
            if (fabs(v) > 65504.0) atomicOr(overflow, 1);
            nat[e] = dbl2half(v);
        } else {
            nat[e] = (Ts)v;
        }
    }
}

template <typename Ts>
__global__ void k_unpack(KGeo g, const Ts *__restrict__ nat, double *__restrict__ canon, int n_rhs, long total,
                         const uint32_t *__restrict__ blk_coords, const uint32_t *__restrict__ loc_coords)
{
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
        const int t = (int)(e % g.S);
        long rest = e / g.S;
        const int off = (int)(rest % g.Vb);
        rest /= g.Vb;
        const int r = (int)(rest % 24);
        rest /= 24;
        const int blk = (int)(rest % g.nblk);
        const int grp = (int)(rest / g.nblk);
        const int k = grp * g.S + t;
        if (k >= n_rhs) continue;
        const uint32_t pb = blk_coords[blk], pl = loc_coords[off];
        long cx = 0, stride = 1;
        for (int mu = 0; mu < 4; ++mu) {
            cx += (long)(unpack_coord(pb, mu) * g.b[mu] + unpack_coord(pl, mu)) * stride;
            stride *= g.L[mu];
        }
        double v;
        if constexpr (sizeof(Ts) == 2) v = (double)__half2float(nat[e]);
        else v = (double)nat[e];
        canon[((long)k * g.V + cx) * 24 + r] = v;
    }
}

// One Hermitian 6x6 block of the clover term per thread (site, half): the inverse by
// Gauss-Jordan elimination with partial pivoting in FP64, written back in the same packed
// form (real diagonal, then the upper triangle (a, b), a < b, row by row; the stored
// off-diagonal element is the mean of M^-1[a][b] and conj(M^-1[b][a])).
__global__ void k_clover_inverse(const double *__restrict__ clover, double *__restrict__ inv, long V,
                                 int *__restrict__ bad)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2 * V) return;
    const double *c = clover + t * 36;
    double ar[6][12], ai[6][12];  // [M | I]
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 12; ++j) {
            ar[i][j] = j == i + 6 ? 1.0 : 0.0;
            ai[i][j] = 0.0;
        }
    for (int i = 0; i < 6; ++i) ar[i][i] = c[i];
    int kk = 0;
    for (int i = 0; i < 6; ++i)
        for (int j = i + 1; j < 6; ++j, ++kk) {
            ar[i][j] = c[6 + 2 * kk];
            ai[i][j] = c[7 + 2 * kk];
            ar[j][i] = c[6 + 2 * kk];
            ai[j][i] = -c[7 + 2 * kk];
        }
    bool ok = true;
    for (int col = 0; col < 6; ++col) {
        int p = col;
        double best = ar[col][col] * ar[col][col] + ai[col][col] * ai[col][col];
        for (int i = col + 1; i < 6; ++i) {
            const double m = ar[i][col] * ar[i][col] + ai[i][col] * ai[i][col];
            if (m > best) {
                best = m;
                p = i;
            }
        }
        if (!(best > 0.0) || !isfinite(best)) {
            ok = false;
            break;
        }
        if (p != col)
            for (int j = 0; j < 12; ++j) {
                double tr = ar[col][j], ti = ai[col][j];
                ar[col][j] = ar[p][j];
                ai[col][j] = ai[p][j];
                ar[p][j] = tr;
                ai[p][j] = ti;
            }
        // row col /= pivot
        const double pr = ar[col][col] / best, pi = -ai[col][col] / best;  // 1 / pivot
        for (int j = 0; j < 12; ++j) {
            const double xr = ar[col][j], xi = ai[col][j];
            ar[col][j] = xr * pr - xi * pi;
            ai[col][j] = xr * pi + xi * pr;
        }
        for (int i = 0; i < 6; ++i) {
            if (i == col) continue;
            const double fr = ar[i][col], fi = ai[i][col];
            for (int j = 0; j < 12; ++j) {
                ar[i][j] -= fr * ar[col][j] - fi * ai[col][j];
                ai[i][j] -= fr * ai[col][j] + fi * ar[col][j];
            }
        }
    }
    double *o = inv + t * 36;
    if (!ok) {
        atomicOr(bad, 1);
        for (int i = 0; i < 36; ++i) o[i] = 0.0;
        return;
    }
    for (int i = 0; i < 6; ++i) o[i] = ar[i][i + 6];
    kk = 0;
    for (int i = 0; i < 6; ++i)
        for (int j = i + 1; j < 6; ++j, ++kk) {
            o[6 + 2 * kk] = 0.5 * (ar[i][j + 6] + ar[j][i + 6]);
            o[7 + 2 * kk] = 0.5 * (ai[i][j + 6] - ai[j][i + 6]);
        }
}

int grid_for(long n, int threads)
{
    long b = (n + threads - 1) / threads;
    return (int)(b < 65536L * 8 ? b : 65536L * 8);
}

}  // namespace

int launch_build_fields(mrhs_op *op, const double *links_canon, double m0, double csw, hipStream_t st)
{
    const KGeo &g = op->k;
    int threads = 128;
    hipLaunchKernelGGL(k_build_fields, dim3((unsigned)((g.V + threads - 1) / threads)), dim3(threads), 0, st, g,
                       links_canon, op->blk_coords, op->loc_coords, m0, csw, op->links64, op->clover64);
    if (int rc = hip_check(hipGetLastError(), "k_build_fields launch")) return rc;
    if (op->links32) {
        long nl = 4L * 18 * g.V, nc = 72L * g.V;
        hipLaunchKernelGGL(k_to_f32, dim3(grid_for(nl, 256)), dim3(256), 0, st, op->links64, op->links32, nl);
        hipLaunchKernelGGL(k_to_f32, dim3(grid_for(nc, 256)), dim3(256), 0, st, op->clover64, op->clover32, nc);
        if (int rc = hip_check(hipGetLastError(), "k_to_f32 launch")) return rc;
    }
    return MRHS_OK;
}

int launch_clover_inverse(mrhs_op *op, int *bad, hipStream_t st)
{
    const long V = op->k.V;
    hipLaunchKernelGGL(k_clover_inverse, dim3((unsigned)((2 * V + 127) / 128)), dim3(128), 0, st, op->clover64,
                       op->cloverinv64, V, bad);
    if (int rc = hip_check(hipGetLastError(), "k_clover_inverse launch")) return rc;
    if (op->cloverinv32) {
        const long nc = 72L * V;
        hipLaunchKernelGGL(k_to_f32, dim3(grid_for(nc, 256)), dim3(256), 0, st, op->cloverinv64, op->cloverinv32, nc);
        if (int rc = hip_check(hipGetLastError(), "k_to_f32 launch")) return rc;
    }
    return MRHS_OK;
}

int launch_pack(const mrhs_op *op, const double *canon, void *native, int dtype, int n_rhs, int *flag, hipStream_t st)
{
    const KGeo &g = op->k;
    long total = (long)native_elems(op, n_rhs);
    dim3 grid(grid_for(total, 256)), block(256);
    if (dtype == MRHS_DTYPE_F64)
        hipLaunchKernelGGL(k_pack<double>, grid, block, 0, st, g, canon, (double *)native, n_rhs, total, op->blk_coords,
                           op->loc_coords, flag);
    else if (dtype == MRHS_DTYPE_F32)
        hipLaunchKernelGGL(k_pack<float>, grid, block, 0, st, g, canon, (float *)native, n_rhs, total, op->blk_coords,
                           op->loc_coords, flag);
    else
        hipLaunchKernelGGL(k_pack<__half>, grid, block, 0, st, g, canon, (__half *)native, n_rhs, total, op->blk_coords,
                           op->loc_coords, flag);
    return hip_check(hipGetLastError(), "k_pack launch");
}

int launch_unpack(const mrhs_op *op, const void *native, int dtype, double *canon, int n_rhs, hipStream_t st)
{
    const KGeo &g = op->k;
    long total = (long)native_elems(op, n_rhs);
    dim3 grid(grid_for(total, 256)), block(256);
    if (dtype == MRHS_DTYPE_F64)
        hipLaunchKernelGGL(k_unpack<double>, grid, block, 0, st, g, (const double *)native, canon, n_rhs, total,
                           op->blk_coords, op->loc_coords);
    else if (dtype == MRHS_DTYPE_F32)
        hipLaunchKernelGGL(k_unpack<float>, grid, block, 0, st, g, (const float *)native, canon, n_rhs, total,
                           op->blk_coords, op->loc_coords);
    else
        hipLaunchKernelGGL(k_unpack<__half>, grid, block, 0, st, g, (const __half *)native, canon, n_rhs, total,
                           op->blk_coords, op->loc_coords);
    return hip_check(hipGetLastError(), "k_unpack launch");
}
