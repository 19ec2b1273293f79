// gs.hip -- block Gram-Schmidt of the test vectors per aggregate and spin half (the
// setup of R = Q^dag and P = Q, Sec. 2; the blocks R^h_i of Alg. 3), in FP64 on the
// matrix cores.
//
// One workgroup (4 wavefronts) per (aggregate i, half h).  V^h_i has 6 Va rows (local site,
// spin in the half, colour) and n_tv <= 32 columns, padded to NP = 16 or 32.  CholQR2:
//   G1 = V^dag V = R1^dag R1,  Q1 = V R1^-1,  G2 = Q1^dag Q1 = R2^dag R2,  Q = V (R1^-1 R2^-1),
// the thin QR factor with a real positive triangular diagonal (the Q that Gram-Schmidt
// with re-orthogonalisation produces).  The products V^dag V, V M and Q1^dag Q1 run on
// v_mfma_f64_16x16x4f64 (16x16 output tiles, complex = 3 real products, only the upper
// tiles of a Hermitian product, only the non-zero K steps of a triangular one); the
// Cholesky factorisations and triangular inverses of the n_tv x n_tv matrices run on the
// vector units in LDS and registers.
//
// V is read three times, in 16-row blocks that each wavefront loads one block ahead of the
// one on the matrix cores; the row offsets of the aggregate's sites are staged in LDS.  Q1
// is never stored: each 16-row block of it passes through the wavefront's own LDS rows
// into the second Gram product.
//
// MFMA lane layout of v_mfma_f64_16x16x4f64 (measured on gfx950): lane l supplies A[l%16][l/16]
// and B[l/16][l%16] and holds D[l/16 + 4r][l%16] in accumulator register r.
#include <algorithm>
#include <climits>

#include "launch.h"

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
constexpr int NTHR = 256;  // 4 wavefronts
constexpr int NW = NTHR / 64;
// aggregate sites whose row offsets are staged in LDS at a time (a 4^4 aggregate in one go;
// at 256 the LDS of three workgroups fits in a CU)
constexpr int SCH = 256;

struct GsArgs {
    KGeo g;
    int Va, n_tv;
    const int32_t *agg_sites;
    const void *V;
    void *Q;
    int32_t *status;
};

struct Cplx {
    double re, im;
};

template <typename T> __device__ inline double to_f64(T v) { return (double)v; }
template <> __device__ inline double to_f64<__half>(__half v) { return (double)__half2float(v); }

__device__ inline d4 mfma(double x, double y, d4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, c, 0, 0, 0); }

// Row n of V^h_i (local site n / 6, spin in the half, colour) inside the staged range of
// sites: native element offset without the column part.
__device__ inline uint32_t row_off(const uint32_t *sbase, int h, uint32_t cstr, int n)
{
    const int sl = n / 6, q = n - 6 * sl;
    const int sp = q >= 3 ? 1 : 0, c = q - 3 * sp;
    return sbase[sl] + (uint32_t)(2 * (3 * (2 * h + sp) + c)) * cstr;
}

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

// X = R^-1 for upper-triangular R (NP x NP in LDS).  Column l is solved by 8 lanes of one
// wavefront, bottom row first: X[k][l] = (delta_kl - sum_{k<j<=l} R[k][j] X[j][l]) / R[k][k];
// lane `sub` keeps rows j = sub (mod 8) of the column in registers, the partial sums are
// combined with shuffles.
template <int NP> __device__ void tri_inverse(const Cplx *R, Cplx *X)
{
    constexpr int NJ = NP / 8;
    const int l = threadIdx.x >> 3, sub = threadIdx.x & 7;
    const bool col = l < NP;
    double xr[NJ], xi[NJ];
#pragma unroll
    for (int m = 0; m < NJ; ++m) xr[m] = xi[m] = 0.0;
#pragma unroll
    for (int k = NP - 1; k >= 0; --k) {
        double sr = 0.0, si = 0.0;
        if (col) {
#pragma unroll
            for (int m = 0; m < NJ; ++m) {
                const int j = sub + 8 * m;
                if (j > k && j <= l) {
                    const Cplx r = R[k * NP + j];
                    sr += r.re * xr[m] - r.im * xi[m];
                    si += r.re * xi[m] + r.im * xr[m];
                }
            }
        }
        sr += __shfl_xor(sr, 1, 64);
        si += __shfl_xor(si, 1, 64);
        sr += __shfl_xor(sr, 2, 64);
        si += __shfl_xor(si, 2, 64);
        sr += __shfl_xor(sr, 4, 64);
        si += __shfl_xor(si, 4, 64);
        if (col && k <= l && sub == (k & 7)) {
            const double d = R[k * NP + k].re;
            xr[k >> 3] = (k == l ? 1.0 : -sr) / d;
            xi[k >> 3] = (k == l ? 0.0 : -si) / d;
        }
    }
    if (col) {
#pragma unroll
        for (int m = 0; m < NJ; ++m) X[(sub + 8 * m) * NP + l] = {xr[m], xi[m]};
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

// Gram accumulators of the tile pairs (0,0), (0,1), (1,1), real and imaginary part.  A
// diagonal pair needs three real products per K step, not four: Re = Xr^T Xr + Xi^T Xi,
// and for the imaginary part only P = Xr^T Xi, whose antisymmetric part P - P^T it is
// (taken once the wavefronts' tiles are summed, gram_fix_diag).  The off-diagonal pair takes
// Xr^T Xi - Xi^T Xr in full, or (G3) three real products as well (Gauss): t1 = Xr^T Xr',
// t2 = Xi^T Xi', t3 = (Xr + Xi)^T (Xr' - Xi'), Re = t1 + t2, Im = t1 - t2 - t3, with re
// holding t1 and im t2 until the tiles are written out.  G3 costs one more accumulator; the
// kernel for FP64 input, at its register limit, keeps the four-product form.
template <bool G3> struct GramAcc {
    d4 re[3], im[3], t3;
    __device__ void zero()
    {
#pragma unroll
        for (int p = 0; p < 3; ++p) re[p] = im[p] = d4{0.0, 0.0, 0.0, 0.0};
        if (G3) t3 = d4{0.0, 0.0, 0.0, 0.0};
    }
};

__device__ inline int pair_index(int ti, int tj) { return ti == 0 ? tj : 2; }

// G += x^dag x for one K step, x the operands of the NT column tiles
template <int NT, bool G3>
__device__ inline void gram_step(const double (&xr)[2], const double (&xi)[2], GramAcc<G3> &acc)
{
#pragma unroll
    for (int ti = 0; ti < NT; ++ti)
#pragma unroll
        for (int tj = ti; tj < NT; ++tj) {
            const int p = pair_index(ti, tj);
            if (G3 && ti != tj) {
                acc.re[p] = mfma(xr[ti], xr[tj], acc.re[p]);
                acc.im[p] = mfma(xi[ti], xi[tj], acc.im[p]);
                acc.t3 = mfma(xr[ti] + xi[ti], xr[tj] - xi[tj], acc.t3);
            } else {
                acc.re[p] = mfma(xr[ti], xr[tj], acc.re[p]);
                acc.re[p] = mfma(xi[ti], xi[tj], acc.re[p]);
                acc.im[p] = mfma(xr[ti], xi[tj], acc.im[p]);
                if (ti != tj) acc.im[p] = mfma(-xi[ti], xr[tj], acc.im[p]);
            }
        }
}

// the imaginary part of the diagonal tiles of G from P (upper triangle: P[r][c] - P[c][r])
template <int NT> __device__ inline void gram_fix_diag(Cplx *G, int NP)
{
    for (int e = threadIdx.x; e < NT * 256; e += blockDim.x) {
        const int t = e >> 8, r = 16 * t + ((e >> 4) & 15), c = 16 * t + (e & 15);
        if (r < c) G[r * NP + c].im -= G[c * NP + r].im;
        else if (r == c) G[r * NP + c].im = 0.0;
    }
    __syncthreads();
}

// add (or, for the first wavefront, write) this wavefront's Gram tiles into G
template <int NT, bool G3>
__device__ inline void gram_accumulate(const GramAcc<G3> &acc, Cplx *G, int NP, int lane, bool first)
{
#pragma unroll
    for (int ti = 0; ti < NT; ++ti)
#pragma unroll
        for (int tj = ti; tj < NT; ++tj) {
            const int p = pair_index(ti, tj);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = ti * 16 + (lane >> 4) + 4 * r, col = tj * 16 + (lane & 15);
                Cplx v = {acc.re[p][r], acc.im[p][r]};
                if (G3 && ti != tj) v = {acc.re[p][r] + acc.im[p][r], acc.re[p][r] - acc.im[p][r] - acc.t3[r]};
                if (!first) {
                    v.re += G[row * NP + col].re;
                    v.im += G[row * NP + col].im;
                }
                G[row * NP + col] = v;
            }
        }
}

// the wavefronts' partial Gram matrices summed into G in a fixed order
template <int NT, bool G3>
__device__ inline void gram_reduce(const GramAcc<G3> &acc, Cplx *G, int NP, int lane, int wave)
{
    for (int w = 0; w < NW; ++w) {
        if (wave == w) gram_accumulate<NT>(acc, G, NP, lane, w == 0);
        __syncthreads();
    }
}

// Operands of one 16-row block for a Gram product: K step j covers rows b0 + 4j .. b0 + 4j + 3;
// lane l holds row b0 + 4j + l/16 of columns 16 t + l%16.
template <typename Tv, int NT> struct GramRaw {
    Tv v[4][NT][2];
    uint32_t ok;  // bit NT j + t: the operand (j, t) is in range (else it reads as zero)
};

// vk[t]: V plus the offset of this lane's column 16 t + l%16 (V itself beyond n_tv).  An
// operand out of range (its row beyond nrows, its column beyond n_tv) reads a valid element
// (row 0, or column 0's group) and the products take it as zero, so that nothing here waits
// for the loads and no load is behind a branch.
template <typename Tv, int NT>
__device__ inline void load_gram(const Tv *const (&vk)[2], const uint32_t *sbase, int h, uint32_t cstr, int b0,
                                 int nrows, int N, int lane, GramRaw<Tv, NT> &o)
{
    o.ok = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int n = b0 + 4 * j + (lane >> 4);
        const bool nok = n < nrows;
        const uint32_t ro = row_off(sbase, h, cstr, nok ? n : 0);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const bool ok = nok && 16 * t + (lane & 15) < N;
            o.v[j][t][0] = vk[t][ro];
            o.v[j][t][1] = vk[t][ro + cstr];
            o.ok |= (uint32_t)ok << (NT * j + t);
        }
    }
}

template <typename Tv, int NT, bool G3>
__device__ inline void gram_block(const GramRaw<Tv, NT> &o, GramAcc<G3> &acc)
{
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        double xr[2] = {0.0, 0.0}, xi[2] = {0.0, 0.0};
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const bool ok = (o.ok >> (NT * j + t)) & 1u;
            xr[t] = ok ? to_f64(o.v[j][t][0]) : 0.0;
            xi[t] = ok ? to_f64(o.v[j][t][1]) : 0.0;
        }
        gram_step<NT>(xr, xi, acc);
        __builtin_amdgcn_sched_barrier(0);
    }
}

// Operands of one 16-row block for a transform V M: lane l holds row b0 + l%16 of columns
// 4 ks + l/16.
template <typename Tv, int NT> struct TransRaw {
    Tv v[4 * NT][2];
    uint32_t ok;  // bit ks: the operand ks is in range (else it reads as zero)
};

// As load_gram: an operand out of range reads a valid element (row 0, or column 0's group)
// and is taken as zero by the products; no load is behind a branch.
template <typename Tv, int NT>
__device__ inline void load_trans(const Tv *V, const uint32_t *sbase, const size_t *coff, int h, uint32_t cstr, int b0,
                                  int nrows, int N, int lane, TransRaw<Tv, NT> &o)
{
    const int n = b0 + (lane & 15);
    const bool nok = n < nrows;
    const Tv *vr = V + row_off(sbase, h, cstr, nok ? n : 0), *vi = vr + cstr;
    o.ok = 0;
#pragma unroll
    for (int ks = 0; ks < 4 * NT; ++ks) {
        const int k = 4 * ks + (lane >> 4);
        const size_t ck = k < N ? coff[k] : 0;
        o.v[ks][0] = vr[ck];
        o.v[ks][1] = vi[ck];
        o.ok |= (uint32_t)(nok && k < N) << ks;
    }
}

// tile tj of (the 16 rows) M for upper-triangular M (NP x NP in LDS); the accumulator of
// tile tj holds rows b0 + l/16 + 4r of columns 16 tj + l%16 in register r.  Three real
// products per complex one (Gauss): with t1 = Vr Mr, t2 = Vi Mi, t3 = (Vr + Vi)(Mr + Mi),
// Re V M = t1 - t2 and Im V M = t3 - t1 - t2.
template <typename Tv, int NT>
__device__ inline void trans_block(const TransRaw<Tv, NT> &o, const Cplx *M, int NP, int lane, d4 (&dr)[2], d4 (&di)[2])
{
    d4 t1[2], t2[2], t3[2];
#pragma unroll
    for (int tj = 0; tj < 2; ++tj) t1[tj] = t2[tj] = t3[tj] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int ks = 0; ks < NT * 4; ++ks) {
        const int k = 4 * ks + (lane >> 4);  // column of V = row of M
        const bool ok = (o.ok >> ks) & 1u;
        const double vr = ok ? to_f64(o.v[ks][0]) : 0.0, vi = ok ? to_f64(o.v[ks][1]) : 0.0, vs = vr + vi;
#pragma unroll
        for (int tj = 0; tj < NT; ++tj) {
            if (ks * 4 >= (tj + 1) * 16) continue;  // M is upper triangular
            const Cplx m = M[k * NP + tj * 16 + (lane & 15)];
            t1[tj] = mfma(vr, m.re, t1[tj]);
            t2[tj] = mfma(vi, m.im, t2[tj]);
            t3[tj] = mfma(vs, m.re + m.im, t3[tj]);
        }
        // one K step at a time: keeps the converted operands of later steps out of registers
        __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int tj = 0; tj < 2; ++tj) {
        dr[tj] = t1[tj] - t2[tj];
        di[tj] = t3[tj] - t1[tj] - t2[tj];
    }
}

// Runs body(operands, b0) for the 16-row blocks b0 = first, first + step, ... < nrows, with the
// loads of each block issued before the products of the previous one.  Two operand sets take
// turns, so that no register copy has to wait for loads still in flight.
template <typename Raw, typename Load, typename Body>
__device__ inline void pipelined_blocks(int first, int step, int nrows, Load load, Body body)
{
    Raw ra, rb;
    int b0 = first;
    if (b0 < nrows) load(b0, ra);
    while (b0 < nrows) {
        if (b0 + step < nrows) load(b0 + step, rb);
        body(ra, b0);
        b0 += step;
        if (b0 >= nrows) break;
        if (b0 + step < nrows) load(b0 + step, ra);
        body(rb, b0);
        b0 += step;
    }
}

// native offsets of the staged aggregate sites [ls0, ls0 + n): block and site part
__device__ inline void stage_sites(const GsArgs &a, int i, int ls0, int n, uint32_t *sbase)
{
    const KGeo &g = a.g;
    __syncthreads();
    for (int s = threadIdx.x; s < n; s += blockDim.x) {
        const int ns = a.agg_sites[(size_t)i * a.Va + ls0 + s];
        const int blk = ns / g.Vb, off = ns - blk * g.Vb;
        sbase[s] = ((uint32_t)blk * 24u * (uint32_t)g.Vb + (uint32_t)off) * (uint32_t)g.S;
    }
    __syncthreads();
}

// One workgroup per (aggregate i, half h).  Every pass walks the rows in 16-row blocks,
// NW blocks apart per wavefront; the first and the last pass load the next block's elements
// while the current one is on the matrix cores.  Three workgroups per CU (at most 168
// VGPRs): the second pass, whose Gram accumulators are live beside the transform's, loads
// each block right before its products, which keeps it within that budget without spilling.
template <typename Tv, typename Tq, int NT>
__global__ void __launch_bounds__(NTHR, 3) k_block_gs(GsArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int NP = NT * 16;
    const int N = a.n_tv;
    Cplx *X1 = reinterpret_cast<Cplx *>(smem);  // R1^-1
    Cplx *G = X1 + NP * NP;                      // Gram matrix / Cholesky factor / R1^-1 R2^-1
    Cplx *X2 = G + NP * NP;                      // R2^-1
    double *diag0 = reinterpret_cast<double *>(X2 + NP * NP);
    size_t *coff = reinterpret_cast<size_t *>(diag0 + NP);
    uint32_t *sbase = reinterpret_cast<uint32_t *>(coff + NP);
    __shared__ int bad;

    const Tv *V = static_cast<const Tv *>(a.V);
    Tq *Q = static_cast<Tq *>(a.Q);
    const int wi = xcd_remap(blockIdx.x, gridDim.x), i = wi >> 1, h = wi & 1;  // runs per XCD
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t cstr = (uint32_t)a.g.Vb * (uint32_t)a.g.S;
    const size_t gstr = (size_t)a.g.nblk * 24 * cstr;  // one group of S test vectors
    if (threadIdx.x == 0) bad = 0;
    for (int k = threadIdx.x; k < NP; k += blockDim.x) coff[k] = (size_t)(k / a.g.S) * gstr + (k % a.g.S);
    int staged = -1;  // first site of the staged range

    // G1 = V^dag V
    constexpr bool G3 = sizeof(Tv) < 8;  // the Gauss form of the off-diagonal Gram tile
    const Tv *vk[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int k = 16 * t + (lane & 15);
        vk[t] = V + (k < N ? (size_t)(k / a.g.S) * gstr + (k % a.g.S) : 0);
    }
    GramAcc<G3> acc;
    acc.zero();
    for (int ls0 = 0; ls0 < a.Va; ls0 += SCH) {
        const int nsc = std::min(SCH, a.Va - ls0), nrows = 6 * nsc;
        if (staged != ls0) {
            stage_sites(a, i, ls0, nsc, sbase);
            staged = ls0;
        }
        pipelined_blocks<GramRaw<Tv, NT>>(
            wave * 16, NW * 16, nrows,
            [&](int b0, GramRaw<Tv, NT> &o) { load_gram<Tv, NT>(vk, sbase, h, cstr, b0, nrows, N, lane, o); },
            [&](const GramRaw<Tv, NT> &o, int) { gram_block<Tv, NT, G3>(o, acc); });
    }
    __syncthreads();
    gram_reduce<NT>(acc, G, NP, lane, wave);
    gram_fix_diag<NT>(G, NP);
    for (int k = threadIdx.x; k < NP; k += blockDim.x) diag0[k] = G[k * NP + k].re;
    cholesky_inplace(G, diag0, N, NP, &bad);
    tri_inverse<NP>(G, X1);

    // G2 = Q1^dag Q1 with Q1 = V R1^-1 formed block by block on the matrix cores
    acc.zero();
    for (int ls0 = 0; ls0 < a.Va; ls0 += SCH) {
        const int nsc = std::min(SCH, a.Va - ls0), nrows = 6 * nsc;
        if (staged != ls0) {
            stage_sites(a, i, ls0, nsc, sbase);
            staged = ls0;
        }
        const auto load = [&](int b0, TransRaw<Tv, NT> &o) {
            load_trans<Tv, NT>(V, sbase, coff, h, cstr, b0, nrows, N, lane, o);
        };
        for (int b0 = wave * 16; b0 < nrows; b0 += NW * 16) {
            TransRaw<Tv, NT> cur;
            load(b0, cur);
            d4 dr[2], di[2];
            trans_block<Tv, NT>(cur, X1, NP, lane, dr, di);
            // the transform leaves row b0 + l/16 + 4r of column 16 t + l%16 in register r of
            // lane l, which is where K step r of the Gram product takes its operand: the 16
            // rows of Q1 go from the accumulators straight into the Gram product
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                double xr[2] = {0.0, 0.0}, xi[2] = {0.0, 0.0};
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    xr[t] = dr[t][j];
                    xi[t] = di[t][j];
                }
                gram_step<NT>(xr, xi, acc);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    }
    __syncthreads();
    gram_reduce<NT>(acc, G, NP, lane, wave);
    gram_fix_diag<NT>(G, NP);
    for (int k = threadIdx.x; k < NP; k += blockDim.x) diag0[k] = 1.0;
    cholesky_inplace(G, diag0, N, NP, &bad);
    tri_inverse<NP>(G, X2);
    tri_product(X1, X2, G, NP);  // G <- R1^-1 R2^-1
    // Q = V (R1^-1 R2^-1)
    for (int ls0 = 0; ls0 < a.Va; ls0 += SCH) {
        const int nsc = std::min(SCH, a.Va - ls0), nrows = 6 * nsc;
        if (staged != ls0) {
            stage_sites(a, i, ls0, nsc, sbase);
            staged = ls0;
        }
        const auto load = [&](int b0, TransRaw<Tv, NT> &o) {
            load_trans<Tv, NT>(V, sbase, coff, h, cstr, b0, nrows, N, lane, o);
        };
        pipelined_blocks<TransRaw<Tv, NT>>(wave * 16, NW * 16, nrows, load, [&](const TransRaw<Tv, NT> &cur, int b0) {
            d4 dr[2], di[2];
            trans_block<Tv, NT>(cur, G, NP, lane, dr, di);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int n = b0 + (lane >> 4) + 4 * r;
                if (n >= nrows) continue;
                const uint32_t ro = row_off(sbase, h, cstr, n);
#pragma unroll
                for (int tj = 0; tj < NT; ++tj) {
                    const int k = tj * 16 + (lane & 15);
                    if (k >= N) continue;
                    const size_t idx = ro + coff[k];
                    Q[idx] = store_as<Tq>(dr[tj][r]);
                    Q[idx + cstr] = store_as<Tq>(di[tj][r]);
                }
            }
        });
    }
    __syncthreads();
    if (threadIdx.x == 0 && bad && a.status) atomicMin(a.status, 1 + (int)blockIdx.x);
}

__global__ void k_status_init(int32_t *s) { *s = INT_MAX; }
__global__ void k_status_final(int32_t *s)
{
    if (*s == INT_MAX) *s = 0;
}

size_t gs_lds(int NP)
{
    return sizeof(Cplx) * 3 * NP * NP + (sizeof(double) + sizeof(size_t)) * NP + 4 * SCH;
}

template <typename Tv, typename Tq, int NT> int launch_typed(const GsArgs &a, int n_agg, size_t max_lds, hipStream_t st)
{
    const size_t lds = gs_lds(NT * 16);
    if (lds > max_lds) return set_error(MRHS_EUNSUPPORTED, "Gram-Schmidt LDS exceeds the workgroup limit");
    static size_t done = 0;
    if (lds > 65536 && lds > done) {
        if (int rc = hip_check(hipFuncSetAttribute((const void *)k_block_gs<Tv, Tq, NT>,
                                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds),
                               "hipFuncSetAttribute(gs LDS)"))
            return rc;
        done = lds;
    }
    hipLaunchKernelGGL((k_block_gs<Tv, Tq, NT>), dim3(2 * n_agg), dim3(NTHR), lds, st, a);
    return hip_check(hipGetLastError(), "k_block_gs launch");
}

template <typename Tv, typename Tq> int launch_nt(const GsArgs &a, int n_agg, size_t max_lds, hipStream_t st)
{
    return a.n_tv > 16 ? launch_typed<Tv, Tq, 2>(a, n_agg, max_lds, st) : launch_typed<Tv, Tq, 1>(a, n_agg, max_lds, st);
}

template <typename Tv> int launch_v(const GsArgs &a, int qdt, int n_agg, size_t max_lds, hipStream_t st)
{
    if (qdt == MRHS_DTYPE_F64) return launch_nt<Tv, double>(a, n_agg, max_lds, st);
    if (qdt == MRHS_DTYPE_F32) return launch_nt<Tv, float>(a, n_agg, max_lds, st);
    return launch_nt<Tv, __half>(a, n_agg, max_lds, st);  // FP16 storage of Q (rounded once from FP64)
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
    a.agg_sites = op->agg_sites;
    a.V = V;
    a.Q = Q;
    a.status = status;
    if (!a.agg_sites || !a.V || !a.Q) return set_error(MRHS_EINVAL, "block_orthonormalize: missing buffer");
    if (status) {
        hipLaunchKernelGGL(k_status_init, dim3(1), dim3(1), 0, st, status);
        if (int rc = hip_check(hipGetLastError(), "k_status_init launch")) return rc;
    }
    int rc;
    if (vdt == MRHS_DTYPE_F64) rc = launch_v<double>(a, qdt, op->n_agg, op->max_lds, st);
    else if (vdt == MRHS_DTYPE_F32) rc = launch_v<float>(a, qdt, op->n_agg, op->max_lds, st);
    else rc = launch_v<__half>(a, qdt, op->n_agg, op->max_lds, st);
    if (rc) return rc;
    if (status) {
        hipLaunchKernelGGL(k_status_final, dim3(1), dim3(1), 0, st, status);
        if (int rc2 = hip_check(hipGetLastError(), "k_status_final launch")) return rc2;
    }
    return MRHS_OK;
}
