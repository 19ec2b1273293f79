// transfer.hip -- the coarse-grid correction's building blocks on all right-hand sides at
// once (the refinement phase of the setup, Alg. 1 and 2): restriction y_c = R y and
// prolongation y = P y_c with R = Q^dag, P = Q per aggregate and spin half (Alg. 3), and the
// coarse operator applied to coarse vectors (the operator of the coarse solve).
//
// With the right-hand sides innermost each of these is a matrix-matrix product (Sec. 6):
//   restriction : (y_c)^h_i [N x n]      = (Q^h_i)^dag [N x 6Va] . y^h_i [6Va x n]
//   prolongation: y^h_i     [6Va x n]    = Q^h_i [6Va x N]       . (y_c)^h_i [N x n]
//   coarse apply: (D_c y_c)(i) [2N x n]  = sum_d Dc[i][d] [2N x 2N] . y_c(nbr_d(i)) [2N x n]
// and runs on v_mfma_f32_16x16x4f32 (complex = 4 real products) with FP32 accumulation.
// Lane l supplies A[l%16][l/16] and B[l/16][l%16] and holds D[4(l/16) + r][l%16] in
// accumulator register r.
//
// Coarse vectors (FP32): element (rhs k, coarse site i, coarse dof c = h n_tv + j, re/im p)
// at ((i * 2 n_tv + c) * 2 + p) * ldc + k, ldc = n rounded up to a multiple of 4.
#include <algorithm>

#include <type_traits>

#include "launch.h"
#include "stencil.h"

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
__device__ inline f4 mfma32(float x, float y, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(x, y, c, 0, 0, 0); }

constexpr int TTHR = 256;  // 4 wavefronts
constexpr int PSPLIT = 4;  // workgroups per aggregate half in the prolongation
constexpr int TNW = TTHR / 64;

template <typename T> __device__ inline float to_f32(T v) { return (float)v; }
template <> __device__ inline float to_f32<__half>(__half v) { return __half2float(v); }

struct TransArgs {
    KGeo g;
    int Va, n_agg, N, n, ldc;
    const int32_t *agg_sites;
    const void *Q;  // native test vectors (N of them)
    const void *y;  // native fine vectors (n of them)
    void *yo;       // native fine output (prolongation)
    const float *yc;
    float *yco;
};

// native element offset (without the vector part) of row r of half h of an aggregate, the
// aggregate's site offsets staged in sbase
__device__ inline uint32_t trow_off(const uint32_t *sbase, int h, uint32_t cstr, int r)
{
    const int sl = r / 6, q = r - 6 * sl;
    const int sp = q >= 3 ? 1 : 0, c = q - 3 * sp;
    return sbase[sl] + (uint32_t)(2 * (3 * (2 * h + sp) + c)) * cstr;
}

// vector k of a native set: group and lane part of the element offset
__device__ inline size_t tcol_off(const KGeo &g, int k)
{
    const int grp = k / g.S, t = k - grp * g.S;
    return (size_t)grp * g.nblk * 24 * g.Vb * g.S + t;
}

__device__ inline void stage_agg_sites(const TransArgs &a, int i, uint32_t *sbase)
{
    for (int s = threadIdx.x; s < a.Va; s += blockDim.x) {
        const int ns = a.agg_sites[(size_t)i * a.Va + s];
        const int blk = ns / a.g.Vb, off = ns - blk * a.g.Vb;
        sbase[s] = ((uint32_t)blk * 24u * (uint32_t)a.g.Vb + (uint32_t)off) * (uint32_t)a.g.S;
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------------------
// restriction: one workgroup per (aggregate i, half h).  Output tiles: rows j (test
// vectors), columns k (right-hand sides), at most 2 x 2.  The wavefronts split the 6Va rows
// (K) and their partial tiles are summed in LDS in a fixed order.
// ---------------------------------------------------------------------------------------
template <typename Tq, typename Ty>
__global__ void __launch_bounds__(TTHR) k_restrict(TransArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t *sbase = reinterpret_cast<uint32_t *>(smem);          // [Va]
    float *part = reinterpret_cast<float *>(sbase + a.Va);          // [2 (re/im)][32][32]
    const int i = blockIdx.x >> 1, h = blockIdx.x & 1;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const Tq *Q = static_cast<const Tq *>(a.Q);
    const Ty *y = static_cast<const Ty *>(a.y);
    const uint32_t cstr = (uint32_t)a.g.Vb * (uint32_t)a.g.S;
    const int TJ = (a.N + 15) / 16, TK = (a.n + 15) / 16;
    stage_agg_sites(a, i, sbase);

    f4 ar[2][2], ai[2][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int z = 0; z < 2; ++z) ar[x][z] = ai[x][z] = f4{0.f, 0.f, 0.f, 0.f};
    // per lane: test vector j = 16 tj + l%16 (A operand column), rhs k = 16 tk + l%16
    size_t qo[2], yo[2];
    bool qok[2], yok[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int j = 16 * t + (lane & 15);
        qok[t] = t < TJ && j < a.N;
        qo[t] = qok[t] ? tcol_off(a.g, j) : 0;
        yok[t] = t < TK && j < a.n;
        yo[t] = yok[t] ? tcol_off(a.g, j) : 0;
    }
    const int rows = 6 * a.Va;
    for (int r0 = 4 * wave; r0 < rows; r0 += 4 * TNW) {
        const int r = r0 + (lane >> 4);
        const bool rok = r < rows;
        const uint32_t ro = rok ? trow_off(sbase, h, cstr, r) : 0;
        float qr[2], qi[2], yr[2], yi[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const bool okq = rok && qok[t], oky = rok && yok[t];
            const size_t iq = okq ? ro + qo[t] : 0, iy = oky ? ro + yo[t] : 0;
            const float a0 = to_f32(Q[iq]), a1 = to_f32(Q[okq ? iq + cstr : 0]);
            const float b0 = to_f32(y[iy]), b1 = to_f32(y[oky ? iy + cstr : 0]);
            qr[t] = okq ? a0 : 0.f;
            qi[t] = okq ? a1 : 0.f;
            yr[t] = oky ? b0 : 0.f;
            yi[t] = oky ? b1 : 0.f;
        }
        // conj(q) y = (qr yr + qi yi) + i (qr yi - qi yr)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj)
#pragma unroll
            for (int tk = 0; tk < 2; ++tk) {
                if (tj >= TJ || tk >= TK) continue;
                ar[tj][tk] = mfma32(qr[tj], yr[tk], ar[tj][tk]);
                ar[tj][tk] = mfma32(qi[tj], yi[tk], ar[tj][tk]);
                ai[tj][tk] = mfma32(qr[tj], yi[tk], ai[tj][tk]);
                ai[tj][tk] = mfma32(-qi[tj], yr[tk], ai[tj][tk]);
            }
    }
    // partial tiles of the wavefronts summed in order
    for (int w = 0; w < TNW; ++w) {
        if (wave == w) {
#pragma unroll
            for (int tj = 0; tj < 2; ++tj)
#pragma unroll
                for (int tk = 0; tk < 2; ++tk) {
                    if (tj >= TJ || tk >= TK) continue;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int j = 16 * tj + 4 * (lane >> 4) + q, k = 16 * tk + (lane & 15);
                        float *pr = part + j * 32 + k, *pi = part + 1024 + j * 32 + k;
                        *pr = w == 0 ? ar[tj][tk][q] : *pr + ar[tj][tk][q];
                        *pi = w == 0 ? ai[tj][tk][q] : *pi + ai[tj][tk][q];
                    }
                }
        }
        __syncthreads();
    }
    // (y_c)^h_i: dof c = h N + j, right-hand side k (padding columns written as zero)
    float *out = a.yco + ((size_t)i * 2 * a.N + h * a.N) * 2 * a.ldc;
    for (int e = threadIdx.x; e < a.N * a.ldc; e += blockDim.x) {
        const int j = e / a.ldc, k = e - j * a.ldc;
        const bool ok = k < a.n;
        out[(size_t)(2 * j) * a.ldc + k] = ok ? part[j * 32 + k] : 0.f;
        out[(size_t)(2 * j + 1) * a.ldc + k] = ok ? part[1024 + j * 32 + k] : 0.f;
    }
}

// ---------------------------------------------------------------------------------------
// prolongation: PSPLIT workgroups per (aggregate i, half h), each taking every PSPLIT-th
// group of 16-row blocks (the output rows are independent).  (y_c)^h_i is staged in LDS;
// each wavefront forms 16-row blocks of Q^h_i (y_c)^h_i, K = the test vectors.
// ---------------------------------------------------------------------------------------
template <typename Tq, typename Ty>
__global__ void __launch_bounds__(TTHR) k_prolong(TransArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t *sbase = reinterpret_cast<uint32_t *>(smem);  // [Va]
    float *ycs = reinterpret_cast<float *>(sbase + a.Va);   // [2 (re/im)][32 (j)][32 (k)]
    const int i = blockIdx.x >> 1, h = blockIdx.x & 1;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const Tq *Q = static_cast<const Tq *>(a.Q);
    Ty *yo = static_cast<Ty *>(a.yo);
    const uint32_t cstr = (uint32_t)a.g.Vb * (uint32_t)a.g.S;
    const int TK = (a.n + 15) / 16, KS = (a.N + 3) / 4;
    for (int e = threadIdx.x; e < 2048; e += blockDim.x) {
        const int p = e >> 10, j = (e >> 5) & 31, k = e & 31;
        float v = 0.f;
        if (j < a.N && k < a.n) v = a.yc[(((size_t)i * 2 * a.N + h * a.N + j) * 2 + p) * a.ldc + k];
        ycs[e] = v;
    }
    stage_agg_sites(a, i, sbase);
    // output lanes: the n right-hand sides and the padding lanes of the last group (zero)
    const int nw = (a.n + a.g.S - 1) / a.g.S * a.g.S;
    size_t yoff[2];
    bool kok[2], kin[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int k = 16 * t + (lane & 15);
        kok[t] = t < TK && k < nw;
        kin[t] = k < a.n;
        yoff[t] = kok[t] ? tcol_off(a.g, k) : 0;
    }
    const int rows = 6 * a.Va;
    for (int b0 = 16 * (wave + TNW * (int)blockIdx.y); b0 < rows; b0 += 16 * TNW * (int)gridDim.y) {
        const int ra = b0 + (lane & 15);  // A operand row
        const bool raok = ra < rows;
        const uint32_t roa = raok ? trow_off(sbase, h, cstr, ra) : 0;
        f4 dr[2], di[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) dr[t] = di[t] = f4{0.f, 0.f, 0.f, 0.f};
        for (int ks = 0; ks < KS; ++ks) {
            const int j = 4 * ks + (lane >> 4);  // K index: test vector
            const bool ok = raok && j < a.N;
            const size_t iq = ok ? roa + tcol_off(a.g, j) : 0;
            const float q0 = to_f32(Q[iq]), q1 = to_f32(Q[ok ? iq + cstr : 0]);
            const float qr = ok ? q0 : 0.f, qi = ok ? q1 : 0.f;
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                if (t >= TK) continue;
                const int k = 16 * t + (lane & 15);
                const float br = ycs[j * 32 + k], bi = ycs[1024 + j * 32 + k];  // j < 32 always
                // q y_c = (qr br - qi bi) + i (qr bi + qi br)
                dr[t] = mfma32(qr, br, dr[t]);
                dr[t] = mfma32(-qi, bi, dr[t]);
                di[t] = mfma32(qr, bi, di[t]);
                di[t] = mfma32(qi, br, di[t]);
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = b0 + 4 * (lane >> 4) + q;
            if (r >= rows) continue;
            const uint32_t ro = trow_off(sbase, h, cstr, r);
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                if (!kok[t]) continue;
                const size_t idx = ro + yoff[t];
                yo[idx] = store_as<Ty>(kin[t] ? dr[t][q] : 0.f);
                yo[idx + cstr] = store_as<Ty>(kin[t] ? di[t][q] : 0.f);
            }
        }
    }
}

// ---------------------------------------------------------------------------------------
// coarse apply: one workgroup per (coarse site, 16-row tile of the 2N output rows).  The
// nine blocks are split over three groups of wavefronts (directions d = g, g + 3, g + 6);
// each group has one wavefront per 16-column tile of right-hand sides.  For each direction
// the group copies the block's 16-row slab (contiguous in D_c) into LDS with 16-byte loads
// and issues all its loads of the neighbour's vector (2N rows x 16 right-hand sides) before
// the KS = ceil(2N / 4) matrix-core steps.  The three partial tiles are summed through LDS in
// the order g = 0, 1, 2.
// ---------------------------------------------------------------------------------------
struct CApplyArgs {
    int na[4];
    int Vc, N, n, ldc;
    const float *Dc;     // [Vc][nblk][2N][2N][2], or null with
    const __half *Dc16;  // the same stored in binary16 (arithmetic stays FP32)
    int nblk;            // 9 (self, +x..+t, -x..-t) or 1 (self only)
    const float *yself;  // input of the self block (null: no self term)
    const float *yhop;   // input of the 8 hop blocks (null: no hop term)
    const float *y0;     // added to the result (nullable)
    float s_hop;         // sign of the hop term
    int parity;          // -1: every coarse site; 0 / 1: only the sites of that parity
    int zero_other;      // the other sites' output: 1 written as zero, 0 left untouched
    float *yco;
    const int *gate;     // nullable: with every one of its gate_n flags zero the launch does nothing
    int gate_n;
};

// uniform over the grid: false when a gate is given and all its flags are zero (at most 32
// flags, one per lane, combined over the wavefront; called with every lane active)
__device__ inline bool apply_gate_open(const CApplyArgs &a)
{
    if (!a.gate) return true;
    const int l = threadIdx.x & 63;
    const int f = l < a.gate_n ? a.gate[l] : 0;
    return __ballot(f != 0) != 0;
}

constexpr int CA_GROUPS = 3;
#ifndef CA_SITE_MIN
#define CA_SITE_MIN 1024
#endif
constexpr int CA_MAXTHR = 64 * CA_GROUPS * 2;  // two right-hand-side tiles (n <= 32)

template <int KS> __global__ void __launch_bounds__(CA_MAXTHR) k_coarse_apply(CApplyArgs a)
{
    __shared__ f4 part[CA_GROUPS - 1][2][2][64];  // [g - 1][tk][re, im][lane]
    __shared__ float slab[CA_GROUPS][16 * 130];  // 16 rows of 2N complex, row stride 4N + 2 floats
    if (!apply_gate_open(a)) return;
    const int N2 = 2 * a.N, TR = (N2 + 15) / 16, TK = (a.n + 15) / 16, RS = 2 * N2 + 2;
    const int i = blockIdx.x / TR, tr = blockIdx.x - i * TR;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = wave / TK, tk = wave - g * TK;
    int c[4], r = i;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        c[m] = r % a.na[m];
        r /= a.na[m];
    }
    const int row = 16 * tr + (lane & 15), k = 16 * tk + (lane & 15);
    const int rows_here = N2 - 16 * tr < 16 ? N2 - 16 * tr : 16;
    const bool rok = row < N2, kok = k < a.n;
    float *out = a.yco + (size_t)i * N2 * 2 * a.ldc;
    if (a.parity >= 0 && ((c[0] + c[1] + c[2] + c[3]) & 1) != a.parity) {
        // a site of the other parity (uniform over the workgroup, before any barrier)
        if (a.zero_other && g == 0)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int orow = 16 * tr + 4 * (lane >> 4) + q;
                if (orow < N2 && k < a.ldc) {
                    out[(size_t)(2 * orow) * a.ldc + k] = 0.f;
                    out[(size_t)(2 * orow + 1) * a.ldc + k] = 0.f;
                }
            }
        return;
    }
    f4 dr = {0.f, 0.f, 0.f, 0.f}, di = {0.f, 0.f, 0.f, 0.f};
    float *sl = slab[g];
    // the same number of rounds (and barriers) for every group
    for (int it = 0; it < (a.nblk + CA_GROUPS - 1) / CA_GROUPS; ++it) {
        const int d = g + CA_GROUPS * it;
        const float *ysrc = d == 0 ? a.yself : a.yhop;
        const bool use = d < a.nblk && ysrc != nullptr;  // uniform over the group
        const float sgn = d == 0 ? 1.f : a.s_hop;
        int cn[4] = {c[0], c[1], c[2], c[3]};
        if (d >= 1 && d <= 4) cn[d - 1] = (cn[d - 1] + 1) % a.na[d - 1];
        if (d >= 5 && d <= 8) cn[d - 5] = (cn[d - 5] - 1 + a.na[d - 5]) % a.na[d - 5];
        const int j = cn[0] + a.na[0] * (cn[1] + a.na[1] * (cn[2] + a.na[2] * cn[3]));
        float br[KS], bi[KS];
        if (use) {
            const size_t blk = ((size_t)i * a.nblk + d) * N2 * N2 * 2 + (size_t)16 * tr * N2 * 2;
            const float *yj = ysrc + (size_t)j * N2 * 2 * a.ldc;
            // the 16-row slab of the block (contiguous) into LDS, four reals per load
            const int nq = rows_here * a.N;  // four reals per load, 2 N2 / 4 = N per row
            for (int q = tk * 64 + lane; q < nq; q += 64 * TK) {
                const int rr = q / a.N, c4 = q - rr * a.N;
                float4 v;
                if (a.Dc16) {
                    const uint2 u = ((const uint2 *)(a.Dc16 + blk))[q];
                    const float2 lo = __half22float2(*reinterpret_cast<const __half2 *>(&u.x));
                    const float2 hi = __half22float2(*reinterpret_cast<const __half2 *>(&u.y));
                    v = make_float4(lo.x, lo.y, hi.x, hi.y);
                } else {
                    v = ((const float4 *)(a.Dc + blk))[q];
                }
                *(float2 *)&sl[rr * RS + 4 * c4] = make_float2(v.x, v.y);
                *(float2 *)&sl[rr * RS + 4 * c4 + 2] = make_float2(v.z, v.w);
            }
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const int col = 4 * ks + (lane >> 4);
                const bool bok = kok && col < N2;
                const size_t ib = bok ? (size_t)(2 * col) * a.ldc + k : 0;
                const float b0 = yj[ib], b1 = yj[bok ? ib + a.ldc : 0];
                br[ks] = bok ? sgn * b0 : 0.f;
                bi[ks] = bok ? sgn * b1 : 0.f;
            }
        }
        __syncthreads();
        if (use) {
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const int col = 4 * ks + (lane >> 4);
                const bool aok = rok && col < N2;
                const float2 v = *(const float2 *)&sl[(aok ? (lane & 15) * RS + 2 * col : 0)];
                const float xr = aok ? v.x : 0.f, xi = aok ? v.y : 0.f;
                dr = mfma32(xr, br[ks], dr);
                dr = mfma32(-xi, bi[ks], dr);
                di = mfma32(xr, bi[ks], di);
                di = mfma32(xi, br[ks], di);
            }
        }
        __syncthreads();
    }
    if (g > 0) {
        part[g - 1][tk][0][lane] = dr;
        part[g - 1][tk][1][lane] = di;
    }
    __syncthreads();
    if (g > 0) return;
#pragma unroll
    for (int q = 0; q < CA_GROUPS - 1; ++q) {
        dr += part[q][tk][0][lane];
        di += part[q][tk][1][lane];
    }
    const float *o0 = a.y0 ? a.y0 + (size_t)i * N2 * 2 * a.ldc : nullptr;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int orow = 16 * tr + 4 * (lane >> 4) + q;
        if (orow < N2 && k < a.ldc) {
            const size_t e = (size_t)(2 * orow) * a.ldc + k;
            const float ar = o0 ? o0[e] : 0.f, ai = o0 ? o0[e + a.ldc] : 0.f;
            out[e] = kok ? ar + dr[q] : 0.f;
            out[e + a.ldc] = kok ? ai + di[q] : 0.f;
        }
    }
}

// ---------------------------------------------------------------------------------------
// coarse apply for large coarse lattices: one workgroup per coarse site, wavefront w owning
// output rows 16w .. 16w + 15 for every right-hand side (up to two 16-column tiles).  For each
// direction the neighbour's coarse vector (2N rows x n right-hand sides) is staged in LDS once
// for all the wavefronts, re/im interleaved per right-hand side, double-buffered so that the
// next direction's copy is in flight during this one's products; each wavefront reads its
// 16-row slab of the direction's block straight into registers (read once per apply, so with
// non-temporal loads), the next direction's slab also in flight.  The order of the columns
// inside a contraction is free: lane (r = l % 16, g = l / 16) loads columns 2(g + 4q) and
// 2(g + 4q) + 1 of row r with one 16-byte load (8 bytes in binary16), and matrix-core step
// (q, h) contracts column 2(g + 4q) + h.  Sites are taken in XCD-contiguous runs, so the
// neighbours along x and y of a site are staged by workgroups of the same XCD close in time.
// ---------------------------------------------------------------------------------------
constexpr int CS_YRS = 36;   // LDS row stride of a staged vector, complex entries (32 + 4 of padding)
constexpr int CS_ROWS = 64;  // 2N <= 64

template <typename TD> struct SlabLoad;
template <> struct SlabLoad<float> {
    using raw = f4;
    static __device__ inline raw load(const float *p) { return __builtin_nontemporal_load((const f4 *)p); }
    static __device__ inline f4 expand(raw v) { return v; }
};
template <> struct SlabLoad<__half> {
    typedef unsigned int u2 __attribute__((ext_vector_type(2)));
    using raw = u2;
    static __device__ inline raw load(const __half *p) { return __builtin_nontemporal_load((const u2 *)p); }
    static __device__ inline f4 expand(raw v)
    {
        const unsigned int x = v.x, y = v.y;
        const float2 lo = __half22float2(*reinterpret_cast<const __half2 *>(&x));
        const float2 hi = __half22float2(*reinterpret_cast<const __half2 *>(&y));
        return f4{lo.x, lo.y, hi.x, hi.y};
    }
};

template <typename TD, int QN, int TK> __global__ void __launch_bounds__(256) k_coarse_apply_site(CApplyArgs a)
{
    __shared__ float2 ys[2][CS_ROWS * CS_YRS];
    if (!apply_gate_open(a)) return;
    using SL = SlabLoad<TD>;
    const int N2 = 2 * a.N, nthr = blockDim.x;
    const int i = xcd_remap(blockIdx.x, a.Vc);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, r = lane & 15, g = lane >> 4;
    int c[4], rem = i;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        c[m] = rem % a.na[m];
        rem /= a.na[m];
    }
    const int row = 16 * w + r;
    float *out = a.yco + (size_t)i * N2 * 2 * a.ldc;
    if (a.parity >= 0 && ((c[0] + c[1] + c[2] + c[3]) & 1) != a.parity) {
        // a site of the other parity (uniform over the workgroup, before any barrier)
        if (a.zero_other)
            for (int tk = 0; tk < TK; ++tk)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int orow = 16 * w + 4 * g + q, k = 16 * tk + r;
                    if (orow < N2 && k < a.ldc) {
                        out[(size_t)(2 * orow) * a.ldc + k] = 0.f;
                        out[(size_t)(2 * orow + 1) * a.ldc + k] = 0.f;
                    }
                }
        return;
    }
    const int nk4 = a.ldc / 4, items = N2 * nk4;  // staging items: 4 right-hand sides of one row
    // neighbour of direction d, its vector (null: no term) and the sign of its term
    auto src_of = [&](int d, float &sgn) -> const float * {
        const float *ysrc = d == 0 ? a.yself : a.yhop;
        sgn = d == 0 ? 1.f : a.s_hop;
        if (!ysrc) return nullptr;
        int cn[4] = {c[0], c[1], c[2], c[3]};
        if (d >= 1 && d <= 4) cn[d - 1] = (cn[d - 1] + 1) % a.na[d - 1];
        if (d >= 5) cn[d - 5] = (cn[d - 5] - 1 + a.na[d - 5]) % a.na[d - 5];
        const int j = cn[0] + a.na[0] * (cn[1] + a.na[1] * (cn[2] + a.na[2] * cn[3]));
        return ysrc + (size_t)j * N2 * 2 * a.ldc;
    };
    // staging registers: at most two items per thread (items <= 16 N <= 2 x threads)
    f4 yre[2], yim[2];
    auto stage_load = [&](const float *src) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int it = threadIdx.x + u * nthr;
            if (it < items) {
                const int cr = it / nk4, k4 = it - cr * nk4;
                yre[u] = *(const f4 *)(src + (size_t)(2 * cr) * a.ldc + 4 * k4);
                yim[u] = *(const f4 *)(src + (size_t)(2 * cr + 1) * a.ldc + 4 * k4);
            }
        }
    };
    auto stage_store = [&](float2 *dst, float sgn) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int it = threadIdx.x + u * nthr;
            if (it < items) {
                const int cr = it / nk4, k4 = it - cr * nk4;
                f4 *p = (f4 *)(dst + cr * CS_YRS + 4 * k4);
                p[0] = f4{sgn * yre[u].x, sgn * yim[u].x, sgn * yre[u].y, sgn * yim[u].y};
                p[1] = f4{sgn * yre[u].z, sgn * yim[u].z, sgn * yre[u].w, sgn * yim[u].w};
            }
        }
    };
    typename SL::raw A[QN], An[QN];
    auto slab_load = [&](int d, typename SL::raw (&dst)[QN]) {
        const size_t base = (((size_t)i * a.nblk + d) * N2 + row) * N2 * 2;
        const TD *D = a.Dc16 ? (const TD *)a.Dc16 : (const TD *)a.Dc;
#pragma unroll
        for (int q = 0; q < QN; ++q) {
            const int c2 = g + 4 * q;
            if (row < N2 && c2 < a.N) dst[q] = SL::load(D + base + 4 * c2);
            else dst[q] = typename SL::raw{};
        }
    };
    f4 dr[2], di[2];
#pragma unroll
    for (int tk = 0; tk < 2; ++tk) dr[tk] = di[tk] = f4{0.f, 0.f, 0.f, 0.f};
    // binary16 D_c with two right-hand-side tiles: three real products per complex one (Gauss);
    // the third accumulator pair fits in the registers of three wavefronts per SIMD there, not
    // with FP32 D_c, whose slab takes twice the registers
    constexpr bool G3 = std::is_same<TD, __half>::value;
    f4 t3[2] = {f4{0.f, 0.f, 0.f, 0.f}, f4{0.f, 0.f, 0.f, 0.f}};

    float sgn0;
    const float *s0 = src_of(0, sgn0);
    if (s0) {
        stage_load(s0);
        slab_load(0, A);
        stage_store(ys[0], sgn0);
    }
    __syncthreads();
#pragma unroll 1
    for (int d = 0; d < a.nblk; ++d) {
        float sgn_c, sgn_n = 1.f;
        const bool cur = src_of(d, sgn_c) != nullptr;
        const float *sn = d + 1 < a.nblk ? src_of(d + 1, sgn_n) : nullptr;
        if (sn) {
            stage_load(sn);
            slab_load(d + 1, An);
        }
        if (cur) {
            const float2 *yb = ys[d & 1];
            // four independent accumulator chains between dependent matrix-core steps: the two
            // right-hand-side tiles, or with one tile its two accumulator pairs (alternate
            // column steps, added at the end)
#pragma unroll
            for (int q = 0; q < QN; ++q) {
                const f4 v = SL::expand(A[q]);
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int col = 2 * (g + 4 * q) + h;
                    const float ar = h ? v.z : v.x, ai = h ? v.w : v.y;
                    float2 b[2];
#pragma unroll
                    for (int tk = 0; tk < 2; ++tk) {
                        const int k = 16 * (TK == 2 ? tk : 0) + r;
                        b[tk] = {0.f, 0.f};
                        if (col < N2 && k < a.n) b[tk] = yb[col * CS_YRS + k];
                    }
                    if (TK == 2 && G3) {
                        // t1 = Ar Br (in dr), t2 = Ai Bi (in di), t3 = (Ar + Ai)(Br + Bi)
                        const float as = ar + ai;
                        dr[0] = mfma32(ar, b[0].x, dr[0]);
                        di[0] = mfma32(ai, b[0].y, di[0]);
                        t3[0] = mfma32(as, b[0].x + b[0].y, t3[0]);
                        dr[1] = mfma32(ar, b[1].x, dr[1]);
                        di[1] = mfma32(ai, b[1].y, di[1]);
                        t3[1] = mfma32(as, b[1].x + b[1].y, t3[1]);
                    } else if (TK == 2) {
                        dr[0] = mfma32(ar, b[0].x, dr[0]);
                        di[0] = mfma32(ar, b[0].y, di[0]);
                        dr[1] = mfma32(ar, b[1].x, dr[1]);
                        di[1] = mfma32(ar, b[1].y, di[1]);
                        dr[0] = mfma32(-ai, b[0].y, dr[0]);
                        di[0] = mfma32(ai, b[0].x, di[0]);
                        dr[1] = mfma32(-ai, b[1].y, dr[1]);
                        di[1] = mfma32(ai, b[1].x, di[1]);
                    } else {
                        const int u = h;  // alternate pairs of accumulators by column step
                        dr[u] = mfma32(ar, b[0].x, dr[u]);
                        di[u] = mfma32(ar, b[0].y, di[u]);
                        dr[u] = mfma32(-ai, b[0].y, dr[u]);
                        di[u] = mfma32(ai, b[0].x, di[u]);
                    }
                }
            }
        }
        if (sn) stage_store(ys[(d + 1) & 1], sgn_n);
        __syncthreads();
#pragma unroll
        for (int q = 0; q < QN; ++q) A[q] = An[q];
    }
    if (TK == 1) {
        dr[0] += dr[1];
        di[0] += di[1];
    } else if (G3) {
        // Re = t1 - t2, Im = t3 - t1 - t2
#pragma unroll
        for (int tk = 0; tk < 2; ++tk) {
            const f4 t1 = dr[tk], t2 = di[tk];
            dr[tk] = t1 - t2;
            di[tk] = t3[tk] - t1 - t2;
        }
    }
    const float *o0 = a.y0 ? a.y0 + (size_t)i * N2 * 2 * a.ldc : nullptr;
    for (int tk = 0; tk < TK; ++tk)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int orow = 16 * w + 4 * g + q, k = 16 * tk + r;
            if (orow < N2 && k < a.ldc) {
                const size_t e = (size_t)(2 * orow) * a.ldc + k;
                const bool kok = k < a.n;
                const float ar = o0 ? o0[e] : 0.f, ai = o0 ? o0[e + a.ldc] : 0.f;
                out[e] = kok ? ar + (tk ? dr[1][q] : dr[0][q]) : 0.f;
                out[e + a.ldc] = kok ? ai + (tk ? di[1][q] : di[0][q]) : 0.f;
            }
        }
}

template <typename TD, int QN> int coarse_apply_site_q(const CApplyArgs &a, int qn, hipStream_t st)
{
    if constexpr (QN < 8) {
        if (qn > QN) return coarse_apply_site_q<TD, QN + 1>(a, qn, st);
    }
    const int waves = (2 * a.N + 15) / 16;
    if (a.n > 16) hipLaunchKernelGGL((k_coarse_apply_site<TD, QN, 2>), dim3(a.Vc), dim3(64 * waves), 0, st, a);
    else hipLaunchKernelGGL((k_coarse_apply_site<TD, QN, 1>), dim3(a.Vc), dim3(64 * waves), 0, st, a);
    return hip_check(hipGetLastError(), "k_coarse_apply_site launch");
}

// KS = ceil(2N / 4) = 1 .. 16 (n_tv <= 32)
template <int KS> int coarse_apply_ks(const CApplyArgs &a, int ks, hipStream_t st)
{
    if constexpr (KS < 16) {
        if (ks > KS) return coarse_apply_ks<KS + 1>(a, ks, st);
    }
    const int TR = (2 * a.N + 15) / 16, TK = (a.n + 15) / 16;
    hipLaunchKernelGGL(k_coarse_apply<KS>, dim3(a.Vc * TR), dim3(64 * CA_GROUPS * TK), 0, st, a);
    return hip_check(hipGetLastError(), "k_coarse_apply launch");
}

TransArgs trans_args(const mrhs_op *op, int n_tv, int n)
{
    TransArgs a{};
    a.g = op->k;
    a.Va = op->Va;
    a.n_agg = op->n_agg;
    a.N = n_tv;
    a.n = n;
    a.ldc = (n + 3) / 4 * 4;
    a.agg_sites = op->agg_sites;
    return a;
}

template <typename Tq, typename Ty> int restrict_typed(const TransArgs &a, hipStream_t st)
{
    const size_t lds = sizeof(uint32_t) * a.Va + sizeof(float) * 2048;
    hipLaunchKernelGGL((k_restrict<Tq, Ty>), dim3(2 * a.n_agg), dim3(TTHR), lds, st, a);
    return hip_check(hipGetLastError(), "k_restrict launch");
}

template <typename Tq, typename Ty> int prolong_typed(const TransArgs &a, hipStream_t st)
{
    const size_t lds = sizeof(uint32_t) * a.Va + sizeof(float) * 2048;
    hipLaunchKernelGGL((k_prolong<Tq, Ty>), dim3(2 * a.n_agg, PSPLIT), dim3(TTHR), lds, st, a);
    return hip_check(hipGetLastError(), "k_prolong launch");
}

template <typename Tq> int restrict_y(const TransArgs &a, int ydt, hipStream_t st)
{
    if (ydt == MRHS_DTYPE_F64) return restrict_typed<Tq, double>(a, st);
    if (ydt == MRHS_DTYPE_F32) return restrict_typed<Tq, float>(a, st);
    return restrict_typed<Tq, __half>(a, st);
}

template <typename Tq> int prolong_y(const TransArgs &a, int ydt, hipStream_t st)
{
    if (ydt == MRHS_DTYPE_F64) return prolong_typed<Tq, double>(a, st);
    if (ydt == MRHS_DTYPE_F32) return prolong_typed<Tq, float>(a, st);
    return prolong_typed<Tq, __half>(a, st);
}

}  // namespace

size_t transfer_lds_bytes(const mrhs_op *op) { return sizeof(uint32_t) * op->Va + sizeof(float) * 2048; }

int launch_restrict(const mrhs_op *op, const void *Q, int qdt, int n_tv, const void *y, int ydt, float *yc, int n,
                    hipStream_t st)
{
    TransArgs a = trans_args(op, n_tv, n);
    a.Q = Q;
    a.y = y;
    a.yco = yc;
    if (qdt == MRHS_DTYPE_F64) return restrict_y<double>(a, ydt, st);
    if (qdt == MRHS_DTYPE_F32) return restrict_y<float>(a, ydt, st);
    return restrict_y<__half>(a, ydt, st);
}

int launch_prolong(const mrhs_op *op, const void *Q, int qdt, int n_tv, const float *yc, void *y, int ydt, int n,
                   hipStream_t st)
{
    TransArgs a = trans_args(op, n_tv, n);
    a.Q = Q;
    a.yc = yc;
    a.yo = y;
    if (qdt == MRHS_DTYPE_F64) return prolong_y<double>(a, ydt, st);
    if (qdt == MRHS_DTYPE_F32) return prolong_y<float>(a, ydt, st);
    return prolong_y<__half>(a, ydt, st);
}

int launch_coarse_apply(const mrhs_op *op, const float *Dc, int n_tv, const float *yc, float *yco, int n,
                        hipStream_t st)
{
    return launch_coarse_apply_ex(op, Dc, 9, n_tv, nullptr, yc, yc, 1.f, -1, false, yco, n, st);
}

namespace {

int coarse_apply_any(const mrhs_op *op, const float *Dc, const __half *Dc16, int nblk, int n_tv, const float *y0,
                     const float *yself, const float *yhop, float s_hop, int parity, bool zero_other, float *yco, int n,
                     hipStream_t st, const int *gate, int gate_n)
{
    CApplyArgs a{};
    a.gate = gate;
    a.gate_n = gate_n;
    a.Dc16 = Dc16;
    for (int mu = 0; mu < 4; ++mu) a.na[mu] = op->na[mu];
    a.Vc = op->n_agg;
    a.N = n_tv;
    a.n = n;
    a.ldc = (n + 3) / 4 * 4;
    a.Dc = Dc;
    a.nblk = nblk;
    a.yself = yself;
    a.yhop = yhop;
    a.y0 = y0;
    a.s_hop = s_hop;
    a.parity = parity;
    a.zero_other = zero_other ? 1 : 0;
    a.yco = yco;
    if (n_tv < 1 || n_tv > 32 || n < 1 || n > 32) return set_error(MRHS_EUNSUPPORTED, "coarse apply: n_tv and n must be 1..32");
    // many coarse sites: one workgroup per site; few: one per (site, 16-row tile), which
    // gives the chip more workgroups
    if (a.Vc >= CA_SITE_MIN) {
        const int qn = (n_tv + 3) / 4;
        return Dc16 ? coarse_apply_site_q<__half, 1>(a, qn, st) : coarse_apply_site_q<float, 1>(a, qn, st);
    }
    return coarse_apply_ks<1>(a, (2 * n_tv + 3) / 4, st);
}

}  // namespace

int launch_coarse_apply_ex(const mrhs_op *op, const float *Dc, int nblk, int n_tv, const float *y0, const float *yself,
                           const float *yhop, float s_hop, int parity, bool zero_other, float *yco, int n,
                           hipStream_t st, const int *gate, int gate_n)
{
    return coarse_apply_any(op, Dc, nullptr, nblk, n_tv, y0, yself, yhop, s_hop, parity, zero_other, yco, n, st, gate,
                            gate_n);
}

int launch_coarse_apply_f16(const mrhs_op *op, const __half *Dc16, int n_tv, const float *yc, float *yco, int n,
                            hipStream_t st, const int *gate, int gate_n)
{
    return coarse_apply_any(op, nullptr, Dc16, 9, n_tv, nullptr, yc, yc, 1.f, -1, false, yco, n, st, gate, gate_n);
}
