// internal.h -- shared declarations of the gfx950 library: the operator handle,
// lattice geometry in block-major order, and the device-side Wilson-clover stencil.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "mrhs.h"

// ---------------------------------------------------------------------------
// Geometry passed to kernels by value.  Native site = blk * Vb + off (block-major,
// both lexicographic); coordinates of blocks and of local offsets come from small
// tables packed 8 bits per direction.
// ---------------------------------------------------------------------------
struct KGeo {
    int L[4];
    int b[4];     // SAP block extents
    int nb[4];    // blocks per direction
    int ostr[4];  // local-offset strides: 1, b0, b0 b1, b0 b1 b2
    int bstr[4];  // block-index strides
    int Vb;       // block volume
    int nblk;     // number of blocks
    long V;       // lattice volume
    int S;        // short-vector length of the native layout
};

__host__ __device__ inline int unpack_coord(uint32_t p, int mu) { return (p >> (8 * mu)) & 0xff; }

// XCD-aware workgroup order: consecutive workgroups are dispatched round-robin over the
// 8 XCDs, so list entry li is given to workgroup w such that each XCD receives a
// contiguous run of the list (neighbouring work items share that XCD's L2).
__device__ inline int xcd_remap(int w, int nwg)
{
    const int q = nwg >> 3, r = nwg & 7, xcd = w & 7, slot = w >> 3;
    return xcd * q + (xcd < r ? xcd : r) + slot;
}

struct mrhs_op {
    mrhs_geom g;
    KGeo k;
    int prec;    // MRHS_PREC_*
    int dtype;   // element type of the op's native vectors
    int device;
    int na[4];   // aggregates per direction
    int Va;      // aggregate volume
    int n_agg;
    // fields in kernel layout: links [V][4][18], clover [V][72] (native site order)
    double *links64 = nullptr, *clover64 = nullptr;
    float *links32 = nullptr, *clover32 = nullptr;
    uint32_t *blk_coords = nullptr;  // [nblk]
    uint32_t *loc_coords = nullptr;  // [Vb]
    int32_t *colour_blocks = nullptr; // blocks of colour 0 then colour 1
    int n_colour[2];
    int32_t *agg_sites = nullptr;    // [n_agg][Va] native site of local site ls of aggregate i
    bool odd_blocks;                 // some direction has an odd number (> 1) of blocks
    int sap_tile, dirac_tile;
    size_t max_lds;
    // SAP block solver (mrhs_set_block_solver).  For the even-odd one: A^-1 per site in the
    // clover layout (two Hermitian 6x6 blocks) and the block-local offsets in parity order,
    // the Vb / 2 even sites first.
    int block_solver = 0;
    double *cloverinv64 = nullptr;
    float *cloverinv32 = nullptr;
    int32_t *eo_sites = nullptr;  // [Vb]
    int *status = nullptr;        // device status word (mrhs_pack's FP16 range flag)
};

// error reporting (abi.hip)
int set_error(int code, const std::string &msg);
int hip_check(hipError_t e, const char *what);

// ---------------------------------------------------------------------------
// Element conversion
// ---------------------------------------------------------------------------
template <typename To> __device__ inline To cvt_to(float v);
template <> __device__ inline float cvt_to<float>(float v) { return v; }
template <> __device__ inline double cvt_to<double>(float v) { return v; }
template <> __device__ inline __half cvt_to<__half>(float v) { return __float2half_rn(v); }

template <typename Tc, typename Ts> __device__ inline Tc load_as(const Ts *p) { return static_cast<Tc>(*p); }
template <> __device__ inline float load_as<float, __half>(const __half *p) { return __half2float(*p); }
template <> __device__ inline double load_as<double, __half>(const __half *p) { return (double)__half2float(*p); }

// type in which a neighbour spinor of storage type Ts is held for arithmetic in Tc
template <typename Tc, typename Ts> struct ChiType { using type = Tc; };
template <> struct ChiType<double, float> { using type = float; };
template <> struct ChiType<double, __half> { using type = float; };

template <typename Ts, typename Tc> __device__ inline Ts store_as(Tc v) { return static_cast<Ts>(v); }
template <> __device__ inline __half store_as<__half, float>(float v) { return __float2half_rn(v); }
// double -> binary16 with a single round-to-nearest-even
__device__ inline __half dbl2half(double v) { return __half_raw{static_cast<_Float16>(v)}; }
template <> __device__ inline __half store_as<__half, double>(double v) { return dbl2half(v); }

// ---------------------------------------------------------------------------
// Spinors in registers: 12 complex components, index 3*spin + colour.
// ---------------------------------------------------------------------------
template <typename T> struct Spinor {
    T re[12], im[12];
};

template <typename T> __device__ inline void spinor_zero(Spinor<T> &s)
{
#pragma unroll
    for (int i = 0; i < 12; ++i) s.re[i] = s.im[i] = T(0);
}

// Gamma matrices of the DeGrand-Rossi chiral basis in sparse form: row r of g_mu has
// one non-zero, phase i^PH(mu,r) in column PERM(mu,r).  Directions 0,1 pair spin rows
// (0<->3, 1<->2), directions 2,3 pair (0<->2, 1<->3).
__host__ __device__ constexpr int gperm(int mu, int r) { return mu < 2 ? 3 - r : (r + 2) & 3; }
__host__ __device__ constexpr int gphase(int mu, int r)
{
    // g0: i, i, -i, -i   g1: -1, 1, 1, -1   g2: i, -i, -i, i   g3: 1, 1, 1, 1   (as powers of i)
    return mu == 0 ? (r < 2 ? 1 : 3) : mu == 1 ? ((r == 0 || r == 3) ? 2 : 0) : mu == 2 ? ((r == 0 || r == 3) ? 1 : 3) : 0;
}

// (re, im) * i^P
template <int P, typename T> __device__ inline void mul_ipow(T re, T im, T &ore, T &oim)
{
    if constexpr ((P & 3) == 0) { ore = re; oim = im; }
    else if constexpr ((P & 3) == 1) { ore = -im; oim = re; }
    else if constexpr ((P & 3) == 2) { ore = -re; oim = -im; }
    else { ore = im; oim = -re; }
}

// One hop term: acc += (1 + SGN g_MU) W chi, where chi is the neighbour's spinor and
// W = U (DAG = false) or U^dag (DAG = true), U given as 18 reals (row-major re, im).
// The spin projector has rank 2: project to a half spinor, multiply two colour vectors,
// then rebuild the lower two spin rows from the upper two.
// chi may be held in a narrower type than the arithmetic (FP32 or FP16 storage read by the
// FP64 residual): its entries are converted (exactly) where they are used.
template <int MU, int SGN, bool DAG, typename T, typename Tx>
__device__ inline void hop_accumulate(const T (&U)[18], const Spinor<Tx> &chi, Spinor<T> &acc)
{
    constexpr int s = SGN > 0 ? 0 : 2;  // phase exponent of the sign
    T hre[2][3], him[2][3];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            T are, aim;
            if (r == 0)
                mul_ipow<gphase(MU, 0) + s>(T(chi.re[3 * gperm(MU, 0) + c]), T(chi.im[3 * gperm(MU, 0) + c]), are, aim);
            else
                mul_ipow<gphase(MU, 1) + s>(T(chi.re[3 * gperm(MU, 1) + c]), T(chi.im[3 * gperm(MU, 1) + c]), are, aim);
            hre[r][c] = T(chi.re[3 * r + c]) + are;
            him[r][c] = T(chi.im[3 * r + c]) + aim;
        }
    }
    // colour row a of W h for both half-spinor rows, added to all four spin rows at once, so
    // that only one colour row of the product is live at a time
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        T wre[2], wim[2];
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            T sr = 0, si = 0;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                T ur, ui;
                if constexpr (DAG) { ur = U[2 * (3 * c + a)]; ui = -U[2 * (3 * c + a) + 1]; }
                else { ur = U[2 * (3 * a + c)]; ui = U[2 * (3 * a + c) + 1]; }
                // one product per statement so that each contracts into an FMA
                sr += ur * hre[r][c];
                sr -= ui * him[r][c];
                si += ur * him[r][c];
                si += ui * hre[r][c];
            }
            wre[r] = sr;
            wim[r] = si;
        }
        acc.re[a] += wre[0];
        acc.im[a] += wim[0];
        acc.re[3 + a] += wre[1];
        acc.im[3 + a] += wim[1];
        T t2r, t2i, t3r, t3i;
        // row 2 = (SGN phase of row 2) * h[perm(2)], row 3 likewise
        mul_ipow<gphase(MU, 2) + s>(wre[gperm(MU, 2)], wim[gperm(MU, 2)], t2r, t2i);
        mul_ipow<gphase(MU, 3) + s>(wre[gperm(MU, 3)], wim[gperm(MU, 3)], t3r, t3i);
        acc.re[6 + a] += t2r;
        acc.im[6 + a] += t2i;
        acc.re[9 + a] += t3r;
        acc.im[9 + a] += t3i;
    }
}

// out[6hf..6hf+5] = A_hf psi[6hf..6hf+5] (ADD: += ) for one chiral half hf of the site term,
// held as 36 reals: 6 real diagonal entries, then the 15 upper entries (i<j, row-major) as
// (re, im); the lower triangle is their conjugate.
template <int HF, bool ADD = false, typename T, typename Tx>
__device__ inline void clover_half(const T (&cl)[36], const Spinor<Tx> &psi, Spinor<T> &out)
{
    constexpr int o = 6 * HF;
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        T sr = cl[i] * T(psi.re[o + i]), si = cl[i] * T(psi.im[o + i]);
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            if (j == i) continue;
            const int a = i < j ? i : j, bb = i < j ? j : i;
            const int kidx = a * 5 - a * (a - 1) / 2 + (bb - a - 1);  // index of pair (a,bb), a<bb
            T ur = cl[6 + 2 * kidx], ui = cl[7 + 2 * kidx];
            if (i > j) ui = -ui;  // lower triangle: conjugate
            sr += ur * T(psi.re[o + j]);
            sr -= ui * T(psi.im[o + j]);
            si += ur * T(psi.im[o + j]);
            si += ui * T(psi.re[o + j]);
        }
        if constexpr (ADD) {
            out.re[o + i] += sr;
            out.im[o + i] += si;
        } else {
            out.re[o + i] = sr;
            out.im[o + i] = si;
        }
    }
}

// Neighbour of a native site within the block-major order.  Returns the neighbour's
// block and offset; 'inside' is true when it stays in the same block without crossing
// a block face, or wraps inside a block that spans the whole direction.
struct NbrSite {
    int blk, off;
    bool same_block;
};

__device__ inline NbrSite nbr_fwd(const KGeo &g, int mu, int blk, int off, const int (&bc)[4], const int (&lc)[4])
{
    NbrSite n;
    if (lc[mu] + 1 < g.b[mu]) {
        n.blk = blk;
        n.off = off + g.ostr[mu];
        n.same_block = true;
    } else {
        n.off = off - (g.b[mu] - 1) * g.ostr[mu];
        n.blk = blk + (bc[mu] + 1 < g.nb[mu] ? g.bstr[mu] : -(g.nb[mu] - 1) * g.bstr[mu]);
        n.same_block = (g.nb[mu] == 1);
    }
    return n;
}

__device__ inline NbrSite nbr_bwd(const KGeo &g, int mu, int blk, int off, const int (&bc)[4], const int (&lc)[4])
{
    NbrSite n;
    if (lc[mu] > 0) {
        n.blk = blk;
        n.off = off - g.ostr[mu];
        n.same_block = true;
    } else {
        n.off = off + (g.b[mu] - 1) * g.ostr[mu];
        n.blk = blk + (bc[mu] > 0 ? -g.bstr[mu] : (g.nb[mu] - 1) * g.bstr[mu]);
        n.same_block = (g.nb[mu] == 1);
    }
    return n;
}

// element index of real component r of (group g, block blk, offset off, lane t)
__device__ inline long vec_index(const KGeo &k, int grp, int blk, int r, int off, int t)
{
    return (((long)grp * k.nblk + blk) * 24 + r) * (long)k.Vb * k.S + (long)off * k.S + t;
}

// Fields are stored site by site in native site order: links [V][4][18] (the 4 forward
// links of a site, 18 reals each, pre-scaled by -1/2), clover [V][72].  A lane loads a
// link or a clover half from one address with immediate offsets (64/128-bit loads).
template <typename T> struct Vec2;
template <> struct Vec2<float> { using type = float2; };
template <> struct Vec2<double> { using type = double2; };

template <typename Tf, typename T> __device__ inline void load_link(const Tf *__restrict__ links, long, int mu, long site, T (&U)[18])
{
    using V2 = typename Vec2<Tf>::type;
    const V2 *p = reinterpret_cast<const V2 *>(links + ((size_t)(uint32_t)site * 4 + mu) * 18);
#pragma unroll
    for (int c = 0; c < 9; ++c) {
        const V2 v = p[c];
        U[2 * c] = (T)v.x;
        U[2 * c + 1] = (T)v.y;
    }
}

template <int HF, typename Tf, typename T>
__device__ inline void load_clover_half(const Tf *__restrict__ cl, long, long site, T (&A)[36])
{
    using V2 = typename Vec2<Tf>::type;
    const V2 *p = reinterpret_cast<const V2 *>(cl + (size_t)(uint32_t)site * 72 + 36 * HF);
#pragma unroll
    for (int c = 0; c < 18; ++c) {
        const V2 v = p[c];
        A[2 * c] = (T)v.x;
        A[2 * c + 1] = (T)v.y;
    }
}
