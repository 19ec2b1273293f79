// coarse.hip -- the coarse operator D_c = R D P from the orthonormalised test vectors
// (Sec. 2: the coarse-grid operator built in the setup; R = Q^dag as in Alg. 3).
//
// Column c = (h', k') of P is q_k' restricted to spin half h' on each aggregate.  Per
// coarse site i the 9 stored blocks are
//   self: Q_i^dag (A + hops that stay inside the aggregate) P_i, formed as G + sigma3 G^dag sigma3
//         with G = Q_i^dag (A/2 + forward hops that stay inside) P_i
//   +mu : Q_i^dag (1 - g_mu) W_mu P_{i+mu} over the sites on the +mu face   (W = -U/2)
//   -mu : sigma3 (+mu block of i-mu)^dag sigma3
// The last line is exact: the -mu face hop of i is the adjoint of the +mu face hop of i-mu
// conjugated by g5, and g5 acts on the coarse index as sigma3 = diag(1, -1) over halves.
//
// k_coarse: per (aggregate i, block d in self,+x..+t), the sites of the block's set (all
//           sites for self, the +mu face for +mu) in chunks of CHS: the chunk's rows
//           conj(q_k) and its columns w_c = (stencil part d) P_c, computed from Q on the
//           vector units, go to LDS; the 2N x 2N product accumulates on the matrix cores.
//           A +mu workgroup writes its block and, by the sigma3 relation, the -mu block of
//           aggregate i + mu.  Nothing is written to memory but D_c.
#include <algorithm>

#include "launch.h"
#include "stencil.h"

namespace {

constexpr int NTHR = 512;  // 8 wavefronts: one column item per thread and chunk at 32 vectors
constexpr int NW = NTHR / 64;
constexpr int CHS = 8;  // sites per LDS chunk
constexpr int MAXVA = 256;
constexpr int MAXFACE = 64;  // face sites of an aggregate whose neighbours the table holds
constexpr int MAXN = 32;     // test vectors
constexpr int QST = MAXN + 1, WST = 2 * MAXN + 1;  // LDS row strides (pairs) of rows and columns
constexpr int RMAX = (CHS * 12 + NTHR / MAXN - 1) / (NTHR / MAXN);  // rows per thread and chunk

template <typename Tq> struct CoarseArgs {
    KGeo g;
    int a[4], na[4], astr[4];
    int Va, n_agg, N;
    int sshift;          // log2 of the short length S
    long gsz;            // elements of one group of S right-hand sides
    int part_major;      // work items part by part (all self blocks first), for short grids
    const int32_t *agg_sites;
    const uint32_t *blk_coords, *loc_coords;
    const Tq *Q;
    float *Dc;       // [n_agg][9][2N][2N][2], or null with
    __half *Dc16;    // the same in binary16 (each entry rounded once from the FP32 sum)
};

// A site the workgroup touches: native index (fields), offset of its first element within a
// group of the native vector layout, and its local coordinates in its aggregate (8 bits each)
struct SiteRef {
    int ns;
    uint32_t vo;
    uint32_t lc;
};

template <typename Tq>
__device__ inline SiteRef site_ref(const CoarseArgs<Tq> &a, int i, int ls)
{
    SiteRef r;
    r.ns = a.agg_sites[(size_t)i * a.Va + ls];
    const int blk = r.ns / a.g.Vb, off = r.ns - blk * a.g.Vb;
    r.vo = (uint32_t)(blk * 24) * (uint32_t)(a.g.Vb * a.g.S) + (uint32_t)(off * a.g.S);
    uint32_t p = 0;
    int q = ls;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        p |= (uint32_t)(q % a.a[mu]) << (8 * mu);
        q /= a.a[mu];
    }
    r.lc = p;
    return r;
}

// spin half HP of column k' of P at a site: q_k' masked to that half (the half is a template
// parameter so that the masked spinor stays in registers); qk points at q_k's group and lane
template <int HP, typename Tc, typename Tq>
__device__ inline void load_half(const Tq *__restrict__ qk, uint32_t vo, uint32_t cs, Spinor<Tc> &s)
{
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        if (c / 6 == HP) {
            s.re[c] = load_as<Tc>(qk + vo + (2 * c) * cs);
            s.im[c] = load_as<Tc>(qk + vo + (2 * c + 1) * cs);
        } else {
            s.re[c] = s.im[c] = Tc(0);
        }
    }
}

// w += the forward hop in direction MU when the neighbour x + mu lies in the same aggregate
template <int MU, int HP, typename Tc, typename Tq>
__device__ inline void inside_fwd_hop(const CoarseArgs<Tq> &a, const Tc *__restrict__ links, const SiteRef *tab,
                                      const SiteRef &me, int ls, const Tq *qk, uint32_t cs, Spinor<Tc> &w)
{
    const int l = unpack_coord(me.lc, MU);
    if (l + 1 < a.a[MU]) {
        const SiteRef n = tab[ls + a.astr[MU]];
        Spinor<Tc> chi;
        load_half<HP, Tc>(qk, n.vo, cs, chi);
        Tc U[18];
        load_link(links, a.g.V, MU, me.ns, U);
        hop_accumulate<MU, -1, false>(U, chi, w);
    }
    hop_fence(w);
}

// local site of the f-th site on the +mu face of an aggregate (local coordinate mu = a_mu - 1)
__device__ inline int face_site(const int (&a)[4], const int (&astr)[4], int mu, int f)
{
    const int st = astr[mu];
    return f % st + st * (a[mu] - 1) + st * a[mu] * (f / st);
}

// column (HP, k') of half the self part at aggregate site ls: (A / 2 + the forward hops that
// stay inside) P_c.  The backward inside hops are g5 (forward hops)^dag g5 and A is
// Hermitian and commutes with g5, so with G = Q^dag (A/2 + forward inside hops) P the self
// block is G + sigma3 G^dag sigma3 (g5 P = P sigma3).
template <int HP, typename Tc, typename Tq>
__device__ inline void self_column(const CoarseArgs<Tq> &a, const Tc *__restrict__ links, const Tc *__restrict__ clover,
                                   const SiteRef *tab, int ls, const Tq *qk, uint32_t cs, Spinor<Tc> &w)
{
    const SiteRef me = tab[ls];
    Spinor<Tc> p;
    load_half<HP, Tc>(qk, me.vo, cs, p);
    // the site term is block-diagonal in the spin halves: only half HP is non-zero
    spinor_zero(w);
    {
        Tc A[36];
        load_clover_half<HP>(clover, a.g.V, me.ns, A);
        clover_half<HP>(A, p, w);
    }
#pragma unroll
    for (int c = 6 * HP; c < 6 * HP + 6; ++c) {
        w.re[c] *= Tc(0.5);
        w.im[c] *= Tc(0.5);
    }
    hop_fence(w);
    inside_fwd_hop<0, HP>(a, links, tab, me, ls, qk, cs, w);
    inside_fwd_hop<1, HP>(a, links, tab, me, ls, qk, cs, w);
    inside_fwd_hop<2, HP>(a, links, tab, me, ls, qk, cs, w);
    inside_fwd_hop<3, HP>(a, links, tab, me, ls, qk, cs, w);
}

// column (HP, k') of the +MU face part at face site f: (1 - g_mu) W_mu P_c(x + mu), the
// neighbour x + mu in aggregate i + mu
template <int MU, int HP, typename Tc, typename Tq>
__device__ inline void face_column(const CoarseArgs<Tq> &a, const Tc *__restrict__ links, const SiteRef &me,
                                   const SiteRef &nb, const Tq *qk, uint32_t cs, Spinor<Tc> &w)
{
    Spinor<Tc> chi;
    load_half<HP, Tc>(qk, nb.vo, cs, chi);
    Tc U[18];
    load_link(links, a.g.V, MU, me.ns, U);
    spinor_zero(w);
    hop_accumulate<MU, -1, false>(U, chi, w);
}

template <int HP, typename Tc, typename Tq>
__device__ inline void part_column(const CoarseArgs<Tq> &a, const Tc *__restrict__ links, const Tc *__restrict__ clover,
                                   int d, const SiteRef *tab, int sidx, int ls, const Tq *qk, uint32_t cs, Spinor<Tc> &w)
{
    switch (d) {
    case 0: self_column<HP>(a, links, clover, tab, ls, qk, cs, w); break;
    case 1: face_column<0, HP>(a, links, tab[sidx], tab[MAXVA + sidx], qk, cs, w); break;
    case 2: face_column<1, HP>(a, links, tab[sidx], tab[MAXVA + sidx], qk, cs, w); break;
    case 3: face_column<2, HP>(a, links, tab[sidx], tab[MAXVA + sidx], qk, cs, w); break;
    default: face_column<3, HP>(a, links, tab[sidx], tab[MAXVA + sidx], qk, cs, w); break;
    }
}

// grid: 5 items per aggregate (self, then +mu).  A 2N x 2N block is a sum over the
// block's sites and the 6 components of each spin half: rows (h, k) = conj(q_k) of half h,
// columns c = (h', k') the stencil part d applied to P_c.  Both are formed a chunk of CHS
// sites at a time in LDS (the columns by one thread per (h', site, k')); the
// products run on v_mfma_f32_16x16x4f32: the block is cut into 16x16 tiles (per half:
// ceil(N/16) x ceil(2N/16)), the wavefronts take tiles round-robin, a K step is 4 of the
// (site, component) rows, and complex = 4 real products.  Lane l supplies
// A[l%16][l/16] = conj(q)[row][kk] and B[l/16][l%16] = w[kk][col], holds D[4(l/16)+r][l%16].
// The sites the workgroup touches are looked up once into an LDS table (native index,
// vector offset, local coordinates), so the per-item work has no integer division.  The
// rows of the next chunk are loaded during the products of the current one, and the
// (aggregate, part) items are taken in contiguous runs per XCD, so that concurrent
// workgroups of one XCD read neighbouring aggregates (the face parts' neighbours) through
// the same L2, and the vector-unit-heavy self parts share CUs with the latency-bound faces.
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ inline f4 mfma32(float x, float y, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(x, y, c, 0, 0, 0); }

// the K steps of one chunk for the wavefront's first NTL tiles: conj(q) w accumulated as four
// real products per complex one, straight-line so that the LDS reads of later steps are in
// flight during the products of earlier ones
template <int NTL>
__device__ inline void tile_products(const float2 *const (&qb)[2], const float2 *const (&wb)[2], f4 (&accr)[2],
                                     f4 (&acci)[2])
{
#pragma unroll
    for (int kk0 = 0; kk0 < CHS * 6; kk0 += 4) {
#pragma unroll
        for (int m = 0; m < NTL; ++m) {
            const float2 q = qb[m][kk0 * QST], w = wb[m][kk0 * WST];
            accr[m] = mfma32(q.x, w.x, accr[m]);
            acci[m] = mfma32(q.x, w.y, acci[m]);
            accr[m] = mfma32(q.y, w.y, accr[m]);
            acci[m] = mfma32(-q.y, w.x, acci[m]);
        }
    }
}

template <typename Tc, typename Tq>
__global__ void __launch_bounds__(NTHR) k_coarse(CoarseArgs<Tq> a, const Tc *__restrict__ links,
                                                 const Tc *__restrict__ clover)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int N = a.N, N2 = 2 * N;
    // Qs and Ws rows are (half, site, component within the half): the K rows of one half are
    // contiguous.  The strides are those of 32 vectors plus one pair (the four rows a
    // matrix-core step reads fall on different LDS banks), so every product read has a fixed
    // offset; entries beyond N (2N) are never written and only reach output rows (columns)
    // that are not stored.
    SiteRef *tab = reinterpret_cast<SiteRef *>(smem);  // [MAXVA] own sites, [MAXFACE] face neighbours
    float2 *Qs = reinterpret_cast<float2 *>(tab + MAXVA + MAXFACE);  // [2][CHS][6][QST]
    float2 *Ws = Qs + CHS * 12 * QST;                               // [2][CHS][6][WST]
    // work item li = 5 i + d: aggregate i, part d (0: the self block; 1 + mu: the +mu face
    // block), so that the five parts of an aggregate are consecutive and a CU runs self and
    // face workgroups side by side; items in contiguous runs per XCD.  A grid of a few waves of
    // resident workgroups takes the parts one after the other instead (the self blocks, the
    // longest items, start first and do not end up as the tail), aggregates in XCD runs.
    int i, d;
    if (a.part_major) {
        d = blockIdx.x / a.n_agg;
        i = xcd_remap(blockIdx.x - d * a.n_agg, a.n_agg);
    } else {
        const int li = xcd_remap(blockIdx.x, gridDim.x);
        i = li / 5;
        d = li - 5 * i;
    }
    const bool self = d == 0;
    const int mu = d - 1;
    const int nsites = self ? a.Va : a.Va / a.a[mu];
    int j = i;  // the aggregate across the +mu face
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int TR = (N + 15) / 16, TC = (N2 + 15) / 16, ntile = 2 * TR * TC;
    constexpr int MAXT = (16 + NW - 1) / NW;  // tiles per wavefront (N <= 32: at most 16 tiles)
    static_assert(MAXT == 2, "the product loop takes two tiles per wavefront");
    f4 accr[MAXT], acci[MAXT];
#pragma unroll
    for (int m = 0; m < MAXT; ++m) accr[m] = acci[m] = f4{0.f, 0.f, 0.f, 0.f};

    // site table: self -- every site of aggregate i by local index; face -- the face sites
    // in face order and their +mu neighbours in aggregate i + mu
    if (self) {
        for (int ls = threadIdx.x; ls < a.Va; ls += blockDim.x) tab[ls] = site_ref(a, i, ls);
    } else {
        int c[4], r = i;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            c[m] = r % a.na[m];
            r /= a.na[m];
        }
        c[mu] = (c[mu] + 1) % a.na[mu];
        j = c[0] + a.na[0] * (c[1] + a.na[1] * (c[2] + a.na[2] * c[3]));
        for (int f = threadIdx.x; f < nsites; f += blockDim.x) {
            const int ls = face_site(a.a, a.astr, mu, f);
            tab[f] = site_ref(a, i, ls);
            tab[MAXVA + f] = site_ref(a, j, ls - (a.a[mu] - 1) * a.astr[mu]);
        }
    }
    // this thread's test vector k (fixed) and its slot among the rows it serves
    const int kt = threadIdx.x % N, rows_per_pass = NTHR / N, prow = threadIdx.x / N;
    const Tq *qk = a.Q + (size_t)(kt >> a.sshift) * a.gsz + (kt & ((1 << a.sshift) - 1));
    const uint32_t cs = (uint32_t)(a.g.Vb * a.g.S);

    // rows: q_k at (site, component) of a chunk, one (site, component) row per thread and pass.
    // The next chunk's rows are loaded into registers before the products of the current one
    // and stored to LDS after them; a row outside the set reads site 0 and is stored as zero.
    float2 rv[RMAX];
    uint32_t rok = 0;
    const auto load_rows = [&](int s0) {
        rok = 0;
#pragma unroll
        for (int it = 0; it < RMAX; ++it) {
            const int rw = prow + it * rows_per_pass, sl = rw / 12, comp = rw - sl * 12, sidx = s0 + sl;
            const bool ok = prow < rows_per_pass && rw < CHS * 12 && sidx < nsites;
            const uint32_t vo = tab[ok ? sidx : 0].vo;
            const int cc = ok ? comp : 0;
            rv[it] = make_float2(load_as<float>(qk + vo + (2 * cc) * cs), load_as<float>(qk + vo + (2 * cc + 1) * cs));
            rok |= (uint32_t)ok << it;
        }
    };
    __syncthreads();  // the site table
    load_rows(0);

    for (int s0 = 0; s0 < nsites; s0 += CHS) {
        __syncthreads();
#pragma unroll
        for (int it = 0; it < RMAX; ++it) {
            const int rw = prow + it * rows_per_pass, sl = rw / 12, comp = rw - sl * 12;
            if (prow < rows_per_pass && rw < CHS * 12)
                Qs[((comp >= 6 ? CHS * 6 : 0) + sl * 6 + comp % 6) * QST + kt] =
                    (rok >> it) & 1u ? rv[it] : make_float2(0.f, 0.f);
        }
        if (prow < rows_per_pass) {
            // columns: (h', site) pairs, k' = kt; h' outermost, so that a wavefront mostly
            // shares one spin half
            for (int pr = prow; pr < 2 * CHS; pr += rows_per_pass) {
                const int hp = pr / CHS, sl = pr - hp * CHS, sidx = s0 + sl;
                Spinor<Tc> w;
                if (sidx < nsites) {
                    const int ls = self ? sidx : 0;
                    if (hp == 0) part_column<0>(a, links, clover, d, tab, sidx, ls, qk, cs, w);
                    else part_column<1>(a, links, clover, d, tab, sidx, ls, qk, cs, w);
                } else {
                    spinor_zero(w);
                }
                const int c = hp * N + kt;
#pragma unroll
                for (int comp = 0; comp < 12; ++comp)
                    Ws[((comp / 6) * CHS * 6 + sl * 6 + comp % 6) * WST + c] =
                        make_float2((float)w.re[comp], (float)w.im[comp]);
            }
        }
        __syncthreads();
        if (s0 + CHS < nsites) load_rows(s0 + CHS);
        // the wavefront's tiles in one K loop: four independent accumulator chains; K row kk of
        // half h is LDS row h CHS 6 + kk
        const float2 *qb[MAXT], *wb[MAXT];
#pragma unroll
        for (int m = 0; m < MAXT; ++m) {
            const int tile = std::min(wave + NW * m, ntile - 1);
            const int h = tile / (TR * TC), rem = tile - h * TR * TC, tr = rem / TC, tc = rem - tr * TC;
            const int r0 = h * CHS * 6 + (lane >> 4);
            qb[m] = Qs + r0 * QST + tr * 16 + (lane & 15);  // A: conj(q) rows k of the half
            wb[m] = Ws + r0 * WST + tc * 16 + (lane & 15);  // B: columns c
        }
        if (wave + NW < ntile) tile_products<2>(qb, wb, accr, acci);
        else if (wave < ntile) tile_products<1>(qb, wb, accr, acci);
    }
    // D_c(i, i) or D_c(i, i + mu); for a face also D_c(i + mu, i) = sigma3 D_c(i, i + mu)^dag sigma3
    // into the -mu slot of aggregate j = i + mu (each slot has exactly one writer)
    const size_t ob = ((size_t)i * 9 + d) * N2 * N2 * 2, bb = ((size_t)j * 9 + 5 + mu) * N2 * N2 * 2;
    auto put = [&](size_t e, float v) {
        if (a.Dc16) a.Dc16[e] = __float2half_rn(v);
        else a.Dc[e] = v;
    };
    if (self) {
        // D_c(i, i) = G + sigma3 G^dag sigma3: G through LDS (over the chunk buffers, free once
        // every wavefront has finished its last products), then written row by row
        const int GST = N2 + 1;
        float2 *Gs = Qs;
        __syncthreads();
#pragma unroll
        for (int m = 0; m < MAXT; ++m) {
            const int tile = wave + NW * m;
            if (tile >= ntile) break;
            const int h = tile / (TR * TC), rem = tile - h * TR * TC, tr = rem / TC, tc = rem - tr * TC;
            const int c = tc * 16 + (lane & 15);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int k = tr * 16 + 4 * (lane >> 4) + r;
                if (k < N && c < N2) Gs[(h * N + k) * GST + c] = make_float2(accr[m][r], acci[m][r]);
            }
        }
        __syncthreads();
        for (int e = threadIdx.x; e < N2 * N2; e += NTHR) {
            const int row = e / N2, c = e - row * N2;
            const float2 g = Gs[row * GST + c], t = Gs[c * GST + row];
            const float sg = ((row < N) == (c < N)) ? 1.f : -1.f;
            put(ob + 2 * (size_t)e, g.x + sg * t.x);
            put(ob + 2 * (size_t)e + 1, g.y - sg * t.y);
        }
        return;
    }
#pragma unroll
    for (int m = 0; m < MAXT; ++m) {
        const int tile = wave + NW * m;
        if (tile >= ntile) break;
        const int h = tile / (TR * TC), rem = tile - h * TR * TC, tr = rem / TC, tc = rem - tr * TC;
        const int c = tc * 16 + (lane & 15);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int k = tr * 16 + 4 * (lane >> 4) + r;
            if (k < N && c < N2) {
                const int row = h * N + k;
                const size_t e = (size_t)row * N2 + c;
                put(ob + 2 * e, accr[m][r]);
                put(ob + 2 * e + 1, acci[m][r]);
                if (!self) {
                    const float sg = ((row < N) == (c < N)) ? 1.f : -1.f;
                    const size_t t = (size_t)c * N2 + row;
                    put(bb + 2 * t, sg * accr[m][r]);
                    put(bb + 2 * t + 1, -sg * acci[m][r]);
                }
            }
        }
    }
}

template <typename Tc, typename Tq>
int coarse_dispatch(const mrhs_op *op, const Tc *links, const Tc *clover, const Tq *Q, int n_tv, void *Dc, bool f16,
                    hipStream_t st)
{
    CoarseArgs<Tq> a{};
    a.g = op->k;
    int s = 1;
    for (int mu = 0; mu < 4; ++mu) {
        a.a[mu] = op->g.agg[mu];
        a.na[mu] = op->na[mu];
        a.astr[mu] = s;
        s *= op->g.agg[mu];
    }
    a.Va = op->Va;
    a.n_agg = op->n_agg;
    a.N = n_tv;
    a.sshift = 0;
    while ((1 << a.sshift) < op->k.S) ++a.sshift;
    a.gsz = (long)op->k.nblk * 24 * op->k.Vb * op->k.S;
    // up to about eight waves of resident workgroups (two per CU): part by part
    a.part_major = op->n_agg * 5 <= 4096;
    a.agg_sites = op->agg_sites;
    a.blk_coords = op->blk_coords;
    a.loc_coords = op->loc_coords;
    a.Q = Q;
    a.Dc = f16 ? nullptr : (float *)Dc;
    a.Dc16 = f16 ? (__half *)Dc : nullptr;
    if (!a.Q || !Dc || !a.agg_sites || !a.blk_coords || !a.loc_coords || !links || !clover)
        return set_error(MRHS_EINVAL, "coarse_op_build: missing buffer");
    if (op->Va > MAXVA) return set_error(MRHS_EUNSUPPORTED, "coarse_op_build: aggregate volume above 256");
    for (int mu = 0; mu < 4; ++mu)
        if (op->Va / op->g.agg[mu] > MAXFACE)
            return set_error(MRHS_EUNSUPPORTED, "coarse_op_build: aggregate face above 64 sites");
    const size_t lds = sizeof(SiteRef) * (MAXVA + MAXFACE) + sizeof(float2) * (size_t)CHS * 12 * (QST + WST);
    hipLaunchKernelGGL((k_coarse<Tc, Tq>), dim3(op->n_agg * 5), dim3(NTHR), lds, st, a, links, clover);
    return hip_check(hipGetLastError(), "k_coarse launch");
}

}  // namespace

size_t ws_bytes_coarse(const mrhs_op *, int) { return 0; }

int launch_coarse(const mrhs_op *op, const void *Q, int qdt, int n_tv, void *Dc, int dcdt, hipStream_t st)
{
    const bool f16 = dcdt == MRHS_DTYPE_F16;
    if (2 * n_tv * 2 * n_tv > 16 * NTHR) return set_error(MRHS_EUNSUPPORTED, "more than 32 test vectors");
    if (op->links32) {
        if (qdt == MRHS_DTYPE_F32)
            return coarse_dispatch<float, float>(op, op->links32, op->clover32, (const float *)Q, n_tv, Dc, f16, st);
        if (qdt == MRHS_DTYPE_F16)
            return coarse_dispatch<float, __half>(op, op->links32, op->clover32, (const __half *)Q, n_tv, Dc, f16, st);
        return coarse_dispatch<float, double>(op, op->links32, op->clover32, (const double *)Q, n_tv, Dc, f16, st);
    }
    if (qdt == MRHS_DTYPE_F32)
        return coarse_dispatch<double, float>(op, op->links64, op->clover64, (const float *)Q, n_tv, Dc, f16, st);
    if (qdt == MRHS_DTYPE_F16)
        return coarse_dispatch<double, __half>(op, op->links64, op->clover64, (const __half *)Q, n_tv, Dc, f16, st);
    return coarse_dispatch<double, double>(op, op->links64, op->clover64, (const double *)Q, n_tv, Dc, f16, st);
}
