// sap.hip -- the Schwarz alternating procedure on all right-hand sides at once.
//
// One launch per colour half-sweep, for one operator or a batch of several (lattices of
// uneven size, each with its own right-hand sides).  Workgroup = one SAP block of that
// colour x a tile of T right-hand sides; thread (off, t) owns one site of the block and
// one right-hand side.  The workgroup
//   1. forms the residual r = b - D x on its block (full stencil, neighbours from global
//      memory; skipped where x is known to be zero),
//   2. runs n_mr minimal-residual steps on the block operator D_j = I_j^T D I_j with the
//      block residual rho kept in LDS ([24][Vb][T], conflict-free for the thread order),
//      the two inner products per step reduced across the block with wavefront shuffles
//      and one LDS exchange, and the correction e kept in registers,
//   3. writes x|_j (+)= e.
// The links and clover of a site are loaded once per stencil for all T lanes of the site.
// With the even-odd block solver (k_sap_batched_eo) step 2 runs on the block's Schur
// complement over its even sites instead (sap_block_eo).
#include <algorithm>

#include "launch.h"
#include "stencil.h"

#include <type_traits>

namespace {

template <typename Ts, typename Tc> struct SapArgs {
    KGeo g;
    const Tc *links, *clover;
    const uint32_t *blk_coords, *loc_coords;
    const int32_t *blocks;  // block ids of this colour
    int nblocks;            // number of blocks of this colour
    int ntiles;             // right-hand-side tiles per block
    int colour;
    int mode;               // 0: x = 0 everywhere; 1: x = 0 on this colour's blocks; 2: general
    int n_mr;
    const Ts *b;
    const Ts *xr;           // where neighbours' x is read (x itself, or a snapshot)
    Ts *x;
    // sigma = b - D_j x_j per block, kept between the visits of a colour (arithmetic type):
    // the residual of a later visit is sigma - (hops across the block's faces)
    Tc *sig;
    int sig_in;             // this colour's sigma is valid (read it instead of forming b - D x)
    int sig_out;            // write sigma for the next visit of this colour
    // incremental residual (no block has a neighbour of its own colour): sig holds the block's
    // residual rho after its last visit, ecor each block's last change of x; a later visit's
    // residual is rho - (face hops of the neighbours' changes since then), the change the
    // other colour made in between
    int inc;
    Tc *ecor;
    int e_out;              // write this visit's change of x (a later visit reads it)
    // even-odd block solver: A^-1 per site (clover layout), block offsets in parity order,
    // number of even sites of a block
    const Tc *cloverinv;
    const int32_t *eo_sites;
    int Ve;
};

// The block residual rho lives in LDS as (re, im) pairs, [12][Vb][T]: lane (off, t)
// reads component c at (c * Vb + off) * T + t, consecutive lanes consecutive pairs.
template <typename Tc> struct LdsPair;
template <> struct LdsPair<float> { using type = float2; };
template <> struct LdsPair<double> { using type = double2; };

template <typename Tc>
__device__ inline void lds_load(const typename LdsPair<Tc>::type *rho, int str, int idx, Spinor<Tc> &s)
{
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        const auto v = rho[c * str + idx];
        s.re[c] = v.x;
        s.im[c] = v.y;
    }
}

// components 6 HF .. 6 HF + 5 (one chiral half) only
template <int HF, typename Tc>
__device__ inline void lds_load_half(const typename LdsPair<Tc>::type *rho, int str, int idx, Spinor<Tc> &s)
{
#pragma unroll
    for (int c = 6 * HF; c < 6 * HF + 6; ++c) {
        const auto v = rho[c * str + idx];
        s.re[c] = v.x;
        s.im[c] = v.y;
    }
}

template <typename Tc>
__device__ inline void lds_store(typename LdsPair<Tc>::type *rho, int str, int idx, const Spinor<Tc> &s)
{
#pragma unroll
    for (int c = 0; c < 12; ++c) rho[c * str + idx] = {s.re[c], s.im[c]};
}

// The links a block operator uses, staged in LDS once per workgroup (the "links in LDS"
// variant, for the tile of four right-hand sides): U_mu(x) for the block's sites x whose
// +mu neighbour is inside the block (local coordinate l_mu < b_mu - 1; every site when the
// block spans the lattice in mu and keeps its wrap-around hop).  Per direction they form a
// box of extents e_mu,nu = b_nu, except e_mu,mu = b_mu - 1, stored lexicographically after
// the boxes of the lower directions, 18 reals per link.
struct LinkBox {
    int base[4];  // first link of direction mu
    int s[4][4];  // lexicographic strides of direction mu's box
    int n;        // links in all four boxes
};

__host__ __device__ inline LinkBox link_box(const KGeo &g)
{
    LinkBox lb;
    int base = 0;
    for (int mu = 0; mu < 4; ++mu) {
        int st = 1;
        for (int nu = 0; nu < 4; ++nu) {
            lb.s[mu][nu] = st;
            st *= (nu == mu && g.nb[mu] > 1) ? g.b[nu] - 1 : g.b[nu];
        }
        lb.base[mu] = base;
        base += st;
    }
    lb.n = base;
    return lb;
}

template <typename Tf, typename T> __device__ inline void lds_link(const Tf *ul, int idx, T (&U)[18])
{
    using V2 = typename Vec2<Tf>::type;
    const V2 *p = reinterpret_cast<const V2 *>(ul + idx * 18);
#pragma unroll
    for (int c = 0; c < 9; ++c) {
        const V2 v = p[c];
        U[2 * c] = (T)v.x;
        U[2 * c + 1] = (T)v.y;
    }
}

// q += hops of D_j rho at site off (lane t), rho from LDS; hops leaving the block dropped.
// ns is the site's native index (opaque to the compiler, so the link loads stay inside
// the MR loop).  With ul (links in LDS) the links come from there: cf is the site's index
// in direction MU's box, sb the box's stride in MU.
template <int MU, typename Tc, bool LL = false>
__device__ inline void block_hops(const KGeo &g, const Tc *__restrict__ links, const typename LdsPair<Tc>::type *rho,
                                  int T, int ns, int off, int t, uint32_t lcp, Spinor<Tc> &q,
                                  const Tc *ul = nullptr, int cf = 0, int sb = 0)
{
    const int str = g.Vb * T;
    const int l = unpack_coord(lcp, MU);
    int noff = -1;
    if (l + 1 < g.b[MU]) noff = off + g.ostr[MU];
    else if (g.nb[MU] == 1) noff = off - (g.b[MU] - 1) * g.ostr[MU];
    if (noff >= 0) {
        Spinor<Tc> chi;
        lds_load<Tc>(rho, str, noff * T + t, chi);
        Tc U[18];
        if constexpr (LL) lds_link(ul, cf, U);
        else load_link(links, g.V, MU, ns, U);
        hop_accumulate<MU, -1, false>(U, chi, q);
    }
    hop_fence(q);
    noff = -1;
    int cb = 0;
    if (l > 0) {
        noff = off - g.ostr[MU];
        cb = cf - sb;
    } else if (g.nb[MU] == 1) {
        noff = off + (g.b[MU] - 1) * g.ostr[MU];
        cb = cf + (g.b[MU] - 1) * sb;
    }
    if (noff >= 0) {
        Spinor<Tc> chi;
        lds_load<Tc>(rho, str, noff * T + t, chi);
        Tc U[18];
        if constexpr (LL) lds_link(ul, cb, U);
        else load_link(links, g.V, MU, ns + (noff - off), U);
        hop_accumulate<MU, +1, true>(U, chi, q);
    }
}

// words of LDS for the reduction scratch of a workgroup: [waves][T][3], rounded to 4
__host__ __device__ inline int red_words(int threads, int T) { return ((threads / 64) * T * 3 + 3) / 4 * 4; }

// One workgroup's share of a half-sweep: block blk, right-hand-side tile `tile`.  LL: the
// block's links are staged in LDS (after rho and the reduction scratch) for the MR steps.
template <typename Ts, typename Tc, int T, bool LL>
__device__ inline void sap_block(const SapArgs<Ts, Tc> &a, int blk, int tile, unsigned char *smem)
{
    using P2 = typename LdsPair<Tc>::type;
    const KGeo &g = a.g;
    P2 *rho = reinterpret_cast<P2 *>(smem);
    const int str = g.Vb * T;
    Tc *red_s = reinterpret_cast<Tc *>(rho + 12 * str);  // [waves][T][3]
    Tc *ul = red_s + red_words(blockDim.x, T);  // used only with LL

    const int off = threadIdx.x / T, t = threadIdx.x % T;
    const bool active = off < g.Vb;
    const int grp = (tile * T) / g.S, tt = (tile * T) % g.S + t;  // T divides S: grp is uniform
    const int me = off * T + t;                                   // this lane's LDS slot
    int bc[4] = {0, 0, 0, 0}, lc[4] = {0, 0, 0, 0};
    if (active) decode_site(g, a.blk_coords, a.loc_coords, blk, off, bc, lc);
    const uint32_t lcp = active ? a.loc_coords[off] : 0u;  // local coordinates, 8 bits each
    // links in LDS: this site's index in each direction's box; the T lanes of a site copy
    // its four forward links (lane t: directions t, t + T, ...)
    int cf[4] = {0, 0, 0, 0}, sb[4] = {0, 0, 0, 0};
    if (LL) {
        const LinkBox lb = link_box(g);
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
            cf[mu] = lb.base[mu] + lc[0] * lb.s[mu][0] + lc[1] * lb.s[mu][1] + lc[2] * lb.s[mu][2] + lc[3] * lb.s[mu][3];
            sb[mu] = lb.s[mu][mu];
        }
        if (active) {
            using V2 = typename Vec2<Tc>::type;
            for (int mu = t; mu < 4; mu += T) {
                if (lc[mu] + 1 < g.b[mu] || g.nb[mu] == 1) {
                    const V2 *src = reinterpret_cast<const V2 *>(a.links + ((size_t)(blk * g.Vb + off) * 4 + mu) * 18);
                    V2 *dst = reinterpret_cast<V2 *>(ul + cf[mu] * 18);
#pragma unroll
                    for (int c = 0; c < 9; ++c) dst[c] = src[c];
                }
            }
        }
    }

    // 1. residual on the block: b - D x, or sigma - (face hops) once sigma is known
    const int colour = a.colour, mode = a.mode;
    const uint32_t *bcs = a.blk_coords;
    auto skip = [=](int nblk) { return mode == 1 && block_colour(g, bcs, nblk) == colour; };
    // The face hops F of this visit (what the other blocks' x contribute) are what sigma for the
    // next visit needs as well (sigma' = rho + F, step 4): where step 1 forms them on their own
    // (a sigma visit, or the first visit of the second colour, where x vanishes on the block so
    // that D x is F), they are kept in this site's sigma slot until step 4.
    const bool keep_f = !a.inc && a.sig_out && (a.sig_in || a.mode == 1);
    if (active) {
        Spinor<Tc> r;
        if (a.mode != 0) {
            Spinor<Tc> bb;
            if constexpr (std::is_same<Ts, Tc>::value) {
                // a visit that knows sigma, and the first visit of the second colour (x vanishes on
                // the block, so D x is its face hops), through one call of the face hops
                if (a.sig_in || a.mode == 1) {
                    spinor_zero(r);
                    const Tc *src = a.sig_in && a.inc ? (const Tc *)a.ecor : a.xr;
                    face_hops_global<Tc>(g, a.links, src, grp, tt, blk, off, bc, lc, r, skip);
                    load_spinor<Tc>(g, a.sig_in ? (const Tc *)a.sig : a.b, grp, blk, off, tt, bb);
                } else {
                    dirac_site_global<Tc>(g, a.links, a.clover, a.xr, grp, tt, blk, off, bc, lc, r, skip);
                    load_spinor<Tc>(g, a.b, grp, blk, off, tt, bb);
                }
            } else if (a.sig_in) {
                spinor_zero(r);
                if (a.inc) face_hops_global<Tc>(g, a.links, (const Tc *)a.ecor, grp, tt, blk, off, bc, lc, r, skip);
                else face_hops_global<Tc>(g, a.links, a.xr, grp, tt, blk, off, bc, lc, r, skip);
                load_spinor<Tc>(g, a.sig, grp, blk, off, tt, bb);
            } else {
                dirac_site_global<Tc>(g, a.links, a.clover, a.xr, grp, tt, blk, off, bc, lc, r, skip);
                load_spinor<Tc>(g, a.b, grp, blk, off, tt, bb);
            }
            if (keep_f) store_spinor(g, a.sig, grp, blk, off, tt, r);
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                r.re[c] = bb.re[c] - r.re[c];
                r.im[c] = bb.im[c] - r.im[c];
            }
        } else {
            load_spinor<Tc>(g, a.b, grp, blk, off, tt, r);
        }
        lds_store<Tc>(rho, str, me, r);
    }

    // 2. minimal residual on the block operator
    Spinor<Tc> e;
    spinor_zero(e);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
    for (int it = 0; it < a.n_mr; ++it) {
        __syncthreads();
        Spinor<Tc> q;
        Tc qq = 0, qrr = 0, qri = 0;
        if (active) {
            // the site index is hidden from the compiler so that the block's fields are
            // re-read from cache in every step instead of held in registers across the loop
            const int ns = opaque_index(blk * g.Vb + off);
            // the clover term one chiral half at a time (it is block-diagonal in them): six
            // components of rho and 36 field values live instead of twelve and 72
            auto clover_term = [&](auto add) {
                {
                    Spinor<Tc> own;
                    Tc A[36];
                    lds_load_half<0, Tc>(rho, str, me, own);
                    load_clover_half<0>(a.clover, g.V, ns, A);
                    clover_half<0, decltype(add)::value>(A, own, q);
                }
                hop_fence(q);
                {
                    Spinor<Tc> own;
                    Tc A[36];
                    lds_load_half<1, Tc>(rho, str, me, own);
                    load_clover_half<1>(a.clover, g.V, ns, A);
                    clover_half<1, decltype(add)::value>(A, own, q);
                }
                hop_fence(q);
            };
            // (the LDS link indices are hidden like ns: the links are re-read in every step)
            auto hops = [&]() {
                block_hops<0, Tc, LL>(g, a.links, rho, T, ns, off, t, lcp, q, ul, LL ? opaque_index(cf[0]) : 0, sb[0]);
                hop_fence(q);
                block_hops<1, Tc, LL>(g, a.links, rho, T, ns, off, t, lcp, q, ul, LL ? opaque_index(cf[1]) : 0, sb[1]);
                hop_fence(q);
                block_hops<2, Tc, LL>(g, a.links, rho, T, ns, off, t, lcp, q, ul, LL ? opaque_index(cf[2]) : 0, sb[2]);
                hop_fence(q);
                block_hops<3, Tc, LL>(g, a.links, rho, T, ns, off, t, lcp, q, ul, LL ? opaque_index(cf[3]) : 0, sb[3]);
                hop_fence(q);
            };
            // Every wavefront starts the step together after the barrier; the clover term is read
            // from global memory, the hops from LDS.  Wavefronts 4-7 and 12-15 take the hops
            // first and add the clover term last, so that some wavefronts compute while the
            // others wait for the clover field (with the wavefronts placed on the four SIMDs in
            // turn, each SIMD holds both kinds).
            if ((wave >> 2) & 1) {
                spinor_zero(q);
                hop_fence(q);
                hops();
                clover_term(std::true_type{});
            } else {
                clover_term(std::false_type{});
                hops();
            }
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                const P2 o = rho[c * str + me];
                qq += q.re[c] * q.re[c];
                qq += q.im[c] * q.im[c];
                qrr += q.re[c] * o.x;
                qrr += q.im[c] * o.y;
                qri += q.re[c] * o.y;
                qri -= q.im[c] * o.x;
            }
        } else {
            spinor_zero(q);
        }
        qq = wave_sum_stride(qq, T);
        qrr = wave_sum_stride(qrr, T);
        qri = wave_sum_stride(qri, T);
        if (lane < T) {
            red_s[(wave * T + lane) * 3 + 0] = qq;
            red_s[(wave * T + lane) * 3 + 1] = qrr;
            red_s[(wave * T + lane) * 3 + 2] = qri;
        }
        __syncthreads();
        Tc sqq = 0, sr = 0, si = 0;
        for (int w = 0; w < nwaves; ++w) {
            sqq += red_s[(w * T + t) * 3 + 0];
            sr += red_s[(w * T + t) * 3 + 1];
            si += red_s[(w * T + t) * 3 + 2];
        }
        const Tc ar = sqq > Tc(0) ? sr / sqq : Tc(0);
        const Tc ai = sqq > Tc(0) ? si / sqq : Tc(0);
        if (active) {
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                const P2 o = rho[c * str + me];
                e.re[c] += ar * o.x;
                e.re[c] -= ai * o.y;
                e.im[c] += ar * o.y;
                e.im[c] += ai * o.x;
                Tc nr = o.x, ni = o.y;
                nr -= ar * q.re[c];
                nr += ai * q.im[c];
                ni -= ar * q.im[c];
                ni -= ai * q.re[c];
                rho[c * str + me] = {nr, ni};
            }
        }
    }

    // 3. x|_j (+)= e; with the incremental residual also the change of the stored x (the
    //    correction as rounded to the storage type)
    if (active) {
        Spinor<Tc> xo;
        if (a.mode == 2) {
            load_spinor<Tc>(g, a.x, grp, blk, off, tt, xo);
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                e.re[c] += xo.re[c];
                e.im[c] += xo.im[c];
            }
        }
        store_spinor(g, a.x, grp, blk, off, tt, e);
        if (a.e_out) {
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                Ts sr = store_as<Ts>(e.re[c]), si = store_as<Ts>(e.im[c]);
                e.re[c] = load_as<Tc>(&sr);
                e.im[c] = load_as<Tc>(&si);
                if (a.mode == 2) {
                    e.re[c] -= xo.re[c];
                    e.im[c] -= xo.im[c];
                }
            }
            store_spinor(g, a.ecor, grp, blk, off, tt, e);
        }
    }
    // 4. sigma for the next visit: b - D_j x_j(new) = rho (the block residual after the MR
    //    steps, this lane's own LDS slot) + the face hops, which this half-sweep leaves unchanged
    //    (kept from step 1, or formed again after a full residual)
    if (active && a.sig_out && a.inc) {
        // the incremental residual keeps rho itself
        Spinor<Tc> rr;
        lds_load<Tc>(rho, str, me, rr);
        store_spinor(g, a.sig, grp, blk, off, tt, rr);
    } else if (active && a.sig_out) {
        Spinor<Tc> sg;
        if (keep_f) {
            load_spinor<Tc>(g, a.sig, grp, blk, off, tt, sg);
        } else if (a.mode != 0) {
            // the coordinates are decoded again rather than kept live through the MR steps
            int bc2[4], lc2[4];
            decode_site(g, a.blk_coords, a.loc_coords, blk, opaque_index(off), bc2, lc2);
            spinor_zero(sg);
            face_hops_global<Tc>(g, a.links, a.xr, grp, tt, blk, off, bc2, lc2, sg, skip);
        }
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            const P2 o = rho[c * str + me];
            if (a.mode != 0) {
                sg.re[c] += o.x;
                sg.im[c] += o.y;
            } else {
                sg.re[c] = o.x;
                sg.im[c] = o.y;
            }
        }
        store_spinor(g, a.sig, grp, blk, off, tt, sg);
    }
}

// The even-odd block solver (DD-alpha-AMG's): with a block's sites split by the parity of
// their block-local coordinate sum (every block extent even, so each hop inside the block
// joins opposite parities), D_j = A + H is solved through the Schur complement over the
// even sites, S = A_ee - H_eo A_oo^-1 H_oe:
//   rhat_e = r_e - H_eo A_oo^-1 r_o,  n_mr MR steps on S e_e = rhat_e,  e_o = A_oo^-1 (r_o - H_oe e_e).
// Threads take the block's sites in parity order (the even half first), so each phase runs
// on whole wavefronts of one parity.  LDS holds rho on the even sites; on the odd sites it
// holds -A_oo^-1 H_oe rho for the step in progress, so that the even sites' hops add
// -H_eo A_oo^-1 H_oe rho to A_ee rho directly.
template <typename Ts, typename Tc, int T>
__device__ inline void eo_hops(const SapArgs<Ts, Tc> &a, const typename LdsPair<Tc>::type *rho, int ns, int off, int t,
                               uint32_t lc, Spinor<Tc> &h)
{
    const KGeo &g = a.g;
    block_hops<0>(g, a.links, rho, T, ns, off, t, lc, h);
    hop_fence(h);
    block_hops<1>(g, a.links, rho, T, ns, off, t, lc, h);
    hop_fence(h);
    block_hops<2>(g, a.links, rho, T, ns, off, t, lc, h);
    hop_fence(h);
    block_hops<3>(g, a.links, rho, T, ns, off, t, lc, h);
    hop_fence(h);
}

template <typename Ts, typename Tc, int T>
__device__ inline void eo_residual(const SapArgs<Ts, Tc> &a, typename LdsPair<Tc>::type *rho, int blk, int off, int grp,
                                   int tt, int t)
{
    const KGeo &g = a.g;
    int bc[4], lc[4];
    decode_site(g, a.blk_coords, a.loc_coords, blk, off, bc, lc);
    Spinor<Tc> r;
    if (a.mode != 0) {
        const int colour = a.colour, mode = a.mode;
        const uint32_t *bcs = a.blk_coords;
        auto skip = [=](int nblk) { return mode == 1 && block_colour(g, bcs, nblk) == colour; };
        dirac_site_global<Tc>(g, a.links, a.clover, a.xr, grp, tt, blk, off, bc, lc, r, skip);
        Spinor<Tc> bb;
        load_spinor<Tc>(g, a.b, grp, blk, off, tt, bb);
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            r.re[c] = bb.re[c] - r.re[c];
            r.im[c] = bb.im[c] - r.im[c];
        }
    } else {
        load_spinor<Tc>(g, a.b, grp, blk, off, tt, r);
    }
    lds_store<Tc>(rho, g.Vb * T, off * T + t, r);
}

template <typename Ts, typename Tc, int T>
__device__ inline void eo_update_x(const SapArgs<Ts, Tc> &a, const typename LdsPair<Tc>::type *rho, int blk, int off,
                                   int grp, int tt, int t)
{
    const KGeo &g = a.g;
    Spinor<Tc> e;
    lds_load<Tc>(rho, g.Vb * T, off * T + t, e);
    if (a.mode == 2) {
        Spinor<Tc> xo;
        load_spinor<Tc>(g, a.x, grp, blk, off, tt, xo);
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            e.re[c] += xo.re[c];
            e.im[c] += xo.im[c];
        }
    }
    store_spinor(g, a.x, grp, blk, off, tt, e);
}

// The even-odd block solver (DD-alpha-AMG's): with a block's sites split by the parity of
// their block-local coordinate sum (every block extent even, so each hop inside the block
// joins opposite parities), D_j = A + H is solved through the Schur complement over the
// even sites, S = A_ee - H_eo A_oo^-1 H_oe:
//   rhat_e = r_e - H_eo A_oo^-1 r_o,  n_mr MR steps on S e_e = rhat_e,  e_o = A_oo^-1 (r_o - H_oe e_e).
// Each thread owns one even and one odd site of the block (the u-th of each, parity order),
// so the workgroup has Vb / 2 x T threads and all of them work in both phases of a step: the
// odd sites' hops and A^-1, then the even sites' clover and hops.  LDS holds rho on the even
// sites and -A_oo^-1 H_oe rho on the odd sites; the residual and the x update run in site
// order (sites u and u + Vb / 2) for coalesced vector access and go through LDS.
template <typename Ts, typename Tc, int T>
__device__ inline void sap_block_eo(const SapArgs<Ts, Tc> &a, int blk, int tile, unsigned char *smem)
{
    using P2 = typename LdsPair<Tc>::type;
    const KGeo &g = a.g;
    P2 *rho = reinterpret_cast<P2 *>(smem);
    const int str = g.Vb * T;
    Tc *red_s = reinterpret_cast<Tc *>(rho + 12 * str);  // [waves][T][3]

    const int u = threadIdx.x / T, t = threadIdx.x % T, Ve = a.Ve;
    const bool active = u < Ve;
    const int grp = (tile * T) / g.S, tt = (tile * T) % g.S + t;
    const int se = active ? a.eo_sites[u] : 0, so = active ? a.eo_sites[Ve + u] : 0;
    const int me = se * T + t, mo = so * T + t;
    // local coordinates of the even and the odd site, 8 bits each
    const uint32_t lce = active ? a.loc_coords[se] : 0u, lco = active ? a.loc_coords[so] : 0u;

    // 1. residual on the block (sites u and u + Ve in site order), to LDS
    if (active) {
        eo_residual<Ts, Tc, T>(a, rho, blk, u, grp, tt, t);
        eo_residual<Ts, Tc, T>(a, rho, blk, u + Ve, grp, tt, t);
    }
    __syncthreads();
    // 2. odd: eo = A_oo^-1 r_o (kept), -eo to LDS; even: rhat_e = r_e + H_eo (-eo)
    Spinor<Tc> ee, eo;
    spinor_zero(ee);
    spinor_zero(eo);
    if (active) {
        const int ns = blk * g.Vb + so;
        Spinor<Tc> r;
        lds_load<Tc>(rho, str, mo, r);
        clover_site(a.cloverinv, g.V, ns, r, eo);
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            r.re[c] = -eo.re[c];
            r.im[c] = -eo.im[c];
        }
        lds_store<Tc>(rho, str, mo, r);
    }
    __syncthreads();
    if (active) {
        const int ns = blk * g.Vb + se;
        Spinor<Tc> r;
        lds_load<Tc>(rho, str, me, r);
        eo_hops<Ts, Tc, T>(a, rho, ns, se, t, lce, r);
        lds_store<Tc>(rho, str, me, r);
    }

    // 3. minimal residual on S over the even sites
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
    for (int it = 0; it < a.n_mr; ++it) {
        __syncthreads();
        if (active) {
            // odd slots: -A_oo^-1 H_oe rho
            const int ns = opaque_index(blk * g.Vb + so);
            Spinor<Tc> h, w;
            spinor_zero(h);
            eo_hops<Ts, Tc, T>(a, rho, ns, so, t, lco, h);
            clover_site(a.cloverinv, g.V, ns, h, w);
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                w.re[c] = -w.re[c];
                w.im[c] = -w.im[c];
            }
            lds_store<Tc>(rho, str, mo, w);
        }
        __syncthreads();
        Spinor<Tc> q;
        Tc qq = 0, qrr = 0, qri = 0;
        if (active) {
            const int ns = opaque_index(blk * g.Vb + se);
            {
                Spinor<Tc> own;
                Tc A[36];
                lds_load_half<0, Tc>(rho, str, me, own);
                load_clover_half<0>(a.clover, g.V, ns, A);
                clover_half<0>(A, own, q);
            }
            hop_fence(q);
            {
                Spinor<Tc> own;
                Tc A[36];
                lds_load_half<1, Tc>(rho, str, me, own);
                load_clover_half<1>(a.clover, g.V, ns, A);
                clover_half<1>(A, own, q);
            }
            hop_fence(q);
            eo_hops<Ts, Tc, T>(a, rho, ns, se, t, lce, q);
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                const P2 o = rho[c * str + me];
                qq += q.re[c] * q.re[c];
                qq += q.im[c] * q.im[c];
                qrr += q.re[c] * o.x;
                qrr += q.im[c] * o.y;
                qri += q.re[c] * o.y;
                qri -= q.im[c] * o.x;
            }
        } else {
            spinor_zero(q);
        }
        qq = wave_sum_stride(qq, T);
        qrr = wave_sum_stride(qrr, T);
        qri = wave_sum_stride(qri, T);
        if (lane < T) {
            red_s[(wave * T + lane) * 3 + 0] = qq;
            red_s[(wave * T + lane) * 3 + 1] = qrr;
            red_s[(wave * T + lane) * 3 + 2] = qri;
        }
        __syncthreads();
        Tc sqq = 0, sr = 0, si = 0;
        for (int w = 0; w < nwaves; ++w) {
            sqq += red_s[(w * T + t) * 3 + 0];
            sr += red_s[(w * T + t) * 3 + 1];
            si += red_s[(w * T + t) * 3 + 2];
        }
        const Tc ar = sqq > Tc(0) ? sr / sqq : Tc(0);
        const Tc ai = sqq > Tc(0) ? si / sqq : Tc(0);
        if (active) {
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                const P2 o = rho[c * str + me];
                ee.re[c] += ar * o.x;
                ee.re[c] -= ai * o.y;
                ee.im[c] += ar * o.y;
                ee.im[c] += ai * o.x;
                Tc nr = o.x, ni = o.y;
                nr -= ar * q.re[c];
                nr += ai * q.im[c];
                ni -= ar * q.im[c];
                ni -= ai * q.re[c];
                rho[c * str + me] = {nr, ni};
            }
        }
    }

    // 4. odd: e_o = A_oo^-1 r_o + A_oo^-1 H_oe (-e_e)
    __syncthreads();
    if (active) {
        Spinor<Tc> m;
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            m.re[c] = -ee.re[c];
            m.im[c] = -ee.im[c];
        }
        lds_store<Tc>(rho, str, me, m);
    }
    __syncthreads();
    if (active) {
        const int ns = blk * g.Vb + so;
        Spinor<Tc> h, w;
        spinor_zero(h);
        eo_hops<Ts, Tc, T>(a, rho, ns, so, t, lco, h);
        clover_site(a.cloverinv, g.V, ns, h, w);
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            eo.re[c] += w.re[c];
            eo.im[c] += w.im[c];
        }
    }

    // 5. e to LDS, then x|_j (+)= e in site order
    __syncthreads();
    if (active) {
        lds_store<Tc>(rho, str, me, ee);
        lds_store<Tc>(rho, str, mo, eo);
    }
    __syncthreads();
    if (active) {
        eo_update_x<Ts, Tc, T>(a, rho, blk, u, grp, tt, t);
        eo_update_x<Ts, Tc, T>(a, rho, blk, u + Ve, grp, tt, t);
    }
}

// Several operators (lattices of uneven size, each with its own right-hand sides) in one
// launch per half-sweep: workgroup w (after the XCD remap) belongs to the instance whose
// range [first[k], first[k+1]) holds it.  Descriptors travel by value in the kernel
// arguments, so a captured graph replays without host memory.
constexpr int MAX_BATCH = 8;

template <typename Ts, typename Tc> struct SapBatch {
    SapArgs<Ts, Tc> inst[MAX_BATCH];
    int first[MAX_BATCH + 1];
    int n_inst;
};

template <typename Ts, typename Tc, int T, bool LL>
__global__ void __launch_bounds__(256 * T) k_sap_batched(SapBatch<Ts, Tc> B)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int w = xcd_remap(blockIdx.x, B.first[B.n_inst]);
    int k = 0;
    while (k + 1 < B.n_inst && w >= B.first[k + 1]) ++k;
    const SapArgs<Ts, Tc> &a = B.inst[k];
    const int li = w - B.first[k];
    const int bi = li / a.ntiles, tile = li - bi * a.ntiles;
    sap_block<Ts, Tc, T, LL>(a, a.blocks[bi], tile, smem);
}

// the same with the even-odd block solver
template <typename Ts, typename Tc, int T>
__global__ void __launch_bounds__(128 * T, (sizeof(Tc) == 4 && T == 2) ? 3 : 1) k_sap_batched_eo(SapBatch<Ts, Tc> B)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int w = xcd_remap(blockIdx.x, B.first[B.n_inst]);
    int k = 0;
    while (k + 1 < B.n_inst && w >= B.first[k + 1]) ++k;
    const SapArgs<Ts, Tc> &a = B.inst[k];
    const int li = w - B.first[k];
    const int bi = li / a.ntiles, tile = li - bi * a.ntiles;
    sap_block_eo<Ts, Tc, T>(a, a.blocks[bi], tile, smem);
}

struct CopyBatch {
    const void *src[MAX_BATCH];
    void *dst[MAX_BATCH];
    long n[MAX_BATCH];  // elements
    int n_inst;
};

template <typename Ts> __global__ void k_copy_batched(CopyBatch c)
{
    for (int k = 0; k < c.n_inst; ++k) {
        const Ts *s = (const Ts *)c.src[k];
        Ts *d = (Ts *)c.dst[k];
        for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < c.n[k]; i += (long)gridDim.x * blockDim.x)
            d[i] = s[i];
    }
}

template <typename Ts> __global__ void k_fill_zero(Ts *__restrict__ p, long n)
{
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) p[i] = Ts(0);
}

int round64(int n) { return (n + 63) / 64 * 64; }

template <typename Tc> const Tc *op_links(const mrhs_op *op);
template <> const double *op_links<double>(const mrhs_op *op) { return op->links64; }
template <> const float *op_links<float>(const mrhs_op *op) { return op->links32; }
template <typename Tc> const Tc *op_clover(const mrhs_op *op);
template <> const double *op_clover<double>(const mrhs_op *op) { return op->clover64; }
template <> const float *op_clover<float>(const mrhs_op *op) { return op->clover32; }
template <typename Tc> const Tc *op_cloverinv(const mrhs_op *op);
template <> const double *op_cloverinv<double>(const mrhs_op *op) { return op->cloverinv64; }
template <> const float *op_cloverinv<float>(const mrhs_op *op) { return op->cloverinv32; }

size_t align256(size_t n) { return (n + 255) / 256 * 256; }

template <typename Ts, typename Tc, int T, bool EO, bool LL = false>
int launch_batched(const SapBatch<Ts, Tc> &B, int threads, size_t lds, hipStream_t st)
{
    const void *fn = EO ? (const void *)k_sap_batched_eo<Ts, Tc, T> : (const void *)k_sap_batched<Ts, Tc, T, LL>;
    static size_t done = 0;
    if (lds > 65536 && lds > done) {
        if (int rc = hip_check(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds),
                               "hipFuncSetAttribute(batched sap LDS)"))
            return rc;
        done = lds;
    }
    if constexpr (EO) {
        hipLaunchKernelGGL((k_sap_batched_eo<Ts, Tc, T>), dim3(B.first[B.n_inst]), dim3(threads), lds, st, B);
        return hip_check(hipGetLastError(), "k_sap_batched_eo launch");
    } else {
        hipLaunchKernelGGL((k_sap_batched<Ts, Tc, T, LL>), dim3(B.first[B.n_inst]), dim3(threads), lds, st, B);
        return hip_check(hipGetLastError(), "k_sap_batched launch");
    }
}

template <typename Ts, typename Tc>
int sap_batched_dispatch(const mrhs_op *const *ops, int n, const void *const *b, void *const *x, const int32_t *n_rhs,
                         int n_sap, int n_mr, char *ws, bool guess, hipStream_t st)
{
    // one tile for the whole batch: the smallest of the operators' tiles (all divide S)
    int T = 4, maxVb = 0;
    size_t max_lds = ops[0]->max_lds;
    const bool eo = ops[0]->block_solver == MRHS_BLOCK_EO_MR;
    for (int k = 0; k < n; ++k) {
        T = std::min(T, ops[k]->sap_tile);
        maxVb = std::max(maxVb, ops[k]->k.Vb);
        if ((ops[k]->block_solver == MRHS_BLOCK_EO_MR) != eo)
            return set_error(MRHS_EINVAL, "the operators of a batch use different block solvers");
    }
    const int threads = round64(maxVb * T);
    const int eo_threads = round64(maxVb / 2 * T);  // even-odd: one even and one odd site per thread
    size_t lds = sizeof(Tc) * (24 * (size_t)maxVb * T + red_words(threads, T));
    if (maxVb * T > 1024 || lds > max_lds) return set_error(MRHS_EUNSUPPORTED, "batched SAP tile does not fit");
    // the plain MR kernel at tile 4 with FP32 arithmetic stages the block's links in LDS when
    // they fit beside rho
    int max_links = 0;
    for (int k = 0; k < n; ++k) max_links = std::max(max_links, link_box(ops[k]->k).n);
    const size_t lds_ll = lds + sizeof(Tc) * 18 * (size_t)max_links;
    const bool ll = !eo && sizeof(Tc) == 4 && T == 4 && lds_ll <= max_lds;
    if (ll) lds = lds_ll;
    if (n_sap == 0) {
        if (guess) return MRHS_OK;  // no sweep: x keeps the starting guess
        for (int k = 0; k < n; ++k) {
            hipLaunchKernelGGL(k_fill_zero<Ts>, dim3(1024), dim3(256), 0, st, (Ts *)x[k], (long)native_elems(ops[k], n_rhs[k]));
            if (int rc = hip_check(hipGetLastError(), "k_fill_zero launch")) return rc;
        }
        return MRHS_OK;
    }
    SapBatch<Ts, Tc> B{};
    CopyBatch C{};
    B.n_inst = n;
    char *wp = ws;
    Ts *snap[MAX_BATCH] = {};
    for (int k = 0; k < n; ++k) {
        const mrhs_op *op = ops[k];
        SapArgs<Ts, Tc> &a = B.inst[k];
        a.g = op->k;
        a.links = op_links<Tc>(op);
        a.clover = op_clover<Tc>(op);
        a.blk_coords = op->blk_coords;
        a.loc_coords = op->loc_coords;
        a.ntiles = (n_rhs[k] + op->k.S - 1) / op->k.S * (op->k.S / T);
        a.n_mr = n_mr;
        a.b = (const Ts *)b[k];
        a.x = (Ts *)x[k];
        a.cloverinv = op_cloverinv<Tc>(op);
        a.eo_sites = op->eo_sites;
        a.Ve = op->k.Vb / 2;
        if (op->odd_blocks) {
            snap[k] = (Ts *)wp;
            wp += align256(native_elems(op, n_rhs[k]) * sizeof(Ts));
        }
        a.sig = (Tc *)wp;
        wp += align256(native_elems(op, n_rhs[k]) * sizeof(Tc));
        a.ecor = nullptr;
        if (!op->odd_blocks) {
            a.ecor = (Tc *)wp;
            wp += align256(native_elems(op, n_rhs[k]) * sizeof(Tc));
        }
    }
    for (int s = 0; s < n_sap; ++s)
        for (int c = 0; c < 2; ++c) {
            C.n_inst = 0;
            B.first[0] = 0;
            for (int k = 0; k < n; ++k) {
                const mrhs_op *op = ops[k];
                SapArgs<Ts, Tc> &a = B.inst[k];
                a.colour = c;
                a.blocks = op->colour_blocks + (c == 0 ? 0 : op->n_colour[0]);
                a.nblocks = op->n_colour[c];
                a.mode = s == 0 && !guess ? c : 2;  // from zero, x vanishes on blocks not yet visited
                // sigma carries a colour's residual from one visit to the next (plain MR only)
                a.sig_in = !eo && s > 0;
                a.sig_out = !eo && s + 1 < n_sap;
                // the incremental residual where no block neighbours one of its own colour: every
                // visit but the call's last one leaves its change of x for the other colour
                a.inc = !eo && !op->odd_blocks;
                a.e_out = a.inc && !(s + 1 == n_sap && c == 1);
                a.xr = a.x;
                if (a.mode == 2 && op->odd_blocks) {
                    C.src[C.n_inst] = a.x;
                    C.dst[C.n_inst] = snap[k];
                    C.n[C.n_inst] = (long)native_elems(op, n_rhs[k]);
                    ++C.n_inst;
                    a.xr = snap[k];
                }
                B.first[k + 1] = B.first[k] + a.nblocks * a.ntiles;
            }
            if (C.n_inst) {
                hipLaunchKernelGGL(k_copy_batched<Ts>, dim3(2048), dim3(256), 0, st, C);
                if (int rc = hip_check(hipGetLastError(), "k_copy_batched launch")) return rc;
            }
            if (B.first[n] == 0) continue;
            int rc;
            const int thr = eo ? eo_threads : threads;
            switch (T * 2 + (eo ? 1 : 0)) {
            case 2: rc = launch_batched<Ts, Tc, 1, false>(B, thr, lds, st); break;
            case 4: rc = launch_batched<Ts, Tc, 2, false>(B, thr, lds, st); break;
            case 3: rc = launch_batched<Ts, Tc, 1, true>(B, thr, lds, st); break;
            case 5: rc = launch_batched<Ts, Tc, 2, true>(B, thr, lds, st); break;
            default:
                // tile 4 only with FP32 arithmetic (FP64 would spill to scratch)
                if constexpr (sizeof(Tc) == 4) {
                    if (T == 4) {
                        rc = eo ? launch_batched<Ts, Tc, 4, true>(B, thr, lds, st)
                           : ll ? launch_batched<Ts, Tc, 4, false, true>(B, thr, lds, st)
                                : launch_batched<Ts, Tc, 4, false>(B, thr, lds, st);
                        break;
                    }
                }
                rc = set_error(MRHS_EUNSUPPORTED, "SAP tile not built");
            }
            if (rc) return rc;
        }
    return MRHS_OK;
}

}  // namespace

size_t ws_bytes_sap_batched(const mrhs_op *const *ops, int n, const int32_t *n_rhs)
{
    size_t w = 0;
    for (int k = 0; k < n; ++k) {
        const size_t ne = native_elems(ops[k], n_rhs[k]);
        const size_t tc = ops[k]->prec == MRHS_PREC_F64 ? sizeof(double) : sizeof(float);
        if (ops[k]->odd_blocks) w += align256(ne * dtype_size(ops[k]->dtype));  // snapshot of x
        else w += align256(ne * tc);                                             // changes of x
        w += align256(ne * tc);                                                  // sigma / rho
    }
    return w;
}

int launch_sap_batched(const mrhs_op *const *ops, int n, const void *const *b, void *const *x, const int32_t *n_rhs,
                       int n_sap, int n_mr, void *ws, hipStream_t st, bool guess)
{
    if (n > MAX_BATCH) return set_error(MRHS_EUNSUPPORTED, "more than 8 operators in one batch");
    switch (ops[0]->prec) {
    case MRHS_PREC_F64:
        return sap_batched_dispatch<double, double>(ops, n, b, x, n_rhs, n_sap, n_mr, (char *)ws, guess, st);
    case MRHS_PREC_F32:
        return sap_batched_dispatch<float, float>(ops, n, b, x, n_rhs, n_sap, n_mr, (char *)ws, guess, st);
    default:
        return sap_batched_dispatch<__half, float>(ops, n, b, x, n_rhs, n_sap, n_mr, (char *)ws, guess, st);
    }
}

size_t ws_bytes_sap(const mrhs_op *op, int n_rhs) { return ws_bytes_sap_batched(&op, 1, &n_rhs); }

int launch_sap(const mrhs_op *op, const void *b, void *x, int n_rhs, int n_sap, int n_mr, void *ws, hipStream_t st,
               bool guess)
{
    return launch_sap_batched(&op, 1, &b, &x, &n_rhs, n_sap, n_mr, ws, st, guess);
}
