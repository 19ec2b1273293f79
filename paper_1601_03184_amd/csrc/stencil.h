// stencil.h -- the Wilson-clover stencil at one site for one right-hand side, with
// neighbours read from a native vector in global memory.  Links in the operator's
// kernel layout are stored pre-scaled by -1/2 (exact in binary floating point), so
//   (D psi)(x) = A(x) psi(x) + sum_mu [ (1 - g_mu) W_mu(x) psi(x+mu) + (1 + g_mu) W_mu(x-mu)^dag psi(x-mu) ],
// W = -U/2.
#pragma once

#include "internal.h"

// Scheduling fences.  Without them the compiler issues the loads of all eight hops
// first and does the arithmetic last, holding ~430 values live, and the kernel spills.
// sched_fence() stops the machine scheduler from moving instructions across it;
// value_fence(s) forces every accumulator in s to be computed at that point (an empty
// volatile asm that reads and writes them).  Neither emits an instruction.
__device__ inline void sched_fence() { __builtin_amdgcn_sched_barrier(0); }

template <typename T> __device__ inline void value_fence(Spinor<T> &s)
{
#pragma unroll
    for (int c = 0; c < 12; ++c) asm volatile("" : "+v"(s.re[c]), "+v"(s.im[c]));
}

// Hide a per-lane index from loop-invariant code motion: loads addressed through it
// are issued inside the loop instead of being hoisted (and held in registers) above it.
__device__ inline int opaque_index(int i)
{
    asm volatile("" : "+v"(i));
    return i;
}

template <typename T> __device__ inline void hop_fence(Spinor<T> &s)
{
    value_fence(s);
    sched_fence();
}

__device__ inline void decode_site(const KGeo &g, const uint32_t *__restrict__ blk_coords,
                                   const uint32_t *__restrict__ loc_coords, int blk, int off, int (&bc)[4], int (&lc)[4])
{
    const uint32_t pb = blk_coords[blk], pl = loc_coords[off];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        bc[mu] = unpack_coord(pb, mu);
        lc[mu] = unpack_coord(pl, mu);
    }
}

// Vector addressing: the group's base pointer and the component stride are uniform
// across the workgroup (all lanes of a tile share a group), so each component is read
// as (uniform base + component * stride)[32-bit lane offset].  One VGPR of address per
// spinor instead of 24 64-bit ones.
__device__ inline uint32_t lane_offset(const KGeo &g, int blk, int off, int t)
{
    return (uint32_t)((blk * 24) * g.Vb * g.S + off * g.S + t);
}

template <typename Ts> __device__ inline const Ts *group_base(const KGeo &g, const Ts *v, int grp)
{
    return v + (size_t)grp * g.nblk * 24 * g.Vb * g.S;
}
template <typename Ts> __device__ inline Ts *group_base(const KGeo &g, Ts *v, int grp)
{
    return v + (size_t)grp * g.nblk * 24 * g.Vb * g.S;
}

template <typename Tc, typename Ts>
__device__ inline void load_spinor(const KGeo &g, const Ts *__restrict__ v, int grp, int blk, int off, int t, Spinor<Tc> &s)
{
    const Ts *vg = group_base(g, v, grp);
    const uint32_t lo = lane_offset(g, blk, off, t);
    const uint32_t str = (uint32_t)(g.Vb * g.S);
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        s.re[c] = load_as<Tc>(vg + (size_t)(2 * c) * str + lo);
        s.im[c] = load_as<Tc>(vg + (size_t)(2 * c + 1) * str + lo);
    }
}

template <typename Tc, typename Ts>
__device__ inline void store_spinor(const KGeo &g, Ts *__restrict__ v, int grp, int blk, int off, int t, const Spinor<Tc> &s)
{
    Ts *vg = group_base(g, v, grp);
    const uint32_t lo = lane_offset(g, blk, off, t);
    const uint32_t str = (uint32_t)(g.Vb * g.S);
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        vg[(size_t)(2 * c) * str + lo] = store_as<Ts>(s.re[c]);
        vg[(size_t)(2 * c + 1) * str + lo] = store_as<Ts>(s.im[c]);
    }
}

__device__ inline int block_colour(const KGeo &g, const uint32_t *__restrict__ blk_coords, int blk)
{
    const uint32_t p = blk_coords[blk];
    return (unpack_coord(p, 0) + unpack_coord(p, 1) + unpack_coord(p, 2) + unpack_coord(p, 3)) & 1;
}

// out = A(x) psi, one chiral half at a time (36 field values live, not 72)
template <typename Tf, typename Tc, typename Tx>
__device__ inline void clover_site(const Tf *__restrict__ clover, long V, long site, const Spinor<Tx> &psi, Spinor<Tc> &out)
{
    {
        Tc A[36];
        load_clover_half<0>(clover, V, site, A);
        clover_half<0>(A, psi, out);
    }
    value_fence(out);
    sched_fence();
    {
        Tc A[36];
        load_clover_half<1>(clover, V, site, A);
        clover_half<1>(A, psi, out);
    }
}

// One direction of the full stencil with neighbours from global memory.
// SKIP(blk) tells whether the vector is known to be zero on a block.
template <int MU, typename Tc, typename Ts, typename Tf, typename Skip>
__device__ inline void hop_pair_global(const KGeo &g, const Tf *__restrict__ links, const Ts *__restrict__ x, int grp,
                                       int t, int blk, int off, const int (&bc)[4], const int (&lc)[4], Spinor<Tc> &out,
                                       Skip skip)
{
    const long ns = (long)blk * g.Vb + off;
    {
        const NbrSite n = nbr_fwd(g, MU, blk, off, bc, lc);
        if (!skip(n.blk)) {
            Spinor<typename ChiType<Tc, Ts>::type> chi;
            load_spinor<typename ChiType<Tc, Ts>::type>(g, x, grp, n.blk, n.off, t, chi);
            Tc U[18];
            load_link(links, g.V, MU, ns, U);
            hop_accumulate<MU, -1, false>(U, chi, out);
        }
    }
    hop_fence(out);
    {
        const NbrSite n = nbr_bwd(g, MU, blk, off, bc, lc);
        if (!skip(n.blk)) {
            Spinor<typename ChiType<Tc, Ts>::type> chi;
            load_spinor<typename ChiType<Tc, Ts>::type>(g, x, grp, n.blk, n.off, t, chi);
            Tc U[18];
            load_link(links, g.V, MU, (long)n.blk * g.Vb + n.off, U);
            hop_accumulate<MU, +1, true>(U, chi, out);
        }
    }
}

// out = (D x)(site) for right-hand side (grp, t).
template <typename Tc, typename Ts, typename Tf, typename Skip>
__device__ inline void dirac_site_global(const KGeo &g, const Tf *__restrict__ links, const Tf *__restrict__ clover,
                                         const Ts *__restrict__ x, int grp, int t, int blk, int off, const int (&bc)[4],
                                         const int (&lc)[4], Spinor<Tc> &out, Skip skip)
{
    if (!skip(blk)) {
        Spinor<typename ChiType<Tc, Ts>::type> own;
        load_spinor<typename ChiType<Tc, Ts>::type>(g, x, grp, blk, off, t, own);
        clover_site(clover, g.V, (long)blk * g.Vb + off, own, out);
    } else {
        spinor_zero(out);
    }
    hop_fence(out);
    hop_pair_global<0>(g, links, x, grp, t, blk, off, bc, lc, out, skip);
    hop_fence(out);
    hop_pair_global<1>(g, links, x, grp, t, blk, off, bc, lc, out, skip);
    hop_fence(out);
    hop_pair_global<2>(g, links, x, grp, t, blk, off, bc, lc, out, skip);
    hop_fence(out);
    hop_pair_global<3>(g, links, x, grp, t, blk, off, bc, lc, out, skip);
    hop_fence(out);
}

// out += the hops of (D x)(site) whose neighbour lies outside the site's SAP block (the
// part of the residual that couples a block to its neighbours); SKIP as above.  A site lies on
// at most one of the two faces of a direction unless its block is one site thick there, so
// both faces' loads are issued in one round (each lane its own face's neighbour and link) and
// the lanes on either face accumulate their hop; a one-site-thick block takes the backward
// face in a second round.  Per lane the hops are added in the same order as face by face.
template <int MU, typename Tc, typename Ts, typename Tf, typename Skip>
__device__ inline void face_pair_global(const KGeo &g, const Tf *__restrict__ links, const Ts *__restrict__ x,
                                        int grp, int t, int blk, int off, const int (&bc)[4], const int (&lc)[4],
                                        Spinor<Tc> &out, Skip skip)
{
    const long ns = (long)blk * g.Vb + off;
    const bool ff = lc[MU] + 1 == g.b[MU] && g.nb[MU] > 1;  // on the +MU face
    const bool fb = lc[MU] == 0 && g.nb[MU] > 1;            // on the -MU face
    if (ff || fb) {
        const NbrSite n = ff ? nbr_fwd(g, MU, blk, off, bc, lc) : nbr_bwd(g, MU, blk, off, bc, lc);
        if (!skip(n.blk)) {
            Spinor<typename ChiType<Tc, Ts>::type> chi;
            load_spinor<typename ChiType<Tc, Ts>::type>(g, x, grp, n.blk, n.off, t, chi);
            Tc U[18];
            load_link(links, g.V, MU, ff ? ns : (long)n.blk * g.Vb + n.off, U);
            if (ff) hop_accumulate<MU, -1, false>(U, chi, out);
            else hop_accumulate<MU, +1, true>(U, chi, out);
        }
    }
    hop_fence(out);
    if (ff && fb) {
        const NbrSite n = nbr_bwd(g, MU, blk, off, bc, lc);
        if (!skip(n.blk)) {
            Spinor<typename ChiType<Tc, Ts>::type> chi;
            load_spinor<typename ChiType<Tc, Ts>::type>(g, x, grp, n.blk, n.off, t, chi);
            Tc U[18];
            load_link(links, g.V, MU, (long)n.blk * g.Vb + n.off, U);
            hop_accumulate<MU, +1, true>(U, chi, out);
        }
    }
}

template <typename Tc, typename Ts, typename Tf, typename Skip>
__device__ inline void face_hops_global(const KGeo &g, const Tf *__restrict__ links, const Ts *__restrict__ x, int grp,
                                        int t, int blk, int off, const int (&bc)[4], const int (&lc)[4],
                                        Spinor<Tc> &out, Skip skip)
{
    hop_fence(out);
    face_pair_global<0>(g, links, x, grp, t, blk, off, bc, lc, out, skip);
    hop_fence(out);
    face_pair_global<1>(g, links, x, grp, t, blk, off, bc, lc, out, skip);
    hop_fence(out);
    face_pair_global<2>(g, links, x, grp, t, blk, off, bc, lc, out, skip);
    hop_fence(out);
    face_pair_global<3>(g, links, x, grp, t, blk, off, bc, lc, out, skip);
    hop_fence(out);
}

struct NoSkip {
    __device__ bool operator()(int) const { return false; }
};

template <typename T> __device__ inline T wave_sum_stride(T v, int T_)
{
    // sum over the lanes of a wave that agree modulo T_ (T_ a power of two <= 32)
    for (int o = 32; o >= T_; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
