// dirac.hip -- y = D x on the full lattice for many right-hand sides, and the FP64
// residual norms ||b - D x|| / ||b||.
//
// One workgroup per (block, tile of T right-hand sides); thread (off, t) owns one site
// and one right-hand side.  The T lanes of a site issue the same link and clover loads,
// so the operator is fetched once per site for the whole tile (the mat-vec -> mat-mat
// argument of Sec. 6); tiles of one block share an XCD's L2 through xcd_remap.
#include <mutex>

#include "launch.h"
#include "stencil.h"

// Scratch of mrhs_residual_norms_noalloc: the partial sums per (tile, block, lane) that
// k_residual writes and k_residual_finish adds up, in place of a caller's workspace.  One
// copy per device, held until the process ends.  Host code never passes the array's name
// to a kernel (in host code it is a host-side stand-in): it uses the device address that
// hipGetSymbolAddress returns for the device the call runs on.
constexpr size_t RESID_SCRATCH_BYTES = size_t(32) << 20;
static __device__ __align__(256) unsigned char scratch[RESID_SCRATCH_BYTES];

namespace {

template <typename Ts, typename Tc, int T>
__global__ void __launch_bounds__(256 * T) k_dirac(KGeo g, const Tc *__restrict__ links, const Tc *__restrict__ clover,
                                                   const uint32_t *__restrict__ blk_coords,
                                                   const uint32_t *__restrict__ loc_coords, const Ts *__restrict__ x,
                                                   Ts *__restrict__ y, int ntiles)
{
    const int nwg = g.nblk * ntiles;
    const int li = xcd_remap(blockIdx.x, nwg);
    const int blk = li / ntiles, tile = li - blk * ntiles;
    const int off = threadIdx.x / T, t = threadIdx.x % T;
    if (off >= g.Vb) return;
    const int grp = (tile * T) / g.S, tt = (tile * T) % g.S + t;  // T divides S: grp is uniform
    int bc[4], lc[4];
    decode_site(g, blk_coords, loc_coords, blk, off, bc, lc);
    Spinor<Tc> out;
    dirac_site_global<Tc>(g, links, clover, x, grp, tt, blk, off, bc, lc, out, NoSkip{});
    store_spinor(g, y, grp, blk, off, tt, out);
}

// The stencil at tile 4 on a short length of 4 (FP32): a workgroup takes two consecutive
// groups of the native layout, 8 lanes per site (lanes t < 4 the first group, t >= 4 the
// second), and walks the block in passes of 128 sites, so that a site's links and clover are
// loaded once for 8 right-hand sides; lanes of a group beyond the last one do nothing.
template <typename Ts, typename Tc>
__global__ void __launch_bounds__(1024) k_dirac_2g(KGeo g, const Tc *__restrict__ links, const Tc *__restrict__ clover,
                                                   const uint32_t *__restrict__ blk_coords,
                                                   const uint32_t *__restrict__ loc_coords, const Ts *__restrict__ x,
                                                   Ts *__restrict__ y, int ntiles, int ngrp)
{
    const int li = xcd_remap(blockIdx.x, g.nblk * ntiles);
    const int blk = li / ntiles, tile = li - blk * ntiles;
    const int lt = tile * 8 + threadIdx.x % 8, grp = lt / g.S, tt = lt % g.S;
    const int nsite = g.Vb < 128 ? g.Vb : 128;
#pragma unroll 1
    for (int o = threadIdx.x / 8; o < g.Vb && grp < ngrp; o += nsite) {
        const int off = opaque_index(o);
        int bc[4], lc[4];
        decode_site(g, blk_coords, loc_coords, blk, off, bc, lc);
        Spinor<Tc> out;
        dirac_site_global<Tc>(g, links, clover, x, grp, tt, blk, off, bc, lc, out, NoSkip{});
        store_spinor(g, y, grp, blk, off, tt, out);
    }
}

// Per (block, tile of T right-hand sides): partial sums of |b - D x|^2 and |b|^2 per
// right-hand side, FP64.  A workgroup of (up to 64 sites) x T lanes walks the block in
// passes of 64 sites, so that a workgroup is small while the FP64 stencil takes ~130
// registers.  The T lanes of a site share its FP64 field loads; with T = 2S a tile spans two
// groups of the native layout (lanes t < S the first, t >= S the second), which halves the
// field loads per right-hand side.  Lanes of a group beyond the last one add nothing.
constexpr int RES_SITES = 64;

template <typename Ts, int T>
__global__ void __launch_bounds__(RES_SITES * T) k_residual(KGeo g, const double *__restrict__ links,
                                                            const double *__restrict__ clover,
                                                            const uint32_t *__restrict__ blk_coords,
                                                            const uint32_t *__restrict__ loc_coords,
                                                            const Ts *__restrict__ b, const Ts *__restrict__ x,
                                                            int ntiles, int ngrp, double *__restrict__ part)
{
    __shared__ double red[RES_SITES * T / 64][T][2];
    // tiles of one block on one XCD, consecutively: the block's FP64 fields and its
    // neighbours' spinors are fetched into that XCD's L2 once for all its tiles
    const int li = xcd_remap(blockIdx.x, g.nblk * ntiles);
    const int blk = li / ntiles, tile = li - blk * ntiles;
    const int lt = tile * T + threadIdx.x % T, grp = lt / g.S, tt = lt % g.S;
    const int nsite = g.Vb < RES_SITES ? g.Vb : RES_SITES;
    double num = 0, den = 0;
#pragma unroll 1
    for (int o = threadIdx.x / T; o < g.Vb && grp < ngrp; o += nsite) {
        const int off = opaque_index(o);
        int bc[4], lc[4];
        decode_site(g, blk_coords, loc_coords, blk, off, bc, lc);
        Spinor<double> Dx, bb;
        dirac_site_global<double>(g, links, clover, x, grp, tt, blk, off, bc, lc, Dx, NoSkip{});
        load_spinor<double>(g, b, grp, blk, off, tt, bb);
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            const double dr = bb.re[c] - Dx.re[c], di = bb.im[c] - Dx.im[c];
            num += dr * dr + di * di;
            den += bb.re[c] * bb.re[c] + bb.im[c] * bb.im[c];
        }
    }
    num = wave_sum_stride(num, T);
    den = wave_sum_stride(den, T);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane < T) {
        red[wave][lane][0] = num;
        red[wave][lane][1] = den;
    }
    __syncthreads();
    if (threadIdx.x < T) {
        double sn = 0, sd = 0;
        const int nw = (blockDim.x + 63) >> 6;
        for (int w = 0; w < nw; ++w) {
            sn += red[w][threadIdx.x][0];
            sd += red[w][threadIdx.x][1];
        }
        double *p = part + (((long)tile * g.nblk + blk) * T + threadIdx.x) * 2;
        p[0] = sn;
        p[1] = sd;
    }
}

// out[k] = sqrt(sum num / sum den), summed over blocks in a fixed order
template <int T>
__global__ void k_residual_finish(const double *__restrict__ part, int nblk, int n_rhs, double *__restrict__ out)
{
    __shared__ double sn[256], sd[256];
    const int k = blockIdx.x;
    const int tile = k / T, t = k % T;
    double a = 0, d = 0;
    for (int blk = threadIdx.x; blk < nblk; blk += blockDim.x) {
        const double *p = part + (((long)tile * nblk + blk) * T + t) * 2;
        a += p[0];
        d += p[1];
    }
    sn[threadIdx.x] = a;
    sd[threadIdx.x] = d;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sn[threadIdx.x] += sn[threadIdx.x + s];
            sd[threadIdx.x] += sd[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0 && k < n_rhs) out[k] = sqrt(sn[0]) / sqrt(sd[0]);
}

int round64(int n) { return (n + 63) / 64 * 64; }

template <typename Ts, typename Tc>
int dirac_dispatch(const mrhs_op *op, const Tc *links, const Tc *clover, const void *x, void *y, int n_rhs,
                   hipStream_t st)
{
    const KGeo &g = op->k;
    const int T = op->dirac_tile;
    const int ngrp = (n_rhs + g.S - 1) / g.S;
    const int ntiles = ngrp * (g.S / T);
    dim3 grid(g.nblk * ntiles), block(round64(g.Vb * T));
    switch (T) {
    case 1:
        hipLaunchKernelGGL((k_dirac<Ts, Tc, 1>), grid, block, 0, st, g, links, clover, op->blk_coords, op->loc_coords,
                           (const Ts *)x, (Ts *)y, ntiles);
        break;
    case 2:
        hipLaunchKernelGGL((k_dirac<Ts, Tc, 2>), grid, block, 0, st, g, links, clover, op->blk_coords, op->loc_coords,
                           (const Ts *)x, (Ts *)y, ntiles);
        break;
    case 4:
        // tile 4 only with FP32 arithmetic (FP64 would spill to scratch)
        if constexpr (sizeof(Tc) == 4) {
            if (g.S == 4) {
                const int nt2 = (ngrp + 1) / 2, ns = g.Vb < 128 ? g.Vb : 128;
                hipLaunchKernelGGL((k_dirac_2g<Ts, Tc>), dim3(g.nblk * nt2), dim3(round64(ns * 8)), 0, st, g, links,
                                   clover, op->blk_coords, op->loc_coords, (const Ts *)x, (Ts *)y, nt2, ngrp);
                break;
            }
            hipLaunchKernelGGL((k_dirac<Ts, Tc, 4>), grid, block, 0, st, g, links, clover, op->blk_coords,
                               op->loc_coords, (const Ts *)x, (Ts *)y, ntiles);
            break;
        }
        return set_error(MRHS_EUNSUPPORTED, "dirac tile not built");
    default:
        return set_error(MRHS_EUNSUPPORTED, "dirac tile not built");
    }
    return hip_check(hipGetLastError(), "k_dirac launch");
}

// lanes per site of the residual: two groups of 4 right-hand sides, else as many lanes as
// the short length allows
int residual_tile(const KGeo &g) { return g.S % 4 == 0 ? 8 : g.S % 2 == 0 ? 2 : 1; }
int residual_tiles(const KGeo &g, int n_rhs, int T)
{
    const int ngrp = (n_rhs + g.S - 1) / g.S;
    return (ngrp * g.S + T - 1) / T;
}

template <typename Ts, int T>
int residual_launch(const mrhs_op *op, const void *b, const void *x, int n_rhs, double *out, void *ws, hipStream_t st)
{
    const KGeo &g = op->k;
    const int ngrp = (n_rhs + g.S - 1) / g.S;
    const int ntiles = residual_tiles(g, n_rhs, T);
    double *part = (double *)ws;
    const int nsite = g.Vb < RES_SITES ? g.Vb : RES_SITES;
    hipLaunchKernelGGL((k_residual<Ts, T>), dim3(g.nblk * ntiles), dim3(round64(nsite * T)), 0, st, g, op->links64,
                       op->clover64, op->blk_coords, op->loc_coords, (const Ts *)b, (const Ts *)x, ntiles, ngrp,
                       part);
    if (int rc = hip_check(hipGetLastError(), "k_residual launch")) return rc;
    hipLaunchKernelGGL((k_residual_finish<T>), dim3(n_rhs), dim3(256), 0, st, part, g.nblk, n_rhs, out);
    return hip_check(hipGetLastError(), "k_residual_finish launch");
}

template <typename Ts>
int residual_dispatch(const mrhs_op *op, const void *b, const void *x, int n_rhs, double *out, void *ws, hipStream_t st)
{
    switch (residual_tile(op->k)) {
    case 8: return residual_launch<Ts, 8>(op, b, x, n_rhs, out, ws, st);
    case 2: return residual_launch<Ts, 2>(op, b, x, n_rhs, out, ws, st);
    default: return residual_launch<Ts, 1>(op, b, x, n_rhs, out, ws, st);
    }
}

}  // namespace

int launch_dirac(const mrhs_op *op, const void *x, void *y, int n_rhs, hipStream_t st)
{
    switch (op->prec) {
    case MRHS_PREC_F64:
        return dirac_dispatch<double, double>(op, op->links64, op->clover64, x, y, n_rhs, st);
    case MRHS_PREC_F32:
        return dirac_dispatch<float, float>(op, op->links32, op->clover32, x, y, n_rhs, st);
    default:
        return dirac_dispatch<__half, float>(op, op->links32, op->clover32, x, y, n_rhs, st);
    }
}

size_t ws_bytes_residual(const mrhs_op *op, int n_rhs)
{
    const KGeo &g = op->k;
    const int T = residual_tile(g);
    return (size_t)residual_tiles(g, n_rhs, T) * T * g.nblk * 2 * sizeof(double);
}

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
void *scratch_ptr[MAX_DEVICES] = {};

// this device's copy of the scratch array, looked up once per device with it current
int device_scratch(int device, void **out)
{
    if (device < 0 || device >= MAX_DEVICES) return set_error(MRHS_EUNSUPPORTED, "device index above 63");
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[device]) {
        int cur = -1;
        if (int rc = hip_check(hipGetDevice(&cur), "hipGetDevice")) return rc;
        if (cur != device)
            if (int rc = hip_check(hipSetDevice(device), "hipSetDevice")) return rc;
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) (void)hipSetDevice(cur);
        if (int rc = hip_check(e, "hipGetSymbolAddress(scratch)")) return rc;
        scratch_ptr[device] = p;
    }
    *out = scratch_ptr[device];
    return MRHS_OK;
}

}  // namespace

int launch_residual_noalloc(const mrhs_op *op, const void *b, const void *x, int n_rhs, double *out, hipStream_t st)
{
    if (ws_bytes_residual(op, n_rhs) > RESID_SCRATCH_BYTES)
        return set_error(MRHS_EUNSUPPORTED, "residual partial sums (" + std::to_string(ws_bytes_residual(op, n_rhs)) +
                                                " bytes) exceed the 32 MiB scratch of the allocation-free call");
    void *ws = nullptr;
    if (int rc = device_scratch(op->device, &ws)) return rc;
    return launch_residual(op, b, x, n_rhs, out, ws, st);
}

int launch_residual(const mrhs_op *op, const void *b, const void *x, int n_rhs, double *out, void *ws, hipStream_t st)
{
    switch (op->dtype) {
    case MRHS_DTYPE_F64:
        return residual_dispatch<double>(op, b, x, n_rhs, out, ws, st);
    case MRHS_DTYPE_F32:
        return residual_dispatch<float>(op, b, x, n_rhs, out, ws, st);
    default:
        return residual_dispatch<__half>(op, b, x, n_rhs, out, ws, st);
    }
}
