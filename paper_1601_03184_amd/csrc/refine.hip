// refine.hip -- one pass of the setup's refinement phase over all test vectors at once
// (Alg. 2 with the block length N_b = n_tv: the loop over test vectors moved into the
// kernels): coarse-grid correction of every test vector, then the smoother started from it,
// and the test vectors replaced by the smoother's result.  R, P and D_c are the current
// ones (from block_orthonormalize and coarse_op_build); rebuilding them from the refined
// vectors is the caller's next step, as in the last line of Alg. 2.
#include <algorithm>

#include "launch.h"

namespace {

template <typename Ts> __global__ void k_copy_vec(const Ts *__restrict__ s, Ts *__restrict__ d, long n)
{
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) d[i] = s[i];
}

size_t a256(size_t n) { return (n + 255) / 256 * 256; }

struct RefineWs {
    float *vc, *uc;
    void *x;
    void *gm;
    void *sap;
    size_t gm_bytes, sap_bytes, total;
};

RefineWs refine_layout(const mrhs_op *op, int n_tv, int m, char *base)
{
    RefineWs w{};
    const size_t cb = (size_t)op->n_agg * 2 * n_tv * 2 * ((n_tv + 3) / 4 * 4) * sizeof(float);
    const size_t xb = native_elems(op, n_tv) * dtype_size(op->dtype);
    w.gm_bytes = ws_bytes_coarse_solve(op, n_tv, n_tv, m);
    w.sap_bytes = ws_bytes_sap(op, n_tv);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *p = base ? base + off : nullptr;
        off += a256(std::max(bytes, (size_t)1));
        return p;
    };
    w.vc = (float *)take(cb);
    w.uc = (float *)take(cb);
    w.x = take(xb);
    w.gm = take(w.gm_bytes);
    w.sap = take(w.sap_bytes);
    w.total = off;
    return w;
}

}  // namespace

size_t ws_bytes_refine(const mrhs_op *op, int n_tv, int m) { return refine_layout(op, n_tv, m, nullptr).total; }

int launch_refine(const mrhs_op *op, void *V, int n_tv, const void *Q, int qdt, const float *Dc, int n_sap, int n_mr,
                  int m, double tol, void *ws, hipStream_t st)
{
    RefineWs w = refine_layout(op, n_tv, m, (char *)ws);
    const int vdt = op->dtype;
    // v_c = R v;  u_c ~ D_c^-1 v_c;  u = P u_c
    if (int rc = launch_restrict(op, Q, qdt, n_tv, V, vdt, w.vc, n_tv, st)) return rc;
    if (int rc = launch_coarse_solve(op, Dc, n_tv, w.vc, w.uc, n_tv, m, tol, nullptr, nullptr, w.gm, st)) return rc;
    if (int rc = launch_prolong(op, Q, qdt, n_tv, w.uc, w.x, vdt, n_tv, st)) return rc;
    // the smoother on D x = v from the coarse-grid correction; the result replaces v
    if (int rc = launch_sap(op, V, w.x, n_tv, n_sap, n_mr, w.sap, st, true)) return rc;
    const long nel = (long)native_elems(op, n_tv);
    switch (vdt) {
    case MRHS_DTYPE_F64:
        hipLaunchKernelGGL(k_copy_vec<double>, dim3(2048), dim3(256), 0, st, (const double *)w.x, (double *)V, nel);
        break;
    case MRHS_DTYPE_F32:
        hipLaunchKernelGGL(k_copy_vec<float>, dim3(2048), dim3(256), 0, st, (const float *)w.x, (float *)V, nel);
        break;
    default:
        hipLaunchKernelGGL(k_copy_vec<__half>, dim3(2048), dim3(256), 0, st, (const __half *)w.x, (__half *)V, nel);
    }
    return hip_check(hipGetLastError(), "k_copy_vec launch");
}
