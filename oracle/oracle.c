/*
 * oracle.c -- plain, slow FP64 CPU reference of the multiple-right-hand-side
 * DD-alpha-AMG setup path (Richtmann, Heybrock, Wettig, "Multiple right-hand-side
 * setup for the DD-alpha-AMG", Lattice 2015).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark load this library.  It shares no source, header, table or
 * constant with the GPU library, and the GPU library never calls it.
 *
 * What it computes (the paper's Sec. 2 "Description of the algorithm"): the initial
 * setup phase -- the Schwarz-alternating-procedure smoother run on every test
 * vector from a zero starting guess, then restriction R, prolongation P = R^dagger
 * and the coarse operator D_c built from the smoothed vectors.  Alg. 3 (Sec. 5)
 * fixes the shape of R: per aggregate i and spin half h, an N_tv x 6 V_block block.
 *
 * The paper does not define the Dirac operator, the SAP variant or the block
 * solver (it cites them).  The readings used here, all standard:
 *   - lattice extents L[0..3] = x,y,z,t, site index x0 + L0*(x1 + L1*(x2 + L2*x3)),
 *     periodic in every direction;
 *   - a vector holds 12 complex numbers per site (4 spins x 3 colours, Sec. 2),
 *     component index 3*spin + colour;
 *   - Wilson-clover operator in DeGrand-Rossi chiral basis,
 *       (D psi)(x) = A(x) psi(x)
 *                    - 1/2 sum_mu [ (1 - g_mu) U_mu(x) psi(x+mu)
 *                                  + (1 + g_mu) U_mu(x-mu)^dag psi(x-mu) ],
 *       A(x) = (4 + m0) + C(x),
 *       C(x) = -(csw/16) sum_{mu<nu} g_mu g_nu (x) (Q_munu(x) - Q_munu(x)^dag),
 *     Q_munu the sum of the four plaquette leaves in the (mu,nu) plane at x;
 *   - SAP: red-black multiplicative Schwarz over lattice blocks, the residual
 *     recomputed before each colour, red (even block-coordinate sum) first;
 *   - block solver: plain minimal residual with a fixed number of steps, step
 *     length set to 0 when the block residual's image is exactly zero; or (the
 *     even-odd variant, DD-alpha-AMG's block solver) the same steps on the block's
 *     Schur complement over its even sites, then the odd sites from the even ones;
 *   - Gram-Schmidt: the unique thin QR factor with positive real diagonal,
 *     computed by modified Gram-Schmidt with one re-orthogonalisation pass.
 *
 * Build: gcc -std=c99 -O2 -fopenmp -fPIC -shared oracle.c -o liboracle.so -lm
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* ------------------------------------------------------------------------ */
/* Lattice geometry                                                          */
/* ------------------------------------------------------------------------ */

static long volume(const int *L) { return (long)L[0] * L[1] * L[2] * L[3]; }

static void site_coords(const int *L, long s, int *x)
{
    for (int mu = 0; mu < 4; ++mu) {
        x[mu] = (int)(s % L[mu]);
        s /= L[mu];
    }
}

static long site_index(const int *L, const int *x)
{
    return x[0] + (long)L[0] * (x[1] + (long)L[1] * (x[2] + (long)L[2] * x[3]));
}

/* the site one step (+1 or -1) from s in direction mu, periodic */
static long neighbour(const int *L, long s, int mu, int step)
{
    int x[4];
    site_coords(L, s, x);
    x[mu] = (x[mu] + step + L[mu]) % L[mu];
    return site_index(L, x);
}

/* Blocks (SAP domains or aggregates): extents b[mu], block coordinate
 * floor(x_mu / b_mu), numbered lexicographically like sites. */
static void block_counts(const int *L, const int *b, int *nb)
{
    for (int mu = 0; mu < 4; ++mu) nb[mu] = L[mu] / b[mu];
}

static long block_of(const int *L, const int *b, long s)
{
    int x[4], nb[4], c[4];
    site_coords(L, s, x);
    block_counts(L, b, nb);
    for (int mu = 0; mu < 4; ++mu) c[mu] = x[mu] / b[mu];
    return site_index(nb, c);
}

static int block_colour(const int *L, const int *b, long j)
{
    int nb[4], c[4];
    block_counts(L, b, nb);
    site_coords(nb, j, c);
    return (c[0] + c[1] + c[2] + c[3]) % 2;
}

/* k-th site, in lexicographic order of local coordinates, of block j */
static long block_site(const int *L, const int *b, long j, long k)
{
    int nb[4], c[4], y[4], x[4];
    block_counts(L, b, nb);
    site_coords(nb, j, c);
    site_coords(b, k, y);
    for (int mu = 0; mu < 4; ++mu) x[mu] = c[mu] * b[mu] + y[mu];
    return site_index(L, x);
}

/* local lexicographic index of site s inside its block */
static long local_index(const int *L, const int *b, long s)
{
    int x[4], y[4];
    site_coords(L, s, x);
    for (int mu = 0; mu < 4; ++mu) y[mu] = x[mu] % b[mu];
    return site_index(b, y);
}

/* ------------------------------------------------------------------------ */
/* Gamma matrices, DeGrand-Rossi chiral basis (g5 = g0 g1 g2 g3 = diag(1,1,-1,-1)) */
/* ------------------------------------------------------------------------ */

static const cplx GAMMA[4][4][4] = {
    {{0, 0, 0, I}, {0, 0, I, 0}, {0, -I, 0, 0}, {-I, 0, 0, 0}},
    {{0, 0, 0, -1}, {0, 0, 1, 0}, {0, 1, 0, 0}, {-1, 0, 0, 0}},
    {{0, 0, I, 0}, {0, 0, 0, -I}, {-I, 0, 0, 0}, {0, I, 0, 0}},
    {{0, 0, 1, 0}, {0, 0, 0, 1}, {1, 0, 0, 0}, {0, 1, 0, 0}},
};

/* out = g_mu (mu = 0..3), or g5 = g0 g1 g2 g3 (mu = 4); 4x4 row-major */
int oracle_gamma(int mu, double *out_)
{
    cplx *out = (cplx *)out_;
    if (mu < 0 || mu > 4) return -1;
    if (mu < 4) {
        memcpy(out, GAMMA[mu], sizeof(GAMMA[mu]));
        return 0;
    }
    cplx acc[4][4], tmp[4][4];
    memcpy(acc, GAMMA[0], sizeof(acc));
    for (int m = 1; m < 4; ++m) {
        for (int r = 0; r < 4; ++r)
            for (int c = 0; c < 4; ++c) {
                cplx s = 0;
                for (int k = 0; k < 4; ++k) s += acc[r][k] * GAMMA[m][k][c];
                tmp[r][c] = s;
            }
        memcpy(acc, tmp, sizeof(acc));
    }
    memcpy(out, acc, sizeof(acc));
    return 0;
}

/* ------------------------------------------------------------------------ */
/* 3x3 colour matrices                                                       */
/* ------------------------------------------------------------------------ */

static const cplx *link(const cplx *U, long V, int mu, long s) { return U + ((long)mu * V + s) * 9; }

static void mat_mul(const cplx *a, const cplx *b, cplx *c)
{
    cplx t[9];
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) {
            cplx s = 0;
            for (int j = 0; j < 3; ++j) s += a[3 * r + j] * b[3 * j + k];
            t[3 * r + k] = s;
        }
    memcpy(c, t, sizeof(t));
}

static void mat_dag(const cplx *a, cplx *c)
{
    cplx t[9];
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) t[3 * r + k] = conj(a[3 * k + r]);
    memcpy(c, t, sizeof(t));
}

/* product of four colour matrices, each optionally daggered */
static void path4(const cplx *m0, int d0, const cplx *m1, int d1, const cplx *m2, int d2,
                  const cplx *m3, int d3, cplx *out)
{
    cplx a[9], b[9];
    if (d0) mat_dag(m0, a); else memcpy(a, m0, sizeof(a));
    if (d1) mat_dag(m1, b); else memcpy(b, m1, sizeof(b));
    mat_mul(a, b, a);
    if (d2) mat_dag(m2, b); else memcpy(b, m2, sizeof(b));
    mat_mul(a, b, a);
    if (d3) mat_dag(m3, b); else memcpy(b, m3, sizeof(b));
    mat_mul(a, b, out);
}

/* Q_munu(x): the four plaquettes in the (mu,nu) plane that start and end at x,
 * all traversed in the same (mu then nu) orientation. */
static void clover_leaves(const int *L, const cplx *U, long x, int mu, int nu, cplx *Q)
{
    long V = volume(L);
    long xpm = neighbour(L, x, mu, +1), xmm = neighbour(L, x, mu, -1);
    long xpn = neighbour(L, x, nu, +1), xmn = neighbour(L, x, nu, -1);
    long xmm_pn = neighbour(L, xmm, nu, +1);
    long xmm_mn = neighbour(L, xmm, nu, -1);
    long xpm_mn = neighbour(L, xpm, nu, -1);
    cplx leaf[9];
    for (int i = 0; i < 9; ++i) Q[i] = 0;
    /* x -> x+mu -> x+mu+nu -> x+nu -> x */
    path4(link(U, V, mu, x), 0, link(U, V, nu, xpm), 0, link(U, V, mu, xpn), 1, link(U, V, nu, x), 1, leaf);
    for (int i = 0; i < 9; ++i) Q[i] += leaf[i];
    /* x -> x+nu -> x+nu-mu -> x-mu -> x */
    path4(link(U, V, nu, x), 0, link(U, V, mu, xmm_pn), 1, link(U, V, nu, xmm), 1, link(U, V, mu, xmm), 0, leaf);
    for (int i = 0; i < 9; ++i) Q[i] += leaf[i];
    /* x -> x-mu -> x-mu-nu -> x-nu -> x */
    path4(link(U, V, mu, xmm), 1, link(U, V, nu, xmm_mn), 1, link(U, V, mu, xmm_mn), 0, link(U, V, nu, xmn), 0, leaf);
    for (int i = 0; i < 9; ++i) Q[i] += leaf[i];
    /* x -> x-nu -> x-nu+mu -> x+mu -> x */
    path4(link(U, V, nu, xmn), 1, link(U, V, mu, xmn), 0, link(U, V, nu, xpm_mn), 0, link(U, V, mu, x), 1, leaf);
    for (int i = 0; i < 9; ++i) Q[i] += leaf[i];
}

/* The site-diagonal term A(x) = (4 + m0) 1 + C(x) as a full 12x12 matrix per site,
 * index 3*spin + colour, row-major: A[(s*12 + row)*12 + col]. */
void oracle_clover(const int *L, const double *U_, double csw, double m0, double *A_)
{
    const cplx *U = (const cplx *)U_;
    cplx *A = (cplx *)A_;
    long V = volume(L);
#pragma omp parallel for schedule(static)
    for (long x = 0; x < V; ++x) {
        cplx *a = A + x * 144;
        for (int i = 0; i < 144; ++i) a[i] = 0;
        for (int i = 0; i < 12; ++i) a[13 * i] = 4.0 + m0;
        for (int mu = 0; mu < 4; ++mu)
            for (int nu = mu + 1; nu < 4; ++nu) {
                cplx Q[9], F[9], G[4][4];
                clover_leaves(L, U, x, mu, nu, Q);
                for (int r = 0; r < 3; ++r)
                    for (int c = 0; c < 3; ++c) F[3 * r + c] = Q[3 * r + c] - conj(Q[3 * c + r]);
                for (int r = 0; r < 4; ++r)
                    for (int c = 0; c < 4; ++c) {
                        cplx s = 0;
                        for (int k = 0; k < 4; ++k) s += GAMMA[mu][r][k] * GAMMA[nu][k][c];
                        G[r][c] = s;
                    }
                for (int sr = 0; sr < 4; ++sr)
                    for (int sc = 0; sc < 4; ++sc)
                        for (int cr = 0; cr < 3; ++cr)
                            for (int cc = 0; cc < 3; ++cc)
                                a[(3 * sr + cr) * 12 + 3 * sc + cc] += -(csw / 16.0) * G[sr][sc] * F[3 * cr + cc];
            }
    }
}

/* ------------------------------------------------------------------------ */
/* Wilson-clover operator                                                    */
/* ------------------------------------------------------------------------ */

/* out += coef * (1 + sign * g_mu) W psi, W a colour matrix (optionally daggered) */
static void hop_term(int mu, int sign, const cplx *W, int dag, const cplx *psi, cplx coef, cplx *out)
{
    cplx Wpsi[12];
    for (int sp = 0; sp < 4; ++sp)
        for (int r = 0; r < 3; ++r) {
            cplx s = 0;
            for (int c = 0; c < 3; ++c) s += (dag ? conj(W[3 * c + r]) : W[3 * r + c]) * psi[3 * sp + c];
            Wpsi[3 * sp + r] = s;
        }
    for (int sr = 0; sr < 4; ++sr)
        for (int sc = 0; sc < 4; ++sc) {
            cplx m = (sr == sc ? 1.0 : 0.0) + sign * GAMMA[mu][sr][sc];
            if (m == 0) continue;
            for (int c = 0; c < 3; ++c) out[3 * sr + c] += coef * m * Wpsi[3 * sc + c];
        }
}

/* Which hops a site update keeps. */
enum { HOPS_ALL = 0, HOPS_SAME_BLOCK = 1, HOPS_INSIDE = 2 };

/* One site of D.  keep = HOPS_ALL: the full periodic operator.
 * HOPS_SAME_BLOCK: only hops to sites of the same block (the block operator
 *   D_j = I_j^T D I_j, which keeps a wrap-around hop when the block spans the
 *   whole lattice in that direction).
 * HOPS_INSIDE: only hops that do not cross a block face (x_mu mod b_mu stays in
 *   range without wrapping): the self-coupling of an aggregate.
 * psi_at(s) gives the input spinor at a lattice site. */
typedef const cplx *(*spinor_fn)(const void *ctx, long s);

static void dirac_site(const int *L, const cplx *U, const cplx *A, long x, int keep, const int *b,
                       spinor_fn psi_at, const void *ctx, cplx *out)
{
    long V = volume(L);
    const cplx *a = A + x * 144;
    const cplx *px = psi_at(ctx, x);
    for (int r = 0; r < 12; ++r) {
        cplx s = 0;
        for (int c = 0; c < 12; ++c) s += a[r * 12 + c] * px[c];
        out[r] = s;
    }
    int xc[4];
    site_coords(L, x, xc);
    long bx = (keep == HOPS_SAME_BLOCK) ? block_of(L, b, x) : -1;
    for (int mu = 0; mu < 4; ++mu) {
        long xf = neighbour(L, x, mu, +1), xb = neighbour(L, x, mu, -1);
        int use_f = 1, use_b = 1;
        if (keep == HOPS_SAME_BLOCK) {
            use_f = block_of(L, b, xf) == bx;
            use_b = block_of(L, b, xb) == bx;
        } else if (keep == HOPS_INSIDE) {
            use_f = (xc[mu] % b[mu]) != b[mu] - 1;
            use_b = (xc[mu] % b[mu]) != 0;
        }
        if (use_f) hop_term(mu, -1, link(U, V, mu, x), 0, psi_at(ctx, xf), -0.5, out);
        if (use_b) hop_term(mu, +1, link(U, V, mu, xb), 1, psi_at(ctx, xb), -0.5, out);
    }
}

static const cplx *full_lattice_spinor(const void *ctx, long s) { return (const cplx *)ctx + 12 * s; }

/* out = D in, for n_rhs vectors, each [V][12] complex */
void oracle_dirac(const int *L, const double *U_, const double *A_, const double *in_, double *out_, int n_rhs)
{
    const cplx *U = (const cplx *)U_, *A = (const cplx *)A_;
    long V = volume(L);
    for (int k = 0; k < n_rhs; ++k) {
        const cplx *in = (const cplx *)in_ + (long)k * 12 * V;
        cplx *out = (cplx *)out_ + (long)k * 12 * V;
#pragma omp parallel for schedule(static)
        for (long x = 0; x < V; ++x) dirac_site(L, U, A, x, HOPS_ALL, NULL, full_lattice_spinor, in, out + 12 * x);
    }
}

/* out = (sum_j I_j D_j I_j^T) in: D with every hop between different blocks dropped */
void oracle_block_dirac(const int *L, const int *b, const double *U_, const double *A_, const double *in_,
                        double *out_, int n_rhs)
{
    const cplx *U = (const cplx *)U_, *A = (const cplx *)A_;
    long V = volume(L);
    for (int k = 0; k < n_rhs; ++k) {
        const cplx *in = (const cplx *)in_ + (long)k * 12 * V;
        cplx *out = (cplx *)out_ + (long)k * 12 * V;
#pragma omp parallel for schedule(static)
        for (long x = 0; x < V; ++x) dirac_site(L, U, A, x, HOPS_SAME_BLOCK, b, full_lattice_spinor, in, out + 12 * x);
    }
}

/* ------------------------------------------------------------------------ */
/* Minimal residual on one block                                             */
/* ------------------------------------------------------------------------ */

typedef struct {
    const int *L, *b;
    long j;
    const cplx *local; /* block-local vector [Vb][12] */
} block_ctx;

/* spinor of a block-local vector at lattice site s (s must lie in the block) */
static const cplx *block_spinor(const void *ctx_, long s)
{
    const block_ctx *ctx = (const block_ctx *)ctx_;
    return ctx->local + 12 * local_index(ctx->L, ctx->b, s);
}

/* q = D_j rho on block j, both block-local [Vb][12] */
static void block_op(const int *L, const int *b, const cplx *U, const cplx *A, long j, const cplx *rho, cplx *q)
{
    long Vb = (long)b[0] * b[1] * b[2] * b[3];
    block_ctx ctx = {L, b, j, rho};
    for (long k = 0; k < Vb; ++k) {
        long x = block_site(L, b, j, k);
        dirac_site(L, U, A, x, HOPS_SAME_BLOCK, b, block_spinor, &ctx, q + 12 * k);
    }
}

/* Minimal residual for D_j e = r on block j, fixed n_mr steps from e = 0:
 *   q = D_j rho, alpha = <q,rho>/<q,q> (0 if <q,q> = 0), e += alpha rho, rho -= alpha q.
 * r, e block-local; rho_norms (nullable) receives ||rho|| before each step and after the last. */
static void mr_block(const int *L, const int *b, const cplx *U, const cplx *A, long j, const cplx *r, int n_mr,
                     cplx *e, double *rho_norms)
{
    long n = 12L * b[0] * b[1] * b[2] * b[3];
    cplx *rho = malloc(n * sizeof(cplx)), *q = malloc(n * sizeof(cplx));
    for (long i = 0; i < n; ++i) { e[i] = 0; rho[i] = r[i]; }
    for (int it = 0; it < n_mr; ++it) {
        if (rho_norms) {
            double s = 0;
            for (long i = 0; i < n; ++i) s += creal(conj(rho[i]) * rho[i]);
            rho_norms[it] = sqrt(s);
        }
        block_op(L, b, U, A, j, rho, q);
        double qq = 0;
        cplx qr = 0;
        for (long i = 0; i < n; ++i) {
            qq += creal(conj(q[i]) * q[i]);
            qr += conj(q[i]) * rho[i];
        }
        cplx alpha = qq > 0 ? qr / qq : 0;
        for (long i = 0; i < n; ++i) {
            e[i] += alpha * rho[i];
            rho[i] -= alpha * q[i];
        }
    }
    if (rho_norms) {
        double s = 0;
        for (long i = 0; i < n; ++i) s += creal(conj(rho[i]) * rho[i]);
        rho_norms[n_mr] = sqrt(s);
    }
    free(rho);
    free(q);
}

/* MR on block j for one full-lattice residual r; e (full lattice) receives the
 * block solution on block j and zero elsewhere. */
void oracle_mr(const int *L, const int *b, const double *U_, const double *A_, long j, const double *r_, int n_mr,
               double *e_, double *rho_norms)
{
    const cplx *U = (const cplx *)U_, *A = (const cplx *)A_, *r = (const cplx *)r_;
    cplx *e = (cplx *)e_;
    long V = volume(L), Vb = (long)b[0] * b[1] * b[2] * b[3];
    cplx *rl = malloc(12 * Vb * sizeof(cplx)), *el = malloc(12 * Vb * sizeof(cplx));
    for (long k = 0; k < Vb; ++k) {
        long x = block_site(L, b, j, k);
        for (int c = 0; c < 12; ++c) rl[12 * k + c] = r[12 * x + c];
    }
    mr_block(L, b, U, A, j, rl, n_mr, el, rho_norms);
    for (long i = 0; i < 12 * V; ++i) e[i] = 0;
    for (long k = 0; k < Vb; ++k) {
        long x = block_site(L, b, j, k);
        for (int c = 0; c < 12; ++c) e[12 * x + c] = el[12 * k + c];
    }
    free(rl);
    free(el);
}

/* ------------------------------------------------------------------------ */
/* Even-odd preconditioned block solve                                       */
/* ------------------------------------------------------------------------ */

/* Parity of a block's k-th site: the sum of its block-local coordinates mod 2.  With every
 * block extent even, each hop inside a block joins sites of opposite parity, so in (even,
 * odd) order the block operator is D_j = [[A_ee, H_eo], [H_oe, A_oo]]: A the site-diagonal
 * clover term, H the hops inside the block.  Then H_oe v_e is the odd part of D_j (v_e, 0)
 * and H_eo u_o the even part of D_j (0, u_o). */
static int local_parity(const int *b, long k)
{
    int y[4];
    site_coords(b, k, y);
    return (y[0] + y[1] + y[2] + y[3]) & 1;
}

/* out_k = M(x_k) in_k at the block's sites of parity p, 0 at the others (M: [V][12][12]) */
static void site_mat(const int *L, const int *b, long j, const cplx *M, int p, const cplx *in, cplx *out)
{
    long Vb = (long)b[0] * b[1] * b[2] * b[3];
    for (long k = 0; k < Vb; ++k) {
        cplx *o = out + 12 * k;
        if (local_parity(b, k) != p) {
            for (int r = 0; r < 12; ++r) o[r] = 0;
            continue;
        }
        const cplx *m = M + block_site(L, b, j, k) * 144, *v = in + 12 * k;
        for (int r = 0; r < 12; ++r) {
            cplx acc = 0;
            for (int c = 0; c < 12; ++c) acc += m[r * 12 + c] * v[c];
            o[r] = acc;
        }
    }
}

/* keep the parity-p part of a block-local vector, zero the rest */
static void keep_parity(const int *b, int p, const cplx *in, cplx *out)
{
    long Vb = (long)b[0] * b[1] * b[2] * b[3];
    for (long k = 0; k < Vb; ++k)
        for (int r = 0; r < 12; ++r) out[12 * k + r] = local_parity(b, k) == p ? in[12 * k + r] : 0;
}

/* q = S v, the Schur complement S = A_ee - H_eo A_oo^-1 H_oe on the even part of v; the odd
 * part of q is zero.  t1, t2: block-local scratch. */
static void schur_op(const int *L, const int *b, const cplx *U, const cplx *A, const cplx *Ainv, long j,
                     const cplx *v, cplx *q, cplx *t1, cplx *t2)
{
    long n = 12L * b[0] * b[1] * b[2] * b[3];
    keep_parity(b, 0, v, t1);
    block_op(L, b, U, A, j, t1, t2);      /* t2 = (A_ee v_e, H_oe v_e) */
    site_mat(L, b, j, Ainv, 1, t2, t1);   /* t1 = (0, A_oo^-1 H_oe v_e) */
    block_op(L, b, U, A, j, t1, q);       /* q_e = H_eo A_oo^-1 H_oe v_e */
    for (long i = 0; i < n; ++i) q[i] = t2[i] - q[i];
    keep_parity(b, 0, q, q);
}

/* D_j e = r on block j by the Schur complement:
 *   rhat_e = r_e - H_eo A_oo^-1 r_o,
 *   n_mr minimal-residual steps on S e_e = rhat_e from e_e = 0 (as in mr_block, S for D_j),
 *   e_o = A_oo^-1 (r_o - H_oe e_e).
 * rho_norms (nullable) receives ||rho_e|| before each step and after the last. */
static void eo_block(const int *L, const int *b, const cplx *U, const cplx *A, const cplx *Ainv, long j,
                     const cplx *r, int n_mr, cplx *e, double *rho_norms)
{
    long n = 12L * b[0] * b[1] * b[2] * b[3];
    cplx *rho = malloc(n * sizeof(cplx)), *q = malloc(n * sizeof(cplx));
    cplx *t1 = malloc(n * sizeof(cplx)), *t2 = malloc(n * sizeof(cplx));
    site_mat(L, b, j, Ainv, 1, r, t1);   /* (0, A_oo^-1 r_o) */
    block_op(L, b, U, A, j, t1, t2);     /* even part: H_eo A_oo^-1 r_o */
    for (long i = 0; i < n; ++i) rho[i] = r[i] - t2[i];
    keep_parity(b, 0, rho, rho);
    for (long i = 0; i < n; ++i) e[i] = 0;
    for (int it = 0; it < n_mr; ++it) {
        if (rho_norms) {
            double s = 0;
            for (long i = 0; i < n; ++i) s += creal(conj(rho[i]) * rho[i]);
            rho_norms[it] = sqrt(s);
        }
        schur_op(L, b, U, A, Ainv, j, rho, q, t1, t2);
        double qq = 0;
        cplx qr = 0;
        for (long i = 0; i < n; ++i) {
            qq += creal(conj(q[i]) * q[i]);
            qr += conj(q[i]) * rho[i];
        }
        cplx alpha = qq > 0 ? qr / qq : 0;
        for (long i = 0; i < n; ++i) {
            e[i] += alpha * rho[i];
            rho[i] -= alpha * q[i];
        }
    }
    if (rho_norms) {
        double s = 0;
        for (long i = 0; i < n; ++i) s += creal(conj(rho[i]) * rho[i]);
        rho_norms[n_mr] = sqrt(s);
    }
    /* odd sites: (D_j (e_e, 0))_o = H_oe e_e */
    block_op(L, b, U, A, j, e, t2);
    for (long i = 0; i < n; ++i) t1[i] = r[i] - t2[i];
    site_mat(L, b, j, Ainv, 1, t1, t2);
    for (long i = 0; i < n; ++i) e[i] += t2[i];
    free(rho);
    free(q);
    free(t1);
    free(t2);
}

static int even_extents(const int *b)
{
    for (int mu = 0; mu < 4; ++mu)
        if (b[mu] % 2) return 0;
    return 1;
}

/* eo_block on block j for one full-lattice residual r; e (full lattice) receives the block
 * solution on block j and zero elsewhere.  Ainv: [V][12][12], the inverse of A per site.
 * Returns -2 if a block extent is odd. */
int oracle_eo_block(const int *L, const int *b, const double *U_, const double *A_, const double *Ainv_, long j,
                    const double *r_, int n_mr, double *e_, double *rho_norms)
{
    if (!even_extents(b)) return -2;
    const cplx *U = (const cplx *)U_, *A = (const cplx *)A_, *Ainv = (const cplx *)Ainv_, *r = (const cplx *)r_;
    cplx *e = (cplx *)e_;
    long V = volume(L), Vb = (long)b[0] * b[1] * b[2] * b[3];
    cplx *rl = malloc(12 * Vb * sizeof(cplx)), *el = malloc(12 * Vb * sizeof(cplx));
    for (long k = 0; k < Vb; ++k) {
        long x = block_site(L, b, j, k);
        for (int c = 0; c < 12; ++c) rl[12 * k + c] = r[12 * x + c];
    }
    eo_block(L, b, U, A, Ainv, j, rl, n_mr, el, rho_norms);
    for (long i = 0; i < 12 * V; ++i) e[i] = 0;
    for (long k = 0; k < Vb; ++k) {
        long x = block_site(L, b, j, k);
        for (int c = 0; c < 12; ++c) e[12 * x + c] = el[12 * k + c];
    }
    free(rl);
    free(el);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Schwarz alternating procedure                                             */
/* ------------------------------------------------------------------------ */

/* x = SAP(b) from x = 0: n_sap sweeps; each sweep visits colour 0 (red) then
 * colour 1 (black).  Per colour: r = b - D x on the colour's blocks, then every
 * block j of that colour adds MR(D_j, r|_j, n_mr) to x|_j, all from the same r. */
/* SAP from a given starting guess: x_io holds x0 on entry and the result on exit (the
 * refinement phase of the setup, Alg. 1 and 2: the smoother starts from the coarse-grid
 * correction).  oracle_sap below is the start from zero of the initial phase. */
static int sap_from(const int *L, const int *b, const double *U_, const double *A_, const double *Ainv_,
                    const double *b_in_, double *x_io_, int n_rhs, int n_sap, int n_mr)
{
    const cplx *U = (const cplx *)U_, *A = (const cplx *)A_, *Ainv = (const cplx *)Ainv_;
    long V = volume(L), Vb = (long)b[0] * b[1] * b[2] * b[3];
    int nb[4];
    for (int mu = 0; mu < 4; ++mu)
        if (b[mu] < 1 || L[mu] % b[mu] != 0) return -1;
    block_counts(L, b, nb);
    long nblocks = (long)nb[0] * nb[1] * nb[2] * nb[3];
    cplx *r = malloc(12 * V * sizeof(cplx));
    for (int k = 0; k < n_rhs; ++k) {
        const cplx *bv = (const cplx *)b_in_ + (long)k * 12 * V;
        cplx *x = (cplx *)x_io_ + (long)k * 12 * V;
        for (int s = 0; s < n_sap; ++s)
            for (int colour = 0; colour < 2; ++colour) {
#pragma omp parallel for schedule(static)
                for (long xs = 0; xs < V; ++xs) {
                    if (block_colour(L, b, block_of(L, b, xs)) != colour) continue;
                    cplx Dx[12];
                    dirac_site(L, U, A, xs, HOPS_ALL, NULL, full_lattice_spinor, x, Dx);
                    for (int c = 0; c < 12; ++c) r[12 * xs + c] = bv[12 * xs + c] - Dx[c];
                }
#pragma omp parallel for schedule(dynamic)
                for (long j = 0; j < nblocks; ++j) {
                    if (block_colour(L, b, j) != colour) continue;
                    cplx *rl = malloc(12 * Vb * sizeof(cplx)), *el = malloc(12 * Vb * sizeof(cplx));
                    for (long kk = 0; kk < Vb; ++kk) {
                        long xs = block_site(L, b, j, kk);
                        for (int c = 0; c < 12; ++c) rl[12 * kk + c] = r[12 * xs + c];
                    }
                    if (Ainv) eo_block(L, b, U, A, Ainv, j, rl, n_mr, el, NULL);
                    else mr_block(L, b, U, A, j, rl, n_mr, el, NULL);
                    for (long kk = 0; kk < Vb; ++kk) {
                        long xs = block_site(L, b, j, kk);
                        for (int c = 0; c < 12; ++c) x[12 * xs + c] += el[12 * kk + c];
                    }
                    free(rl);
                    free(el);
                }
            }
    }
    free(r);
    return 0;
}

int oracle_sap_from(const int *L, const int *b, const double *U_, const double *A_, const double *b_in_,
                    double *x_io_, int n_rhs, int n_sap, int n_mr)
{
    return sap_from(L, b, U_, A_, NULL, b_in_, x_io_, n_rhs, n_sap, n_mr);
}

/* SAP from a starting guess with the even-odd block solver (eo_block); Ainv: [V][12][12] */
int oracle_sap_from_eo(const int *L, const int *b, const double *U_, const double *A_, const double *Ainv_,
                       const double *b_in_, double *x_io_, int n_rhs, int n_sap, int n_mr)
{
    if (!even_extents(b)) return -2;
    return sap_from(L, b, U_, A_, Ainv_, b_in_, x_io_, n_rhs, n_sap, n_mr);
}

int oracle_sap(const int *L, const int *b, const double *U_, const double *A_, const double *b_in_, double *x_out_,
               int n_rhs, int n_sap, int n_mr)
{
    long V = volume(L);
    for (long i = 0; i < (long)n_rhs * 24 * V; ++i) x_out_[i] = 0;
    return oracle_sap_from(L, b, U_, A_, b_in_, x_out_, n_rhs, n_sap, n_mr);
}

/* rel[k] = ||b_k - D x_k|| / ||b_k|| */
void oracle_residual_norms(const int *L, const double *U_, const double *A_, const double *b_in_, const double *x_,
                           int n_rhs, double *rel)
{
    const cplx *U = (const cplx *)U_, *A = (const cplx *)A_;
    long V = volume(L);
    for (int k = 0; k < n_rhs; ++k) {
        const cplx *bv = (const cplx *)b_in_ + (long)k * 12 * V;
        const cplx *x = (const cplx *)x_ + (long)k * 12 * V;
        double num = 0, den = 0;
#pragma omp parallel for reduction(+ : num, den) schedule(static)
        for (long xs = 0; xs < V; ++xs) {
            cplx Dx[12];
            dirac_site(L, U, A, xs, HOPS_ALL, NULL, full_lattice_spinor, x, Dx);
            for (int c = 0; c < 12; ++c) {
                cplx d = bv[12 * xs + c] - Dx[c];
                num += creal(conj(d) * d);
                den += creal(conj(bv[12 * xs + c]) * bv[12 * xs + c]);
            }
        }
        rel[k] = sqrt(num) / sqrt(den);
    }
}

/* ------------------------------------------------------------------------ */
/* Aggregates: block Gram-Schmidt, restriction, prolongation, coarse operator */
/* ------------------------------------------------------------------------ */

/* Row n of the aggregate-half matrix V^h_i: (local site k, spin s' in {0,1}, colour c),
 * n = 6k + 3s' + c; it holds component 3(2h + s') + c of lattice site k of aggregate i. */
static long agg_elem(const int *L, const int *a, long i, int h, long n)
{
    long k = n / 6;
    int sp = (int)((n % 6) / 3), c = (int)(n % 3);
    long x = block_site(L, a, i, k);
    return 12 * x + 3 * (2 * h + sp) + c;
}

/* In: V = n_tv vectors [n_tv][V][12].  Out: Q (same shape) with, for every aggregate i
 * and half h, V^h_i = Q^h_i T^h_i, (Q^h_i)^dag Q^h_i = 1, T upper triangular with real
 * positive diagonal.  T_out (nullable): [n_agg][2][n_tv][n_tv] row-major.
 * Returns 0, -1 for bad geometry, or 1 + (aggregate*2 + h) of the first rank-deficient
 * block (T_kk <= 1e-12 * ||v_k||). */
int oracle_block_gs(const int *L, const int *a, const double *V_, int n_tv, double *Q_, double *T_out_)
{
    const cplx *Vin = (const cplx *)V_;
    cplx *Q = (cplx *)Q_, *T_out = (cplx *)T_out_;
    long V = volume(L);
    int na[4];
    for (int mu = 0; mu < 4; ++mu)
        if (a[mu] < 1 || L[mu] % a[mu] != 0) return -1;
    block_counts(L, a, na);
    long n_agg = (long)na[0] * na[1] * na[2] * na[3];
    long rows = 6L * a[0] * a[1] * a[2] * a[3];
    int status = 0;
#pragma omp parallel for schedule(dynamic)
    for (long ih = 0; ih < 2 * n_agg; ++ih) {
        long i = ih / 2;
        int h = (int)(ih % 2);
        cplx *M = malloc(rows * n_tv * sizeof(cplx)); /* column k at M + k*rows */
        cplx *T = calloc((size_t)n_tv * n_tv, sizeof(cplx));
        for (int k = 0; k < n_tv; ++k)
            for (long n = 0; n < rows; ++n) M[k * rows + n] = Vin[(long)k * 12 * V + agg_elem(L, a, i, h, n)];
        for (int k = 0; k < n_tv; ++k) {
            cplx *v = M + k * rows;
            double norm0 = 0;
            for (long n = 0; n < rows; ++n) norm0 += creal(conj(v[n]) * v[n]);
            norm0 = sqrt(norm0);
            for (int pass = 0; pass < 2; ++pass)
                for (int j = 0; j < k; ++j) {
                    const cplx *qj = M + j * rows;
                    cplx c = 0;
                    for (long n = 0; n < rows; ++n) c += conj(qj[n]) * v[n];
                    for (long n = 0; n < rows; ++n) v[n] -= c * qj[n];
                    T[j * n_tv + k] += c;
                }
            double nk = 0;
            for (long n = 0; n < rows; ++n) nk += creal(conj(v[n]) * v[n]);
            nk = sqrt(nk);
            if (!(nk > 1e-12 * norm0)) {
#pragma omp critical
                if (status == 0 || 1 + ih < status) status = (int)(1 + ih);
                nk = nk > 0 ? nk : 1.0;
            }
            T[k * n_tv + k] = nk;
            for (long n = 0; n < rows; ++n) v[n] /= nk;
        }
        for (int k = 0; k < n_tv; ++k)
            for (long n = 0; n < rows; ++n) Q[(long)k * 12 * V + agg_elem(L, a, i, h, n)] = M[k * rows + n];
        if (T_out)
            for (int r = 0; r < n_tv * n_tv; ++r) T_out[ih * n_tv * n_tv + r] = T[r];
        free(M);
        free(T);
    }
    return status;
}

/* Coarse vectors: [n_rhs][Vc][2][n_tv] complex, coarse dof index h*n_tv + k,
 * coarse sites numbered lexicographically like fine sites. */

/* y_c = R y with R = Q^dag per aggregate and half (Alg. 3 of Sec. 5): the entry j of
 * column n of R^h_i is conj(Q^h_i[n, j]). */
void oracle_restrict(const int *L, const int *a, const double *Q_, int n_tv, const double *y_, double *yc_, int n_rhs)
{
    const cplx *Qv = (const cplx *)Q_;
    long V = volume(L);
    int na[4];
    block_counts(L, a, na);
    long n_agg = (long)na[0] * na[1] * na[2] * na[3];
    long rows = 6L * a[0] * a[1] * a[2] * a[3];
    for (int r = 0; r < n_rhs; ++r) {
        const cplx *y = (const cplx *)y_ + (long)r * 12 * V;
        cplx *yc = (cplx *)yc_ + (long)r * n_agg * 2 * n_tv;
#pragma omp parallel for schedule(static)
        for (long i = 0; i < n_agg; ++i)
            for (int h = 0; h < 2; ++h)
                for (int j = 0; j < n_tv; ++j) {
                    cplx s = 0;
                    for (long n = 0; n < rows; ++n) {
                        long e = agg_elem(L, a, i, h, n);
                        s += conj(Qv[(long)j * 12 * V + e]) * y[e];
                    }
                    yc[(i * 2 + h) * n_tv + j] = s;
                }
    }
}

/* y = P y_c with P = Q: y^h_i[n] = sum_j Q^h_i[n, j] (y_c)^h_i[j] */
void oracle_prolong(const int *L, const int *a, const double *Q_, int n_tv, const double *yc_, double *y_, int n_rhs)
{
    const cplx *Qv = (const cplx *)Q_;
    long V = volume(L);
    int na[4];
    block_counts(L, a, na);
    long n_agg = (long)na[0] * na[1] * na[2] * na[3];
    long rows = 6L * a[0] * a[1] * a[2] * a[3];
    for (int r = 0; r < n_rhs; ++r) {
        const cplx *yc = (const cplx *)yc_ + (long)r * n_agg * 2 * n_tv;
        cplx *y = (cplx *)y_ + (long)r * 12 * V;
#pragma omp parallel for schedule(static)
        for (long i = 0; i < n_agg; ++i)
            for (int h = 0; h < 2; ++h)
                for (long n = 0; n < rows; ++n) {
                    long e = agg_elem(L, a, i, h, n);
                    cplx s = 0;
                    for (int j = 0; j < n_tv; ++j) s += Qv[(long)j * 12 * V + e] * yc[(i * 2 + h) * n_tv + j];
                    y[e] = s;
                }
    }
}

/* The part of D that maps aggregate 'src' onto site x of aggregate i:
 * which = 0: site term plus the hops that stay inside aggregate i without crossing
 *            one of its faces;
 * which = 1+mu: the hop from x across the +mu face of aggregate i;
 * which = 5+mu: the hop from x across the -mu face of aggregate i.
 * out = that part applied to psi (a full-lattice vector). */
static void coarse_part(const int *L, const int *a, const cplx *U, const cplx *A, long x, int which, const cplx *psi,
                        cplx *out)
{
    long V = volume(L);
    int xc[4];
    site_coords(L, x, xc);
    for (int c = 0; c < 12; ++c) out[c] = 0;
    if (which == 0) {
        dirac_site(L, U, A, x, HOPS_INSIDE, a, full_lattice_spinor, psi, out);
        return;
    }
    int mu = (which - 1) % 4, fwd = which <= 4;
    if (fwd) {
        if (xc[mu] % a[mu] != a[mu] - 1) return;
        hop_term(mu, -1, link(U, V, mu, x), 0, psi + 12 * neighbour(L, x, mu, +1), -0.5, out);
    } else {
        if (xc[mu] % a[mu] != 0) return;
        long xb = neighbour(L, x, mu, -1);
        hop_term(mu, +1, link(U, V, mu, xb), 1, psi + 12 * xb, -0.5, out);
    }
}

/* Coarse operator D_c = R D P, stored per coarse site i as 9 blocks
 * [self, +x, +y, +z, +t, -x, -y, -z, -t], each 2 n_tv x 2 n_tv row-major complex,
 * row = h*n_tv + k (output dof), column = h'*n_tv + k' (input dof):
 *   Dc[i][d][(h,k)][(h',k')] = sum_{x in i} <mask_h q_k(x), part_d(mask_h' q_k')(x)>.
 * agg_list (nullable): only these coarse sites are computed (their output slots are
 * written at their own positions in Dc). */
void oracle_coarse_op(const int *L, const int *a, const double *U_, const double *A_, const double *Q_, int n_tv,
                      double *Dc_, const long *agg_list, long n_list)
{
    const cplx *U = (const cplx *)U_, *A = (const cplx *)A_, *Qv = (const cplx *)Q_;
    cplx *Dc = (cplx *)Dc_;
    long V = volume(L), Va = (long)a[0] * a[1] * a[2] * a[3];
    int na[4];
    block_counts(L, a, na);
    long n_agg = (long)na[0] * na[1] * na[2] * na[3];
    long nc = 2L * n_tv;
    long count = agg_list ? n_list : n_agg;
    /* column vectors mask_h' q_k' as full-lattice vectors */
    cplx *P = malloc(nc * 12 * V * sizeof(cplx));
    for (int hp = 0; hp < 2; ++hp)
        for (int kp = 0; kp < n_tv; ++kp) {
            cplx *p = P + (hp * n_tv + kp) * 12 * V;
            const cplx *q = Qv + (long)kp * 12 * V;
            for (long x = 0; x < V; ++x)
                for (int s = 0; s < 4; ++s)
                    for (int c = 0; c < 3; ++c) p[12 * x + 3 * s + c] = (s / 2 == hp) ? q[12 * x + 3 * s + c] : 0;
        }
#pragma omp parallel for schedule(dynamic)
    for (long t = 0; t < count; ++t) {
        long i = agg_list ? agg_list[t] : t;
        for (int d = 0; d < 9; ++d) {
            cplx *blk = Dc + (i * 9 + d) * nc * nc;
            for (long e = 0; e < nc * nc; ++e) blk[e] = 0;
            for (long col = 0; col < nc; ++col) {
                const cplx *p = P + col * 12 * V;
                for (long k = 0; k < Va; ++k) {
                    long x = block_site(L, a, i, k);
                    cplx w[12];
                    coarse_part(L, a, U, A, x, d, p, w);
                    for (int h = 0; h < 2; ++h)
                        for (int kk = 0; kk < n_tv; ++kk) {
                            const cplx *q = Qv + (long)kk * 12 * V + 12 * x;
                            cplx s = 0;
                            for (int sp = 2 * h; sp < 2 * h + 2; ++sp)
                                for (int c = 0; c < 3; ++c) s += conj(q[3 * sp + c]) * w[3 * sp + c];
                            blk[(h * n_tv + kk) * nc + col] += s;
                        }
                }
            }
        }
    }
    free(P);
}

/* y_out = D_c y_in on the coarse lattice (the coarse-grid operator applied in the coarse
 * solve of the setup's refinement phase, Alg. 1): per coarse site i,
 *   y_out(i) = Dc[i][self] y_in(i) + sum_mu ( Dc[i][+mu] y_in(i+mu) + Dc[i][-mu] y_in(i-mu) ),
 * neighbours periodic on the coarse lattice L/a (coinciding neighbours are separate
 * terms).  Coarse vectors [n_rhs][Vc][2 n_tv] complex, blocks [Vc][9][2 n_tv][2 n_tv]. */
void oracle_coarse_apply(const int *L, const int *a, const double *Dc_, int n_tv, const double *yin_, double *yout_,
                         int n_rhs)
{
    const cplx *Dc = (const cplx *)Dc_;
    int na[4];
    block_counts(L, a, na);
    long Vc = (long)na[0] * na[1] * na[2] * na[3];
    int nc = 2 * n_tv;
    for (int r = 0; r < n_rhs; ++r) {
        const cplx *yin = (const cplx *)yin_ + (long)r * Vc * nc;
        cplx *yout = (cplx *)yout_ + (long)r * Vc * nc;
#pragma omp parallel for schedule(static)
        for (long i = 0; i < Vc; ++i) {
            int c[4];
            long rem = i;
            for (int mu = 0; mu < 4; ++mu) {
                c[mu] = (int)(rem % na[mu]);
                rem /= na[mu];
            }
            for (int row = 0; row < nc; ++row) yout[i * nc + row] = 0;
            for (int d = 0; d < 9; ++d) {
                int cn[4] = {c[0], c[1], c[2], c[3]};
                if (d >= 1 && d <= 4) cn[d - 1] = (cn[d - 1] + 1) % na[d - 1];
                if (d >= 5) cn[d - 5] = (cn[d - 5] - 1 + na[d - 5]) % na[d - 5];
                long j = cn[0] + (long)na[0] * (cn[1] + (long)na[1] * (cn[2] + (long)na[2] * cn[3]));
                const cplx *blk = Dc + (i * 9 + d) * nc * nc;
                for (int row = 0; row < nc; ++row) {
                    cplx s = 0;
                    for (int col = 0; col < nc; ++col) s += blk[row * nc + col] * yin[j * nc + col];
                    yout[i * nc + row] += s;
                }
            }
        }
    }
}

/* u = approximate D_c^-1 b on the coarse lattice (the low-accuracy coarse solve of the
 * refinement phase, Alg. 1), per right-hand side: GMRES from a zero start, at most m
 * iterations, Arnoldi with classical Gram-Schmidt applied twice, complex Givens rotations
 * (c real) on the Hessenberg matrix; a right-hand side stops once its residual estimate
 * |g_{j+1}| falls to tol * ||b|| (tol = 0: exactly m iterations, or fewer on breakdown).
 * res_out[k] (nullable) = final |g_J| / ||b||, iters_out[k] (nullable) = J.
 * Coarse vectors [n_rhs][Vc][2 n_tv]. */
/* one right-hand side of the GMRES described above, for the operator apply(ctx, in, out) on
 * vectors of dim complex entries */
typedef void (*coarse_op_fn)(const void *ctx, const cplx *in, cplx *out);

static void gmres_one(long dim, coarse_op_fn apply, const void *ctx, const cplx *b, cplx *u, int m, double tol,
                      double *res, int *iters)
{
        cplx *Vb = calloc((size_t)(m + 1) * dim, sizeof(cplx));
        cplx *w = malloc(dim * sizeof(cplx));
        cplx *H = calloc((size_t)(m + 1) * m, sizeof(cplx)); /* H[i][j] at i * m + j */
        cplx *g = calloc((size_t)(m + 1), sizeof(cplx)), *sn = calloc((size_t)m, sizeof(cplx));
        double *cs = calloc((size_t)m, sizeof(double));
        double beta = 0;
        for (long e = 0; e < dim; ++e) beta += creal(conj(b[e]) * b[e]);
        beta = sqrt(beta);
        for (long e = 0; e < dim; ++e) u[e] = 0;
        int J = 0;
        double est = beta;
        if (beta > 0) {
            for (long e = 0; e < dim; ++e) Vb[e] = b[e] / beta;
            g[0] = beta;
            for (int j = 0; j < m; ++j) {
                if (!(est > tol * beta)) break;
                apply(ctx, Vb + (long)j * dim, w);
                for (int pass = 0; pass < 2; ++pass) {
                    cplx h[65];
                    for (int i = 0; i <= j; ++i) {
                        cplx s = 0;
                        for (long e = 0; e < dim; ++e) s += conj(Vb[(long)i * dim + e]) * w[e];
                        h[i] = s;
                    }
                    for (int i = 0; i <= j; ++i) {
                        for (long e = 0; e < dim; ++e) w[e] -= h[i] * Vb[(long)i * dim + e];
                        H[(long)i * m + j] += h[i];
                    }
                }
                double nw = 0;
                for (long e = 0; e < dim; ++e) nw += creal(conj(w[e]) * w[e]);
                nw = sqrt(nw);
                H[(long)(j + 1) * m + j] = nw;
                if (nw > 0)
                    for (long e = 0; e < dim; ++e) Vb[(long)(j + 1) * dim + e] = w[e] / nw;
                /* earlier rotations on column j, then a new one that zeroes H[j+1][j] */
                for (int i = 0; i < j; ++i) {
                    cplx x0 = H[(long)i * m + j], x1 = H[(long)(i + 1) * m + j];
                    H[(long)i * m + j] = cs[i] * x0 + sn[i] * x1;
                    H[(long)(i + 1) * m + j] = -conj(sn[i]) * x0 + cs[i] * x1;
                }
                cplx hj = H[(long)j * m + j];
                double ah = cabs(hj), rho = sqrt(ah * ah + nw * nw);
                if (ah == 0) {
                    cs[j] = 0;
                    sn[j] = 1;
                } else {
                    cs[j] = ah / rho;
                    sn[j] = (hj / ah) * nw / rho;
                }
                H[(long)j * m + j] = cs[j] * hj + sn[j] * nw;
                H[(long)(j + 1) * m + j] = 0;
                g[j + 1] = -conj(sn[j]) * g[j];
                g[j] = cs[j] * g[j];
                est = cabs(g[j + 1]);
                J = j + 1;
                if (!(nw > 0)) break; /* invariant subspace: the solution is exact */
            }
            /* H[0..J)[0..J) y = g[0..J), back substitution; u = sum y_i V_i */
            cplx y[64];
            for (int i = J - 1; i >= 0; --i) {
                cplx s = g[i];
                for (int l = i + 1; l < J; ++l) s -= H[(long)i * m + l] * y[l];
                y[i] = s / H[(long)i * m + i];
            }
            for (int i = 0; i < J; ++i)
                for (long e = 0; e < dim; ++e) u[e] += y[i] * Vb[(long)i * dim + e];
        }
        if (res) *res = beta > 0 ? est / beta : 0;
        if (iters) *iters = J;
        free(Vb);
        free(w);
        free(H);
        free(g);
        free(sn);
        free(cs);
}

typedef struct {
    const int *L, *a;
    const double *Dc;
    int n_tv;
} coarse_ctx;

static void dc_apply(const void *ctx_, const cplx *in, cplx *out)
{
    const coarse_ctx *c = (const coarse_ctx *)ctx_;
    oracle_coarse_apply(c->L, c->a, c->Dc, c->n_tv, (const double *)in, (double *)out, 1);
}

void oracle_coarse_gmres(const int *L, const int *a, const double *Dc_, int n_tv, const double *b_, double *u_,
                         int n_rhs, int m, double tol, double *res_out, int *iters_out)
{
    int na[4];
    block_counts(L, a, na);
    long dim = (long)na[0] * na[1] * na[2] * na[3] * 2 * n_tv;
    coarse_ctx ctx = {L, a, Dc_, n_tv};
    for (int k = 0; k < n_rhs; ++k)
        gmres_one(dim, dc_apply, &ctx, (const cplx *)b_ + (long)k * dim, (cplx *)u_ + (long)k * dim, m, tol,
                  res_out ? res_out + k : NULL, iters_out ? iters_out + k : NULL);
}

/* ------------------------------------------------------------------------ */
/* Even-odd preconditioned coarse solve                                      */
/* ------------------------------------------------------------------------ */

/* Coarse sites split by the parity of their coordinate sum.  With every coarse extent even,
 * each of the 8 hop blocks joins sites of opposite parity, so in (even, odd) order
 * D_c = [[A_ee, H_eo], [H_oe, A_oo]], A the self blocks and H the hop blocks: H_oe v_e is the
 * odd part of D_c (v_e, 0) and H_eo u_o the even part of D_c (0, u_o).  Ainv: [Vc][2 n_tv]^2,
 * the inverse of each self block (only the odd sites' are used). */
typedef struct {
    coarse_ctx c;
    const cplx *Ainv;
    long Vc;
    int nc;
    const int *par;
    cplx *t1, *t2;
} eo_coarse_ctx;

/* out = in on the sites of parity p, 0 on the others */
static void keep_coarse_parity(const eo_coarse_ctx *e, int p, const cplx *in, cplx *out)
{
    for (long i = 0; i < e->Vc; ++i)
        for (int r = 0; r < e->nc; ++r) out[i * e->nc + r] = e->par[i] == p ? in[i * e->nc + r] : 0;
}

/* out = A_oo^-1 in on the odd sites, 0 on the even ones */
static void odd_self_inverse(const eo_coarse_ctx *e, const cplx *in, cplx *out)
{
    int nc = e->nc;
    for (long i = 0; i < e->Vc; ++i) {
        for (int r = 0; r < nc; ++r) {
            cplx s = 0;
            if (e->par[i] == 1)
                for (int c = 0; c < nc; ++c) s += e->Ainv[(i * nc + r) * nc + c] * in[i * nc + c];
            out[i * nc + r] = s;
        }
    }
}

/* out = S v = A_ee v_e - H_eo A_oo^-1 H_oe v_e on the even sites, 0 on the odd ones */
static void schur_coarse_apply(const void *ctx_, const cplx *in, cplx *out)
{
    const eo_coarse_ctx *e = (const eo_coarse_ctx *)ctx_;
    long dim = e->Vc * e->nc;
    keep_coarse_parity(e, 0, in, e->t1);
    dc_apply(&e->c, e->t1, e->t2);         /* (A_ee v_e, H_oe v_e) */
    odd_self_inverse(e, e->t2, e->t1);     /* (0, A_oo^-1 H_oe v_e) */
    dc_apply(&e->c, e->t1, out);           /* even part: H_eo A_oo^-1 H_oe v_e */
    for (long x = 0; x < dim; ++x) out[x] = e->t2[x] - out[x];
    keep_coarse_parity(e, 0, out, out);
}

/* u ~ D_c^-1 b through the Schur complement: bhat_e = b_e - H_eo A_oo^-1 b_o, GMRES (gmres_one,
 * m iterations, tolerance tol relative to ||bhat_e||) on S u_e = bhat_e from zero, then
 * u_o = A_oo^-1 (b_o - H_oe u_e).  res_out / iters_out as in oracle_coarse_gmres, for the Schur
 * system.  Returns -2 if a coarse extent is odd. */
int oracle_coarse_gmres_eo(const int *L, const int *a, const double *Dc_, const double *Ainv_, int n_tv,
                           const double *b_, double *u_, int n_rhs, int m, double tol, double *res_out,
                           int *iters_out)
{
    int na[4];
    block_counts(L, a, na);
    for (int mu = 0; mu < 4; ++mu)
        if (na[mu] % 2) return -2;
    long Vc = (long)na[0] * na[1] * na[2] * na[3];
    int nc = 2 * n_tv;
    long dim = Vc * nc;
    int *par = malloc(Vc * sizeof(int));
    for (long i = 0; i < Vc; ++i) {
        int c[4];
        site_coords(na, i, c);
        par[i] = (c[0] + c[1] + c[2] + c[3]) & 1;
    }
    eo_coarse_ctx e = {{L, a, Dc_, n_tv}, (const cplx *)Ainv_, Vc, nc, par, malloc(dim * sizeof(cplx)),
                       malloc(dim * sizeof(cplx))};
    cplx *bh = malloc(dim * sizeof(cplx)), *t = malloc(dim * sizeof(cplx)), *t2 = malloc(dim * sizeof(cplx));
    for (int k = 0; k < n_rhs; ++k) {
        const cplx *b = (const cplx *)b_ + (long)k * dim;
        cplx *u = (cplx *)u_ + (long)k * dim;
        odd_self_inverse(&e, b, t);          /* (0, A_oo^-1 b_o) */
        dc_apply(&e.c, t, t2);               /* even part: H_eo A_oo^-1 b_o */
        for (long x = 0; x < dim; ++x) bh[x] = b[x] - t2[x];
        keep_coarse_parity(&e, 0, bh, bh);
        gmres_one(dim, schur_coarse_apply, &e, bh, u, m, tol, res_out ? res_out + k : NULL,
                  iters_out ? iters_out + k : NULL);
        dc_apply(&e.c, u, t2);               /* odd part: H_oe u_e */
        for (long x = 0; x < dim; ++x) t[x] = b[x] - t2[x];
        odd_self_inverse(&e, t, t2);         /* (0, A_oo^-1 (b_o - H_oe u_e)) */
        for (long x = 0; x < dim; ++x) u[x] += t2[x];
    }
    free(par);
    free(e.t1);
    free(e.t2);
    free(bh);
    free(t);
    free(t2);
    return 0;
}
