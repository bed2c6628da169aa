/*
 * FP64 CPU oracle for NURBS surface evaluation and its adjoint.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this file: it is used by the test-suite, by the package's smoke check
 * and by the benchmark's CPU-baseline leg.  It shares no code, header, table
 * or constant with the HIP implementation.
 *
 * What it computes, and where the paper defines it (NURBS-Diff, arXiv
 * 2104.14547):
 *   - rational surface point          -- Sec. 3.1.1, eq. (NURBS)
 *   - Cox-de Boor recursion            -- Sec. 3.1.1, eq. (NURBSBasis)
 *   - degree-0 indicator, knot span    -- Sec. 3.1.1 eq. (BSplineBasis2) and
 *                                         Sec. 3.1.2 step 1 (half-open span)
 *   - homogeneous weighting, divide    -- Sec. 3.1.2 step 3
 *   - dS/dP_ij  (rational basis)       -- Sec. 3.2.1, eq. (NURBSuDerivative4)
 *   - dS/dw_ij                         -- Sec. 3.2.1, eq. (NURBSvDerivative5)
 *   - dS/dN_i(u)                       -- Sec. 3.2.1, eq. (NURBSvDerivative6)
 *   - dN_i^p/dU_k by the chain rule up the recursion -- Sec. 3.2.1
 *   - dS/du (parametric derivative)    -- Appendix A, eq. (NURBSuDerivative1)
 *   - curves: eq. (NURBS) with one direction dropped, and its gradients -- Sec. 3
 *   - surfaces at scattered (u, v) pairs: eq. (NURBS) at each pair
 *   - Chamfer and Hausdorff distances and their gradients
 *                                      -- Sec. 4, eqs. (ChamferDistance),
 *                                         (HausdorffDistance)
 *
 * Readings taken where the paper is silent or inconsistent:
 *   - The degree-0 indicator is half-open [U_i, U_{i+1}); a parameter equal
 *     to the last domain knot U_{n+1} belongs to span n.
 *   - A Cox-de Boor term whose knot difference is 0 is dropped, value and
 *     derivative alike (0/0 := 0).
 *   - The derivative of the degree-0 indicator with respect to a knot is
 *     taken as 0 (the zero-bandwidth limit of the paper's Gaussian
 *     smoothing); for p >= 1 this is the exact derivative of the
 *     piecewise-polynomial basis wherever it exists.
 *   - Parameters are clamped into [U_p, U_{n+1}]; the clamp carries no
 *     gradient.
 *   - Backward accumulates (+=) over the whole (p+1)x(q+1) patch and returns
 *     gradients for P, W, U and V.
 *
 * Two modes compute the same sums:
 *   dense (local == 0): every basis function of every degree, every control
 *       point, every knot -- the definitions written out;
 *   local (local != 0): only the p+1 (q+1) non-zero functions of the span
 *       and the 2p+2 (2q+2) knots they depend on (Sec. 3.1.2 step 2).
 * Summation order is the plain loop order (a, b, i, j) in IEEE FP64.
 *
 * Packed batch convention (this file's own): for surface s,
 *   shapes[6*s + 0..5] = p, q, nu_c, nv_c, nu_s, nv_s
 *   offs[7*s + 0..6]   = element offsets of ctrl, w, ku, kv, us, vs, pts
 *   ctrl  [nu_c][nv_c][3], w [nu_c][nv_c], ku [nu_c+p+1], kv [nv_c+q+1],
 *   us [nu_s], vs [nv_s], pts / grad_pts [nu_s][nv_s][3];
 *   gradients reuse the offsets of the arrays they are gradients of.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_EARG -1
#define OR_EDEGREE -2
#define OR_EKNOTS -3
#define OR_EWEIGHTS -5
#define OR_ENOMEM -9

/* ---------------------------------------------------------------------- */
/* knot vector helpers                                                      */
/* ---------------------------------------------------------------------- */

/* number of control points implied by a knot vector of length nU, degree p */
static int n_ctrl_of(int nU, int p) { return nU - p - 1; }

/* clamp a parameter into the domain [U_p, U_{n+1}] (no gradient) */
static double clamp_param(const double *U, int nU, int p, double u)
{
    const int n = n_ctrl_of(nU, p) - 1;
    if (u < U[p]) u = U[p];
    if (u > U[n + 1]) u = U[n + 1];
    return u;
}

/* Knot span from the degree-0 indicator of eq. (BSplineBasis2), read as the
 * half-open interval of Sec. 3.1.2 step 1: the unique i with
 * U_i <= u < U_{i+1}; u == U_{n+1} maps to n.  Linear scan. */
int oracle_find_span(const double *U, int nU, int p, double u)
{
    const int n = n_ctrl_of(nU, p) - 1;
    u = clamp_param(U, nU, p, u);
    if (u >= U[n + 1]) return n;
    for (int i = 0; i + 1 < nU; ++i)
        if (U[i] <= u && u < U[i + 1]) return i;
    return -1; /* unreachable for a valid, clamped parameter */
}

/* ---------------------------------------------------------------------- */
/* dense basis: every N_i^d, with derivatives w.r.t. every knot and w.r.t. u */
/* ---------------------------------------------------------------------- */

/* Outputs (any may be NULL):
 *   N[i]          = N_i^p(u),               i = 0..n
 *   dNdU[i*nU+k]  = dN_i^p(u) / dU_k
 *   dNdu[i]       = dN_i^p(u) / du
 * Returns 0, or OR_ENOMEM. */
int oracle_basis_dense(const double *U, int nU, int p, double u,
                       double *N, double *dNdU, double *dNdu)
{
    const int n = n_ctrl_of(nU, p) - 1;
    const int m = nU - 1; /* number of degree-0 functions */
    double *val = (double *)calloc((size_t)m, sizeof(double));
    double *nval = (double *)calloc((size_t)m, sizeof(double));
    double *dk = (double *)calloc((size_t)m * nU, sizeof(double));
    double *ndk = (double *)calloc((size_t)m * nU, sizeof(double));
    double *du = (double *)calloc((size_t)m, sizeof(double));
    double *ndu = (double *)calloc((size_t)m, sizeof(double));
    if (!val || !nval || !dk || !ndk || !du || !ndu) {
        free(val); free(nval); free(dk); free(ndk); free(du); free(ndu);
        return OR_ENOMEM;
    }
    u = clamp_param(U, nU, p, u);

    /* degree 0: N_i^0 = 1 on [U_i, U_{i+1}); at the domain's right end the
     * last non-degenerate span n takes the value. */
    if (u >= U[n + 1]) {
        val[n] = 1.0;
    } else {
        for (int i = 0; i < m; ++i) val[i] = (U[i] <= u && u < U[i + 1]) ? 1.0 : 0.0;
    }
    /* d N^0 / dU = 0 and d N^0 / du = 0: already zero. */

    for (int d = 1; d <= p; ++d) {
        const int cnt = m - d; /* functions of degree d: i = 0..m-d-1 */
        for (int i = 0; i < cnt; ++i) {
            double v = 0.0, vdu = 0.0;
            double *g = ndk + (size_t)i * nU;
            memset(g, 0, sizeof(double) * nU);
            /* alpha term: (u - U_i)/(U_{i+d} - U_i) * N_i^{d-1} */
            const double den1 = U[i + d] - U[i];
            if (den1 != 0.0) {
                const double a = (u - U[i]) / den1;
                const double Ni = val[i];
                const double *gi = dk + (size_t)i * nU;
                v += a * Ni;
                vdu += a * du[i] + Ni / den1;
                for (int k = 0; k < nU; ++k) g[k] += a * gi[k];
                g[i] += Ni * (u - U[i + d]) / (den1 * den1);
                g[i + d] += -Ni * (u - U[i]) / (den1 * den1);
            }
            /* beta term: (U_{i+d+1} - u)/(U_{i+d+1} - U_{i+1}) * N_{i+1}^{d-1} */
            const double den2 = U[i + d + 1] - U[i + 1];
            if (den2 != 0.0) {
                const double b = (U[i + d + 1] - u) / den2;
                const double Ni1 = val[i + 1];
                const double *gi1 = dk + (size_t)(i + 1) * nU;
                v += b * Ni1;
                vdu += b * du[i + 1] - Ni1 / den2;
                for (int k = 0; k < nU; ++k) g[k] += b * gi1[k];
                g[i + 1] += Ni1 * (U[i + d + 1] - u) / (den2 * den2);
                g[i + d + 1] += Ni1 * (u - U[i + 1]) / (den2 * den2);
            }
            nval[i] = v;
            ndu[i] = vdu;
        }
        /* swap level buffers */
        double *t;
        t = val; val = nval; nval = t;
        t = dk; dk = ndk; ndk = t;
        t = du; du = ndu; ndu = t;
    }
    for (int i = 0; i <= n; ++i) {
        if (N) N[i] = val[i];
        if (dNdu) dNdu[i] = du[i];
        if (dNdU) memcpy(dNdU + (size_t)i * nU, dk + (size_t)i * nU, sizeof(double) * nU);
    }
    free(val); free(nval); free(dk); free(ndk); free(du); free(ndu);
    return OR_OK;
}

/* ---------------------------------------------------------------------- */
/* local basis: the p+1 non-zero functions of span k                        */
/* ---------------------------------------------------------------------- */

#define OR_PMAX 15

/* Non-zero functions N_{k-p+r}^p(u), r = 0..p, by eq. (NURBSBasis) restricted
 * to the triangle of functions that can be non-zero on span k.
 * dNdU[r*(2p+2) + t] = d N_{k-p+r} / d U_{k-p+t}, t = 0..2p+1.
 * dNdu[r]            = d N_{k-p+r} / du.  Returns the span k. */
int oracle_basis_local(const double *U, int nU, int p, double u,
                       double *N, double *dNdU, double *dNdu)
{
    const int k = oracle_find_span(U, nU, p, u);
    const int W = 2 * p + 2;
    double val[OR_PMAX + 1], nval[OR_PMAX + 1];
    double du[OR_PMAX + 1], ndu[OR_PMAX + 1];
    double dk[(OR_PMAX + 1) * (2 * OR_PMAX + 2)], ndk[(OR_PMAX + 1) * (2 * OR_PMAX + 2)];
    u = clamp_param(U, nU, p, u);
    /* level 0: only N_k^0 = 1 (index 0 of the level) */
    val[0] = 1.0;
    du[0] = 0.0;
    memset(dk, 0, sizeof(double) * W);
    const int base = k - p; /* knot index of window slot 0 */
    for (int d = 1; d <= p; ++d) {
        /* level d holds N_{k-d+idx}^d, idx = 0..d;
         * level d-1 holds N_{k-d+1+j}^{d-1}, j = 0..d-1 */
        for (int idx = 0; idx <= d; ++idx) {
            const int i = k - d + idx;
            double v = 0.0, vdu = 0.0;
            double *g = ndk + (size_t)idx * W;
            memset(g, 0, sizeof(double) * W);
            if (idx >= 1) { /* alpha * N_i^{d-1}, N_i^{d-1} at level index idx-1 */
                const double den1 = U[i + d] - U[i];
                if (den1 != 0.0) {
                    const double a = (u - U[i]) / den1;
                    const double Ni = val[idx - 1];
                    const double *gi = dk + (size_t)(idx - 1) * W;
                    v += a * Ni;
                    vdu += a * du[idx - 1] + Ni / den1;
                    for (int t = 0; t < W; ++t) g[t] += a * gi[t];
                    g[i - base] += Ni * (u - U[i + d]) / (den1 * den1);
                    g[i + d - base] += -Ni * (u - U[i]) / (den1 * den1);
                }
            }
            if (idx <= d - 1) { /* beta * N_{i+1}^{d-1}, at level index idx */
                const double den2 = U[i + d + 1] - U[i + 1];
                if (den2 != 0.0) {
                    const double b = (U[i + d + 1] - u) / den2;
                    const double Ni1 = val[idx];
                    const double *gi1 = dk + (size_t)idx * W;
                    v += b * Ni1;
                    vdu += b * du[idx] - Ni1 / den2;
                    for (int t = 0; t < W; ++t) g[t] += b * gi1[t];
                    g[i + 1 - base] += Ni1 * (U[i + d + 1] - u) / (den2 * den2);
                    g[i + d + 1 - base] += Ni1 * (u - U[i + 1]) / (den2 * den2);
                }
            }
            nval[idx] = v;
            ndu[idx] = vdu;
        }
        memcpy(val, nval, sizeof(double) * (d + 1));
        memcpy(du, ndu, sizeof(double) * (d + 1));
        memcpy(dk, ndk, sizeof(double) * (d + 1) * W);
    }
    for (int r = 0; r <= p; ++r) {
        if (N) N[r] = val[r];
        if (dNdu) dNdu[r] = du[r];
        if (dNdU) memcpy(dNdU + (size_t)r * W, dk + (size_t)r * W, sizeof(double) * W);
    }
    return k;
}

/* ---------------------------------------------------------------------- */
/* per-direction tables: basis of every sample along one parameter          */
/* ---------------------------------------------------------------------- */

typedef struct {
    int nc;       /* control points along the direction */
    int nk;       /* knots */
    int deg;
    int local;
    int *span;    /* [ns] */
    int lo_w;     /* width of the index window per sample (nc or deg+1) */
    int kw;       /* width of the knot window (nk or 2deg+2) */
    double *N;    /* [ns][lo_w] */
    double *dNdU; /* [ns][lo_w][kw] */
    double *dNdu; /* [ns][lo_w] */
} dir_table;

static void dir_free(dir_table *t)
{
    free(t->span); free(t->N); free(t->dNdU); free(t->dNdu);
}

static int dir_build(dir_table *t, const double *U, int nk, int deg,
                     const double *x, int ns, int local, int want_knots)
{
    t->nc = n_ctrl_of(nk, deg);
    t->nk = nk;
    t->deg = deg;
    t->local = local;
    t->lo_w = local ? deg + 1 : t->nc;
    t->kw = local ? 2 * deg + 2 : nk;
    t->span = (int *)malloc(sizeof(int) * (size_t)(ns > 0 ? ns : 1));
    t->N = (double *)malloc(sizeof(double) * (size_t)(ns > 0 ? ns : 1) * t->lo_w);
    t->dNdu = (double *)malloc(sizeof(double) * (size_t)(ns > 0 ? ns : 1) * t->lo_w);
    t->dNdU = want_knots
        ? (double *)malloc(sizeof(double) * (size_t)(ns > 0 ? ns : 1) * t->lo_w * t->kw)
        : NULL;
    if (!t->span || !t->N || !t->dNdu || (want_knots && !t->dNdU)) return OR_ENOMEM;
    for (int a = 0; a < ns; ++a) {
        double *Na = t->N + (size_t)a * t->lo_w;
        double *Da = t->dNdu + (size_t)a * t->lo_w;
        double *Ka = want_knots ? t->dNdU + (size_t)a * t->lo_w * t->kw : NULL;
        if (local) {
            t->span[a] = oracle_basis_local(U, nk, deg, x[a], Na, Ka, Da);
        } else {
            t->span[a] = oracle_find_span(U, nk, deg, x[a]);
            if (oracle_basis_dense(U, nk, deg, x[a], Na, Ka, Da) != OR_OK) return OR_ENOMEM;
        }
    }
    return OR_OK;
}

/* control index and knot index of table column c / knot column t at sample a */
static int dir_ctrl(const dir_table *t, int a, int c)
{
    return t->local ? t->span[a] - t->deg + c : c;
}
static int dir_knot(const dir_table *t, int a, int kt)
{
    return t->local ? t->span[a] - t->deg + kt : kt;
}

/* ---------------------------------------------------------------------- */
/* validation (R3 rules)                                                    */
/* ---------------------------------------------------------------------- */

static int check_surface(int p, int q, int nu_c, int nv_c, int nu_s, int nv_s,
                         const double *ku, const double *kv, const double *w)
{
    if (p < 1 || q < 1 || p > OR_PMAX || q > OR_PMAX) return OR_EDEGREE;
    if (nu_c < p + 1 || nv_c < q + 1) return OR_EDEGREE;
    if (nu_s < 0 || nv_s < 0) return OR_EARG;
    const int nU = nu_c + p + 1, nV = nv_c + q + 1;
    for (int i = 0; i + 1 < nU; ++i) if (!(ku[i] <= ku[i + 1])) return OR_EKNOTS;
    for (int i = 0; i + 1 < nV; ++i) if (!(kv[i] <= kv[i + 1])) return OR_EKNOTS;
    if (!(ku[p] < ku[p + 1]) || !(ku[nu_c - 1] < ku[nu_c])) return OR_EKNOTS;
    if (!(kv[q] < kv[q + 1]) || !(kv[nv_c - 1] < kv[nv_c])) return OR_EKNOTS;
    for (int i = 0; i < nu_c * nv_c; ++i) if (!(w[i] > 0.0)) return OR_EWEIGHTS;
    return OR_OK;
}

/* ---------------------------------------------------------------------- */
/* one surface: forward                                                     */
/* ---------------------------------------------------------------------- */

static int surface_fwd(int p, int q, int nu_c, int nv_c, int nu_s, int nv_s,
                       const double *P, const double *w, const double *ku,
                       const double *kv, const double *us, const double *vs,
                       double *S, double *Su, double *Sv, int local)
{
    int rc = check_surface(p, q, nu_c, nv_c, nu_s, nv_s, ku, kv, w);
    if (rc) return rc;
    dir_table tu, tv;
    memset(&tu, 0, sizeof tu);
    memset(&tv, 0, sizeof tv);
    rc = dir_build(&tu, ku, nu_c + p + 1, p, us, nu_s, local, 0);
    if (!rc) rc = dir_build(&tv, kv, nv_c + q + 1, q, vs, nv_s, local, 0);
    if (rc) { dir_free(&tu); dir_free(&tv); return rc; }
    for (int a = 0; a < nu_s; ++a) {
        for (int b = 0; b < nv_s; ++b) {
            /* eq. (NURBS), split as eq. (NURBSsplit): NR / w(u,v) */
            double NR[3] = {0, 0, 0}, Wsum = 0.0;
            double NRu[3] = {0, 0, 0}, Wu = 0.0, NRv[3] = {0, 0, 0}, Wv = 0.0;
            for (int ci = 0; ci < tu.lo_w; ++ci) {
                const int i = dir_ctrl(&tu, a, ci);
                const double Ni = tu.N[(size_t)a * tu.lo_w + ci];
                const double Niu = tu.dNdu[(size_t)a * tu.lo_w + ci];
                for (int cj = 0; cj < tv.lo_w; ++cj) {
                    const int j = dir_ctrl(&tv, b, cj);
                    const double Nj = tv.N[(size_t)b * tv.lo_w + cj];
                    const double Njv = tv.dNdu[(size_t)b * tv.lo_w + cj];
                    const double wij = w[(size_t)i * nv_c + j];
                    const double *Pij = P + ((size_t)i * nv_c + j) * 3;
                    const double c = Ni * Nj * wij;
                    for (int x = 0; x < 3; ++x) NR[x] += c * Pij[x];
                    Wsum += c;
                    if (Su) {
                        const double cu = Niu * Nj * wij;
                        for (int x = 0; x < 3; ++x) NRu[x] += cu * Pij[x];
                        Wu += cu;
                    }
                    if (Sv) {
                        const double cv = Ni * Njv * wij;
                        for (int x = 0; x < 3; ++x) NRv[x] += cv * Pij[x];
                        Wv += cv;
                    }
                }
            }
            double *out = S + ((size_t)a * nv_s + b) * 3;
            for (int x = 0; x < 3; ++x) out[x] = NR[x] / Wsum;
            /* Appendix A, eq. (NURBSuDerivative1) */
            if (Su) {
                double *o = Su + ((size_t)a * nv_s + b) * 3;
                for (int x = 0; x < 3; ++x) o[x] = (NRu[x] * Wsum - NR[x] * Wu) / (Wsum * Wsum);
            }
            if (Sv) {
                double *o = Sv + ((size_t)a * nv_s + b) * 3;
                for (int x = 0; x < 3; ++x) o[x] = (NRv[x] * Wsum - NR[x] * Wv) / (Wsum * Wsum);
            }
        }
    }
    dir_free(&tu);
    dir_free(&tv);
    return OR_OK;
}

/* ---------------------------------------------------------------------- */
/* one surface: backward (vector-Jacobian product)                         */
/* ---------------------------------------------------------------------- */

static int surface_bwd(int p, int q, int nu_c, int nv_c, int nu_s, int nv_s,
                       const double *P, const double *w, const double *ku,
                       const double *kv, const double *us, const double *vs,
                       const double *G, double *dP, double *dW, double *dU,
                       double *dV, int local)
{
    int rc = check_surface(p, q, nu_c, nv_c, nu_s, nv_s, ku, kv, w);
    if (rc) return rc;
    const int nU = nu_c + p + 1, nV = nv_c + q + 1;
    dir_table tu, tv;
    memset(&tu, 0, sizeof tu);
    memset(&tv, 0, sizeof tv);
    rc = dir_build(&tu, ku, nU, p, us, nu_s, local, 1);
    if (!rc) rc = dir_build(&tv, kv, nV, q, vs, nv_s, local, 1);
    double *rowsum = (double *)malloc(sizeof(double) * 4 * (size_t)(tu.lo_w > 0 ? tu.lo_w : 1));
    double *colsum = (double *)malloc(sizeof(double) * 4 * (size_t)(tv.lo_w > 0 ? tv.lo_w : 1));
    if (rc || !rowsum || !colsum) {
        dir_free(&tu); dir_free(&tv); free(rowsum); free(colsum);
        return rc ? rc : OR_ENOMEM;
    }
    memset(dP, 0, sizeof(double) * (size_t)nu_c * nv_c * 3);
    memset(dW, 0, sizeof(double) * (size_t)nu_c * nv_c);
    memset(dU, 0, sizeof(double) * (size_t)nU);
    memset(dV, 0, sizeof(double) * (size_t)nV);

    for (int a = 0; a < nu_s; ++a) {
        for (int b = 0; b < nv_s; ++b) {
            const double *g = G + ((size_t)a * nv_s + b) * 3;
            /* NR(u,v) and w(u,v) of eq. (NURBSsplit) */
            double NR[3] = {0, 0, 0}, Wsum = 0.0;
            for (int ci = 0; ci < tu.lo_w; ++ci) {
                const int i = dir_ctrl(&tu, a, ci);
                const double Ni = tu.N[(size_t)a * tu.lo_w + ci];
                for (int cj = 0; cj < tv.lo_w; ++cj) {
                    const int j = dir_ctrl(&tv, b, cj);
                    const double Nj = tv.N[(size_t)b * tv.lo_w + cj];
                    const double c = Ni * Nj * w[(size_t)i * nv_c + j];
                    const double *Pij = P + ((size_t)i * nv_c + j) * 3;
                    for (int x = 0; x < 3; ++x) NR[x] += c * Pij[x];
                    Wsum += c;
                }
            }
            const double W2 = Wsum * Wsum;
            /* control points and weights: eqs. (NURBSuDerivative4), (NURBSvDerivative5) */
            for (int ci = 0; ci < tu.lo_w; ++ci) {
                const int i = dir_ctrl(&tu, a, ci);
                const double Ni = tu.N[(size_t)a * tu.lo_w + ci];
                for (int cj = 0; cj < tv.lo_w; ++cj) {
                    const int j = dir_ctrl(&tv, b, cj);
                    const double Nj = tv.N[(size_t)b * tv.lo_w + cj];
                    const size_t ij = (size_t)i * nv_c + j;
                    const double *Pij = P + ij * 3;
                    const double R = Ni * Nj * w[ij] / Wsum;
                    double sw = 0.0;
                    for (int x = 0; x < 3; ++x) {
                        dP[ij * 3 + x] += R * g[x];
                        sw += g[x] * (Ni * Nj * Pij[x] * Wsum - NR[x] * Ni * Nj) / W2;
                    }
                    dW[ij] += sw;
                }
            }
            /* knots of U: eq. (NURBSvDerivative6) times dN_i^p(u)/dU_k */
            for (int ci = 0; ci < tu.lo_w; ++ci) {
                const int i = dir_ctrl(&tu, a, ci);
                double num[3] = {0, 0, 0}, den = 0.0;
                for (int cj = 0; cj < tv.lo_w; ++cj) {
                    const int j = dir_ctrl(&tv, b, cj);
                    const double Nj = tv.N[(size_t)b * tv.lo_w + cj];
                    const size_t ij = (size_t)i * nv_c + j;
                    for (int x = 0; x < 3; ++x) num[x] += Nj * w[ij] * P[ij * 3 + x];
                    den += Nj * w[ij];
                }
                double c = 0.0;
                for (int x = 0; x < 3; ++x) c += g[x] * (num[x] / Wsum - NR[x] / W2 * den);
                rowsum[ci] = c;
            }
            for (int ci = 0; ci < tu.lo_w; ++ci) {
                const double *dk = tu.dNdU + ((size_t)a * tu.lo_w + ci) * tu.kw;
                for (int kt = 0; kt < tu.kw; ++kt) {
                    const int kk = dir_knot(&tu, a, kt);
                    if (kk >= 0 && kk < nU) dU[kk] += rowsum[ci] * dk[kt];
                }
            }
            /* knots of V: the same with the roles of u and v exchanged */
            for (int cj = 0; cj < tv.lo_w; ++cj) {
                const int j = dir_ctrl(&tv, b, cj);
                double num[3] = {0, 0, 0}, den = 0.0;
                for (int ci = 0; ci < tu.lo_w; ++ci) {
                    const int i = dir_ctrl(&tu, a, ci);
                    const double Ni = tu.N[(size_t)a * tu.lo_w + ci];
                    const size_t ij = (size_t)i * nv_c + j;
                    for (int x = 0; x < 3; ++x) num[x] += Ni * w[ij] * P[ij * 3 + x];
                    den += Ni * w[ij];
                }
                double c = 0.0;
                for (int x = 0; x < 3; ++x) c += g[x] * (num[x] / Wsum - NR[x] / W2 * den);
                colsum[cj] = c;
            }
            for (int cj = 0; cj < tv.lo_w; ++cj) {
                const double *dk = tv.dNdU + ((size_t)b * tv.lo_w + cj) * tv.kw;
                for (int kt = 0; kt < tv.kw; ++kt) {
                    const int kk = dir_knot(&tv, b, kt);
                    if (kk >= 0 && kk < nV) dV[kk] += colsum[cj] * dk[kt];
                }
            }
        }
    }
    dir_free(&tu);
    dir_free(&tv);
    free(rowsum);
    free(colsum);
    return OR_OK;
}

/* ---------------------------------------------------------------------- */
/* batch entry points                                                       */
/* ---------------------------------------------------------------------- */

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* S (and optionally dS/du, dS/dv) for every surface of a packed batch.
 * Surfaces are independent; OpenMP spreads them over nthreads threads
 * (nthreads <= 0 keeps the runtime default).  Returns the first error. */
int oracle_fwd(int nsurf, const int32_t *shapes, const int64_t *offs,
               const double *ctrl, const double *w, const double *ku,
               const double *kv, const double *us, const double *vs,
               double *pts, double *pts_du, double *pts_dv, int local,
               int nthreads)
{
    int err = OR_OK;
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
    for (int s = 0; s < nsurf; ++s) {
        const int32_t *sh = shapes + 6 * (size_t)s;
        const int64_t *o = offs + 7 * (size_t)s;
        int rc = surface_fwd(sh[0], sh[1], sh[2], sh[3], sh[4], sh[5],
                             ctrl + o[0], w + o[1], ku + o[2], kv + o[3],
                             us + o[4], vs + o[5], pts + o[6],
                             pts_du ? pts_du + o[6] : NULL,
                             pts_dv ? pts_dv + o[6] : NULL, local);
        if (rc) {
#pragma omp critical
            if (!err) err = rc;
        }
    }
    return err;
}

/* dL/dP, dL/dW, dL/dU, dL/dV for every surface given dL/dS (grad_pts). */
int oracle_bwd(int nsurf, const int32_t *shapes, const int64_t *offs,
               const double *ctrl, const double *w, const double *ku,
               const double *kv, const double *us, const double *vs,
               const double *grad_pts, double *grad_ctrl, double *grad_w,
               double *grad_ku, double *grad_kv, int local, int nthreads)
{
    int err = OR_OK;
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
    for (int s = 0; s < nsurf; ++s) {
        const int32_t *sh = shapes + 6 * (size_t)s;
        const int64_t *o = offs + 7 * (size_t)s;
        int rc = surface_bwd(sh[0], sh[1], sh[2], sh[3], sh[4], sh[5],
                             ctrl + o[0], w + o[1], ku + o[2], kv + o[3],
                             us + o[4], vs + o[5], grad_pts + o[6],
                             grad_ctrl + o[0], grad_w + o[1], grad_ku + o[2],
                             grad_kv + o[3], local);
        if (rc) {
#pragma omp critical
            if (!err) err = rc;
        }
    }
    return err;
}

/* ---------------------------------------------------------------------- */
/* curves                                                                   */
/* ---------------------------------------------------------------------- */
/* A rational B-spline curve C(u) = sum_i N_i^p(u) w_i P_i / sum_i N_i^p(u) w_i
 * with P_i in R^dim (dim 2 or 3): eq. (NURBS) with one parametric direction
 * dropped, the way Sec. 3 obtains curves from the surface formulas.  Its
 * derivatives are those of Sec. 3.2.1 with the v direction dropped:
 *   dC/dP_i = N_i w_i / W                      (eq. NURBSuDerivative4)
 *   dC/dw_i = N_i (P_i - C) / W                (eq. NURBSvDerivative5)
 *   dC/dN_i = w_i (P_i - C) / W                (eq. NURBSvDerivative6)
 * times dN_i/dU_k from the recursion's knot duals for the knots, and
 *   dC/du   = (A_u W - A W_u) / W^2            (eq. NURBSuDerivative1)
 * with A = sum_i N_i w_i P_i, W = sum_i N_i w_i.  Dense mode only: every
 * basis function of the knot vector at every sample.
 *
 * Packed batch convention: for curve s,
 *   shapes[4*s + 0..3] = p, nc, ns, dim
 *   offs[5*s + 0..4]   = element offsets of ctrl [nc][dim], w [nc],
 *                        knots [nc+p+1], us [ns], pts [ns][dim];
 *   gradients reuse the offsets of the arrays they are gradients of. */

static int check_curve(int p, int nc, int ns, int dim, const double *U, const double *w)
{
    if (p < 1 || p > OR_PMAX || nc < p + 1) return OR_EDEGREE;
    if (ns < 0 || (dim != 2 && dim != 3)) return OR_EARG;
    const int nU = nc + p + 1;
    for (int i = 0; i + 1 < nU; ++i) if (!(U[i] <= U[i + 1])) return OR_EKNOTS;
    if (!(U[p] < U[p + 1]) || !(U[nc - 1] < U[nc])) return OR_EKNOTS;
    for (int i = 0; i < nc; ++i) if (!(w[i] > 0.0)) return OR_EWEIGHTS;
    return OR_OK;
}

static int curve_fwd(int p, int nc, int ns, int dim, const double *P, const double *w,
                     const double *U, const double *us, double *C, double *Cu)
{
    int rc = check_curve(p, nc, ns, dim, U, w);
    if (rc) return rc;
    const int nU = nc + p + 1;
    double *N = (double *)malloc(sizeof(double) * (size_t)nc);
    double *dN = (double *)malloc(sizeof(double) * (size_t)nc);
    if (!N || !dN) { free(N); free(dN); return OR_ENOMEM; }
    for (int a = 0; a < ns && rc == OR_OK; ++a) {
        rc = oracle_basis_dense(U, nU, p, us[a], N, NULL, dN);
        double A[3] = {0, 0, 0}, Wsum = 0.0, Au[3] = {0, 0, 0}, Wu = 0.0;
        for (int i = 0; i < nc; ++i) {
            const double c = N[i] * w[i], cu = dN[i] * w[i];
            for (int x = 0; x < dim; ++x) {
                A[x] += c * P[(size_t)i * dim + x];
                Au[x] += cu * P[(size_t)i * dim + x];
            }
            Wsum += c;
            Wu += cu;
        }
        for (int x = 0; x < dim; ++x) {
            C[(size_t)a * dim + x] = A[x] / Wsum;
            if (Cu) Cu[(size_t)a * dim + x] = (Au[x] * Wsum - A[x] * Wu) / (Wsum * Wsum);
        }
    }
    free(N);
    free(dN);
    return rc;
}

static int curve_bwd(int p, int nc, int ns, int dim, const double *P, const double *w,
                     const double *U, const double *us, const double *G,
                     double *dP, double *dW, double *dU)
{
    int rc = check_curve(p, nc, ns, dim, U, w);
    if (rc) return rc;
    const int nU = nc + p + 1;
    double *N = (double *)malloc(sizeof(double) * (size_t)nc);
    double *dNdU = (double *)malloc(sizeof(double) * (size_t)nc * nU);
    if (!N || !dNdU) { free(N); free(dNdU); return OR_ENOMEM; }
    memset(dP, 0, sizeof(double) * (size_t)nc * dim);
    memset(dW, 0, sizeof(double) * (size_t)nc);
    memset(dU, 0, sizeof(double) * (size_t)nU);
    for (int a = 0; a < ns && rc == OR_OK; ++a) {
        rc = oracle_basis_dense(U, nU, p, us[a], N, dNdU, NULL);
        const double *g = G + (size_t)a * dim;
        double A[3] = {0, 0, 0}, Wsum = 0.0;
        for (int i = 0; i < nc; ++i) {
            const double c = N[i] * w[i];
            for (int x = 0; x < dim; ++x) A[x] += c * P[(size_t)i * dim + x];
            Wsum += c;
        }
        double C[3];
        for (int x = 0; x < dim; ++x) C[x] = A[x] / Wsum;
        for (int i = 0; i < nc; ++i) {
            double pg = 0.0; /* (P_i - C) . g */
            for (int x = 0; x < dim; ++x) {
                dP[(size_t)i * dim + x] += N[i] * w[i] / Wsum * g[x];
                pg += (P[(size_t)i * dim + x] - C[x]) * g[x];
            }
            dW[i] += N[i] * pg / Wsum;
            const double coef = w[i] * pg / Wsum; /* dL/dN_i at this sample */
            for (int k = 0; k < nU; ++k) dU[k] += coef * dNdU[(size_t)i * nU + k];
        }
    }
    free(N);
    free(dNdU);
    return rc;
}

/* C (and optionally dC/du) for every curve of a packed batch. */
int oracle_curve_fwd(int ncurve, const int32_t *shapes, const int64_t *offs,
                     const double *ctrl, const double *w, const double *knots,
                     const double *us, double *pts, double *pts_du, int nthreads)
{
    int err = OR_OK;
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
    for (int s = 0; s < ncurve; ++s) {
        const int32_t *sh = shapes + 4 * (size_t)s;
        const int64_t *o = offs + 5 * (size_t)s;
        int rc = curve_fwd(sh[0], sh[1], sh[2], sh[3], ctrl + o[0], w + o[1], knots + o[2],
                           us + o[3], pts + o[4], pts_du ? pts_du + o[4] : NULL);
        if (rc) {
#pragma omp critical
            if (!err) err = rc;
        }
    }
    return err;
}

/* dL/dP, dL/dw, dL/dU of every curve given dL/dC (grad_pts). */
int oracle_curve_bwd(int ncurve, const int32_t *shapes, const int64_t *offs,
                     const double *ctrl, const double *w, const double *knots,
                     const double *us, const double *grad_pts, double *grad_ctrl,
                     double *grad_w, double *grad_knots, int nthreads)
{
    int err = OR_OK;
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
    for (int s = 0; s < ncurve; ++s) {
        const int32_t *sh = shapes + 4 * (size_t)s;
        const int64_t *o = offs + 5 * (size_t)s;
        int rc = curve_bwd(sh[0], sh[1], sh[2], sh[3], ctrl + o[0], w + o[1], knots + o[2],
                           us + o[3], grad_pts + o[4], grad_ctrl + o[0], grad_w + o[1],
                           grad_knots + o[2]);
        if (rc) {
#pragma omp critical
            if (!err) err = rc;
        }
    }
    return err;
}

/* ---------------------------------------------------------------------- */
/* point-set losses: Chamfer and Hausdorff distances                        */
/* ---------------------------------------------------------------------- */
/*
 * Sec. 4, eq. (ChamferDistance) and eq. (HausdorffDistance), between the
 * evaluated points P (n of them) and a target cloud Q (m), with the
 * Euclidean (non-squared) norm, two-sided, summed (CD) or maximised (HD)
 * exactly as printed:
 *   CD = sum_i min_j |P_i - Q_j| + sum_j min_i |P_i - Q_j|
 *   HD = max_i min_j |P_i - Q_j| + max_j min_i |P_i - Q_j|
 * Which point is nearest (and which is farthest) is an integer decision.
 * It is taken on the float32 inputs in float32, with the squared distance
 * written as  d2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx))  (dz = 0 in the
 * plane) on float32 differences, a strictly smaller value winning, so the
 * first index wins ties; the distances, the sums and the gradients are then
 * taken in FP64 from the chosen pairs.  The gradient with respect to P is
 *   dCD/dP_i = (P_i - Q_a(i)) / |.| + sum_{j : b(j) = i} (P_i - Q_j) / |.|
 *   dHD/dP_i = [i = i*] (P_i - Q_a(i)) / |.| + [i = b(j*)] (P_i - Q_j*) / |.|
 * (a = nearest target of each point, b = nearest point of each target,
 * i* and j* the farthest ones), with a zero distance contributing zero.
 */
static float nn_d2(int dim, const float *p, const float *q)
{
    const float dx = p[0] - q[0], dy = p[1] - q[1];
    const float dz = dim == 3 ? p[2] - q[2] : 0.0f;
    return fmaf(dz, dz, fmaf(dy, dy, dx * dx));
}

/* For each P_i the index of its nearest Q_j and that squared distance. */
int oracle_nearest(int dim, const float *P, int n, const float *Q, int m, int32_t *idx, float *d2, int nthreads)
{
    if ((dim != 2 && dim != 3) || n < 0 || m < 1) return OR_EARG;
    set_threads(nthreads);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
        int best = 0;
        float bd = nn_d2(dim, P + (size_t)i * dim, Q);
        for (int j = 1; j < m; ++j) {
            const float d = nn_d2(dim, P + (size_t)i * dim, Q + (size_t)j * dim);
            if (d < bd) { bd = d; best = j; }
        }
        idx[i] = best;
        d2[i] = bd;
    }
    return OR_OK;
}

static double pair_dist(int dim, const float *p, const float *q, double *dir)
{
    double s = 0.0;
    for (int x = 0; x < dim; ++x) {
        dir[x] = (double)p[x] - (double)q[x];
        s += dir[x] * dir[x];
    }
    const double d = sqrt(s);
    for (int x = 0; x < dim; ++x) dir[x] = d > 0.0 ? dir[x] / d : 0.0;
    return d;
}

/* out[0] = CD, out[1] = HD; gcd, ghd [n][dim] (either may be NULL). */
int oracle_chamfer_hausdorff(int dim, const float *P, int n, const float *Q, int m, double *out, double *gcd,
                             double *ghd, int nthreads)
{
    if ((dim != 2 && dim != 3) || n < 1 || m < 1) return OR_EARG;
    int32_t *a = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *b = (int32_t *)malloc(sizeof(int32_t) * (size_t)m);
    float *da = (float *)malloc(sizeof(float) * (size_t)n);
    float *db = (float *)malloc(sizeof(float) * (size_t)m);
    if (!a || !b || !da || !db) { free(a); free(b); free(da); free(db); return OR_ENOMEM; }
    oracle_nearest(dim, P, n, Q, m, a, da, nthreads);
    oracle_nearest(dim, Q, m, P, n, b, db, nthreads);
    if (gcd) memset(gcd, 0, sizeof(double) * (size_t)n * dim);
    if (ghd) memset(ghd, 0, sizeof(double) * (size_t)n * dim);
    double cd = 0.0, dir[3];
    int istar = 0, jstar = 0;
    for (int i = 0; i < n; ++i) {
        cd += pair_dist(dim, P + (size_t)i * dim, Q + (size_t)a[i] * dim, dir);
        if (gcd)
            for (int x = 0; x < dim; ++x) gcd[(size_t)i * dim + x] += dir[x];
        if (da[i] > da[istar]) istar = i;
    }
    for (int j = 0; j < m; ++j) {
        const int i = b[j];
        cd += pair_dist(dim, P + (size_t)i * dim, Q + (size_t)j * dim, dir);
        if (gcd)
            for (int x = 0; x < dim; ++x) gcd[(size_t)i * dim + x] += dir[x];
        if (db[j] > db[jstar]) jstar = j;
    }
    double hd = pair_dist(dim, P + (size_t)istar * dim, Q + (size_t)a[istar] * dim, dir);
    if (ghd)
        for (int x = 0; x < dim; ++x) ghd[(size_t)istar * dim + x] += dir[x];
    hd += pair_dist(dim, P + (size_t)b[jstar] * dim, Q + (size_t)jstar * dim, dir);
    if (ghd)
        for (int x = 0; x < dim; ++x) ghd[(size_t)b[jstar] * dim + x] += dir[x];
    out[0] = cd;
    out[1] = hd;
    free(a); free(b); free(da); free(db);
    return OR_OK;
}

/* ---------------------------------------------------------------------- */
/* scattered parameters                                                     */
/* ---------------------------------------------------------------------- */
/*
 * Surface points at scattered parameter pairs (u_k, v_k), k = 0..npts-1,
 * in any order (eq. NURBS at each pair; Sec. 3.1 evaluates a grid, which is
 * the special case of all pairs of two parameter lists).  Each pair is the
 * 1x1 grid {u_k} x {v_k} of the grid functions above; the gradients are the
 * sums over the pairs of the per-pair gradients.
 *   uv [npts][2], S / Su / Sv / G [npts][3]; dP, dW, dU, dV as for a grid.
 */
int oracle_scattered_fwd(int p, int q, int nu_c, int nv_c, int npts, const double *P, const double *w,
                         const double *ku, const double *kv, const double *uv, double *S, double *Su, double *Sv,
                         int local)
{
    for (int k = 0; k < npts; ++k) {
        int rc = surface_fwd(p, q, nu_c, nv_c, 1, 1, P, w, ku, kv, uv + 2 * (size_t)k, uv + 2 * (size_t)k + 1,
                             S + 3 * (size_t)k, Su ? Su + 3 * (size_t)k : NULL, Sv ? Sv + 3 * (size_t)k : NULL,
                             local);
        if (rc) return rc;
    }
    return OR_OK;
}

int oracle_scattered_bwd(int p, int q, int nu_c, int nv_c, int npts, const double *P, const double *w,
                         const double *ku, const double *kv, const double *uv, const double *G, double *dP,
                         double *dW, double *dU, double *dV, int local)
{
    const size_t ncp = (size_t)nu_c * nv_c, nU = (size_t)nu_c + p + 1, nV = (size_t)nv_c + q + 1;
    double *t = (double *)malloc(sizeof(double) * (4 * ncp + nU + nV));
    if (!t) return OR_ENOMEM;
    double *tP = t, *tW = t + 3 * ncp, *tU = tW + ncp, *tV = tU + nU;
    memset(dP, 0, sizeof(double) * 3 * ncp);
    memset(dW, 0, sizeof(double) * ncp);
    memset(dU, 0, sizeof(double) * nU);
    memset(dV, 0, sizeof(double) * nV);
    int rc = OR_OK;
    for (int k = 0; k < npts && rc == OR_OK; ++k) {
        rc = surface_bwd(p, q, nu_c, nv_c, 1, 1, P, w, ku, kv, uv + 2 * (size_t)k, uv + 2 * (size_t)k + 1,
                         G + 3 * (size_t)k, tP, tW, tU, tV, local);
        for (size_t i = 0; rc == OR_OK && i < 3 * ncp; ++i) dP[i] += tP[i];
        for (size_t i = 0; rc == OR_OK && i < ncp; ++i) dW[i] += tW[i];
        for (size_t i = 0; rc == OR_OK && i < nU; ++i) dU[i] += tU[i];
        for (size_t i = 0; rc == OR_OK && i < nV; ++i) dV[i] += tV[i];
    }
    free(t);
    return rc;
}
