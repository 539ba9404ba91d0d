/*
 * Plain FP64 CPU oracle for the sliding-mesh mortar interface operator of
 * arXiv 2008.04356 ("An Efficient Sliding Mesh Interface Method for High-Order
 * Discontinuous Galerkin Schemes").
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU-baseline
 * leg of the benchmark.  The GPU library neither links nor calls it, and the two
 * share no code (no headers, helpers, tables or generators).
 *
 * The oracle follows the plain definitions that the method's matrix operators reach:
 *   - mortar states are the face polynomials EVALUATED at the mortar nodes (the L2
 *     projection onto a same-degree mortar is exact, Sec. 3.2 "Projection Domain ->
 *     Mortar");
 *   - fluxes are pointwise Riemann + BR1 viscous fluxes (Sec. 2 and 3.1);
 *   - face fluxes are DIRECT L2 projections of the piecewise mortar-flux polynomials,
 *     integrated with a (2N+2)-point Gauss rule on every overlap interval and solved
 *     with the exact mass matrix (Sec. 3.2 "Projection Mortar -> Domain");
 *   - the static/moving pairing is found by brute-force interval containment and
 *     checked against the index relation (Sec. 4.3);
 *   - the mortar order is a plain nested sort (Sec. 4.4, Appendix A).
 * Positions along the sliding direction are kept relative to a nearby integer face
 * boundary so that large face counts do not cost precision.
 *
 * Where the paper is silent or garbled this code takes one reading each: the node set
 * is a parameter, the sub-intervals are named by their position on the face, the Roe
 * solver carries the Harten-Hyman fix on the acoustic fields only, BR1 uses gradients
 * of the conservative variables, a sliding interface has no grid-velocity term, and
 * per-point metrics (curved interfaces, Fig. of interface shapes) give the flux the
 * static side's interpolated normal scaled to unit length and its interpolated surface
 * element.
 *
 * Compiled with -ffp-contract=off: every product and sum is rounded as written.
 */
#include "mortar_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAXN 16
#define ORC_MAXQ (2 * ORC_MAXN + 2)

/* ------------------------------------------------------------------------- */
/* Legendre polynomials and node sets (Sec. 3.1: Legendre-Gauss and          */
/* Legendre-Gauss-Lobatto points).                                           */
/* ------------------------------------------------------------------------- */

/* P_n(x), P_n'(x), P_n''(x) by the three-term recurrence and its derivatives. */
static void legendre(int n, double x, double *P, double *dP, double *d2P)
{
    double p0 = 1.0, d0 = 0.0, s0 = 0.0;  /* P_{k-1} and derivatives */
    double p1 = x, d1 = 1.0, s1 = 0.0;    /* P_k */
    if (n == 0) {
        *P = 1.0; *dP = 0.0; *d2P = 0.0;
        return;
    }
    for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        double d2 = x * d1 + k * p1;          /* P_k' = x P_{k-1}' + k P_{k-1} */
        double s2 = x * s1 + (k + 1.0) * d1;  /* derivative of the line above */
        p0 = p1; d0 = d1; s0 = s1;
        p1 = p2; d1 = d2; s1 = s2;
    }
    (void)d0; (void)s0;
    *P = p1; *dP = d1; *d2P = s1;
}

int orc_gauss_rule(int q, double *x, double *w)
{
    if (q < 1 || q > ORC_MAXQ) return -1;
    for (int i = 0; i < q; ++i) {
        /* Newton iteration for the i-th root of P_q from a Chebyshev-like guess. */
        double r = cos(M_PI * (i + 0.75) / (q + 0.5));
        double P, dP, d2P;
        for (int it = 0; it < 100; ++it) {
            legendre(q, r, &P, &dP, &d2P);
            double dr = P / dP;
            r -= dr;
            if (fabs(dr) < 1e-17) break;
        }
        legendre(q, r, &P, &dP, &d2P);
        x[q - 1 - i] = r;
        w[q - 1 - i] = 2.0 / ((1.0 - r * r) * dP * dP);
    }
    return 0;
}

int orc_nodes(int N, int node_set, double *x, double *w)
{
    if (N < 1 || N >= ORC_MAXN) return -1;
    if (node_set == ORC_GAUSS) return orc_gauss_rule(N + 1, x, w);
    if (node_set != ORC_LGL) return -1;
    /* LGL: the end points and the roots of P_N'; weights 2 / (N(N+1) P_N(x)^2). */
    x[0] = -1.0;
    x[N] = 1.0;
    for (int i = 1; i < N; ++i) {
        double r = cos(M_PI * i / N);
        double P, dP, d2P;
        for (int it = 0; it < 100; ++it) {
            legendre(N, r, &P, &dP, &d2P);
            double dr = dP / d2P;
            r -= dr;
            if (fabs(dr) < 1e-17) break;
        }
        x[N - i] = r;
    }
    for (int i = 0; i <= N; ++i) {
        double P, dP, d2P;
        legendre(N, x[i], &P, &dP, &d2P);
        w[i] = 2.0 / (N * (N + 1.0) * P * P);
    }
    return 0;
}

/* Lagrange basis l_j of the nodes x[0..N], product form (Sec. 3.1 cardinal property). */
double orc_lagrange(int N, const double *x, int j, double xi)
{
    double v = 1.0;
    for (int m = 0; m <= N; ++m)
        if (m != j) v *= (xi - x[m]) / (x[j] - x[m]);
    return v;
}

/* ------------------------------------------------------------------------- */
/* Displacement and pairing (Sec. 4.3).                                      */
/* ------------------------------------------------------------------------- */

void orc_decompose(double delta, double l_par, int64_t *n, double *s)
{
    /* Delta = (n + s) l_par with n integer and s in [0,1). */
    double q = delta / l_par;
    double fl = floor(q);
    double f = q - fl;
    int64_t nn = (int64_t)fl;
    if (f >= 1.0) { f -= 1.0; nn += 1; }
    if (f < 0.0 || f == 0.0) f = 0.0; /* also turns -0.0 into +0.0 */
    *n = nn;
    *s = f;
}

static int64_t mod_pos(int64_t a, int64_t m)
{
    int64_t r = a % m;
    return r < 0 ? r + m : r;
}

int orc_pair_relation(int n_par, int64_t n, int i_par, int i_sub)
{
    /* moving index = static index - n + i_sub - 1, wrapped periodically */
    return (int)mod_pos((int64_t)i_par - mod_pos(n, n_par) + i_sub - 1, n_par);
}

/* Mortar (i, k) spans [i + oa, i + ob] (face lengths) with oa, ob below. */
static void mortar_offsets(int k, double s, double *oa, double *ob)
{
    /* i_sub = 0: the part of the static face below the hanging node (Eq. for i_sub). */
    if (k == 0) { *oa = 0.0; *ob = s; }
    else        { *oa = s;   *ob = 1.0; }
}

/* Brute force: every moving face jt, in the periodic images -1, 0, +1, spans
 * [base + s, base + 1 + s] with base = jt + (n mod n_par) + image*n_par.  The face that
 * contains the mortar is returned, with rel = i - base (small integer) so that local
 * coordinates can be formed without large numbers.  A zero-length mortar touches two
 * faces: i_sub = 0 lies at the upper end of its moving face, i_sub = 1 at the lower end. */
static int pair_full(int n_par, int64_t n, double s, int i, int k, int64_t *rel_out)
{
    int64_t nm = mod_pos(n, n_par);
    double oa, ob;
    mortar_offsets(k, s, &oa, &ob);
    int cand_jt[16];
    int64_t cand_rel[16];
    int nc = 0;
    for (int jt = 0; jt < n_par; ++jt) {
        for (int img = -1; img <= 1; ++img) {
            int64_t base = jt + nm + (int64_t)img * n_par;
            int64_t rel = (int64_t)i - base;
            if (rel < -2 || rel > 2) continue; /* far away: cannot contain the mortar */
            double a = (double)rel + oa, b = (double)rel + ob;
            if (a >= s && b <= 1.0 + s && nc < 16) {
                cand_jt[nc] = jt;
                cand_rel[nc] = rel;
                nc++;
            }
        }
    }
    int pick = -1;
    if (nc == 1) {
        pick = 0;
    } else if (nc > 1) {
        /* only a zero-length mortar touches two faces; i_sub = 0 sits at the upper
         * end of its moving face, i_sub = 1 at the lower end */
        for (int c = 0; c < nc; ++c) {
            double a = (double)cand_rel[c] + oa, b = (double)cand_rel[c] + ob;
            if (a != b) return -1;
            if ((k == 0 && b == 1.0 + s) || (k == 1 && a == s)) pick = c;
        }
    }
    if (pick < 0) return -1;
    if (rel_out) *rel_out = cand_rel[pick];
    return cand_jt[pick];
}

int orc_pair_bruteforce(int n_par, int64_t n, double s, int i_par, int i_sub)
{
    return pair_full(n_par, n, s, i_par, i_sub, NULL);
}

/* ------------------------------------------------------------------------- */
/* Small dense linear algebra (plain).                                       */
/* ------------------------------------------------------------------------- */

static int invert(int n, const double *A, double *Ainv)
{
    double a[ORC_MAXN * ORC_MAXN * 2];
    int w = 2 * n;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            a[i * w + j] = A[i * n + j];
            a[i * w + n + j] = (i == j) ? 1.0 : 0.0;
        }
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (fabs(a[r * w + c]) > fabs(a[piv * w + c])) piv = r;
        if (a[piv * w + c] == 0.0) return -1;
        if (piv != c)
            for (int j = 0; j < w; ++j) {
                double t = a[c * w + j]; a[c * w + j] = a[piv * w + j]; a[piv * w + j] = t;
            }
        double d = a[c * w + c];
        for (int j = 0; j < w; ++j) a[c * w + j] /= d;
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            double f = a[r * w + c];
            if (f != 0.0)
                for (int j = 0; j < w; ++j) a[r * w + j] -= f * a[c * w + j];
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Ainv[i * n + j] = a[i * w + n + j];
    return 0;
}

/* Cholesky factor L (lower) of a symmetric positive definite matrix. */
static int cholesky(int n, const double *A, double *L)
{
    memset(L, 0, sizeof(double) * n * n);
    for (int j = 0; j < n; ++j) {
        double d = A[j * n + j];
        for (int k = 0; k < j; ++k) d -= L[j * n + k] * L[j * n + k];
        if (d <= 0.0) return -1;
        L[j * n + j] = sqrt(d);
        for (int i = j + 1; i < n; ++i) {
            double v = A[i * n + j];
            for (int k = 0; k < j; ++k) v -= L[i * n + k] * L[j * n + k];
            L[i * n + j] = v / L[j * n + j];
        }
    }
    return 0;
}

static void cholesky_solve(int n, const double *L, const double *b, double *x)
{
    double y[ORC_MAXN];
    for (int i = 0; i < n; ++i) {
        double v = b[i];
        for (int k = 0; k < i; ++k) v -= L[i * n + k] * y[k];
        y[i] = v / L[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double v = y[i];
        for (int k = i + 1; k < n; ++k) v -= L[k * n + i] * x[k];
        x[i] = v / L[i * n + i];
    }
}

/* Mass matrix M_ij = int_{-1}^{1} l_i l_j, by a (2N+2)-point Gauss rule (exact). */
static int mass_matrix(int N, const double *x, double *M)
{
    int NP = N + 1, Q = 2 * N + 2;
    double t[ORC_MAXQ], wt[ORC_MAXQ];
    if (orc_gauss_rule(Q, t, wt)) return -1;
    for (int i = 0; i < NP; ++i)
        for (int j = 0; j < NP; ++j) {
            double v = 0.0;
            for (int r = 0; r < Q; ++r)
                v += wt[r] * orc_lagrange(N, x, i, t[r]) * orc_lagrange(N, x, j, t[r]);
            M[i * NP + j] = v;
        }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Matrix form (Eqs. for M, S, face->mortar and mortar->face projections).   */
/* ------------------------------------------------------------------------- */

int orc_projection_matrices(int N, int node_set, double s, double *M, double *S,
                            double *Pf, double *Pb, double *J)
{
    int NP = N + 1, Q = 2 * N + 2;
    double x[ORC_MAXN], w[ORC_MAXN], t[ORC_MAXQ], wt[ORC_MAXQ], Minv[ORC_MAXN * ORC_MAXN];
    if (orc_nodes(N, node_set, x, w)) return -1;
    if (orc_gauss_rule(Q, t, wt)) return -1;
    if (mass_matrix(N, x, M)) return -1;
    if (invert(NP, M, Minv)) return -2;
    /* Sub-interval k in the face coordinate: xi = lower + (z + 1) * frac. */
    double lower[4] = {-1.0, -1.0 + 2.0 * s, 1.0 - 2.0 * s, -1.0};
    double frac[4] = {s, 1.0 - s, s, 1.0 - s};
    for (int k = 0; k < 4; ++k) {
        double *Sk = S + k * NP * NP, *Pfk = Pf + k * NP * NP, *Pbk = Pb + k * NP * NP;
        J[k] = frac[k];
        for (int i = 0; i < NP; ++i)
            for (int j = 0; j < NP; ++j) {
                double v = 0.0;
                for (int r = 0; r < Q; ++r) {
                    double xi = lower[k] + (t[r] + 1.0) * frac[k];
                    v += wt[r] * orc_lagrange(N, x, i, xi) * orc_lagrange(N, x, j, t[r]);
                }
                Sk[i * NP + j] = v;
            }
        /* face -> mortar: M Qhat = S^T Uhat */
        for (int q = 0; q < NP; ++q)
            for (int i = 0; i < NP; ++i) {
                double v = 0.0;
                for (int j = 0; j < NP; ++j) v += Minv[q * NP + j] * Sk[i * NP + j];
                Pfk[q * NP + i] = v;
            }
        /* mortar -> face: M Fhat = J S Fhat_mortar */
        for (int j = 0; j < NP; ++j)
            for (int q = 0; q < NP; ++q) {
                double v = 0.0;
                for (int i = 0; i < NP; ++i) v += Minv[j * NP + i] * Sk[i * NP + q];
                Pbk[j * NP + q] = frac[k] * v;
            }
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Fluxes (Sec. 2 equations; Roe solver with Harten-Hyman fix, Sec. 3.1).    */
/* ------------------------------------------------------------------------- */

static void primitive(const double *U, double gamma, double *rho, double *v, double *p)
{
    *rho = U[0];
    v[0] = U[1] / U[0];
    v[1] = U[2] / U[0];
    v[2] = U[3] / U[0];
    *p = (gamma - 1.0) * (U[4] - 0.5 * U[0] * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]));
}

void orc_euler_normal_flux(const double *U, const double *nrm, double gamma, double *F)
{
    double rho, v[3], p;
    primitive(U, gamma, &rho, v, &p);
    double vn = v[0] * nrm[0] + v[1] * nrm[1] + v[2] * nrm[2];
    F[0] = rho * vn;
    F[1] = U[1] * vn + p * nrm[0];
    F[2] = U[2] * vn + p * nrm[1];
    F[3] = U[3] * vn + p * nrm[2];
    F[4] = (U[4] + p) * vn;
}

static void flux_lf(const double *UL, const double *UR, const double *nrm, double gamma, double *F)
{
    double FL[5], FR[5], rL, vL[3], pL, rR, vR[3], pR;
    orc_euler_normal_flux(UL, nrm, gamma, FL);
    orc_euler_normal_flux(UR, nrm, gamma, FR);
    primitive(UL, gamma, &rL, vL, &pL);
    primitive(UR, gamma, &rR, vR, &pR);
    double vnL = vL[0] * nrm[0] + vL[1] * nrm[1] + vL[2] * nrm[2];
    double vnR = vR[0] * nrm[0] + vR[1] * nrm[1] + vR[2] * nrm[2];
    double lamL = fabs(vnL) + sqrt(gamma * pL / rL);
    double lamR = fabs(vnR) + sqrt(gamma * pR / rR);
    double lam = lamL > lamR ? lamL : lamR;
    for (int v = 0; v < 5; ++v) F[v] = 0.5 * (FL[v] + FR[v]) - 0.5 * lam * (UR[v] - UL[v]);
}

/* Harten-Hyman adjusted modulus of an acoustic eigenvalue. */
static double hh_abs(double lam, double lamL, double lamR)
{
    double d = 0.0;
    if (lam - lamL > d) d = lam - lamL;
    if (lamR - lam > d) d = lamR - lam;
    double a = fabs(lam);
    if (a < d) a = 0.5 * (lam * lam / d + d);
    return a;
}

static void flux_roe(const double *UL, const double *UR, const double *nrm, double gamma,
                     int entropy_fix, double *F)
{
    double FL[5], FR[5], rL, vL[3], pL, rR, vR[3], pR;
    orc_euler_normal_flux(UL, nrm, gamma, FL);
    orc_euler_normal_flux(UR, nrm, gamma, FR);
    primitive(UL, gamma, &rL, vL, &pL);
    primitive(UR, gamma, &rR, vR, &pR);
    double HL = (UL[4] + pL) / rL, HR = (UR[4] + pR) / rR;
    double sL = sqrt(rL), sR = sqrt(rR);
    double u[3];
    for (int d = 0; d < 3; ++d) u[d] = (sL * vL[d] + sR * vR[d]) / (sL + sR);
    double H = (sL * HL + sR * HR) / (sL + sR);
    double q2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    double c = sqrt((gamma - 1.0) * (H - 0.5 * q2));
    double rho = sL * sR;
    double un = u[0] * nrm[0] + u[1] * nrm[1] + u[2] * nrm[2];
    double vnL = vL[0] * nrm[0] + vL[1] * nrm[1] + vL[2] * nrm[2];
    double vnR = vR[0] * nrm[0] + vR[1] * nrm[1] + vR[2] * nrm[2];
    double cL = sqrt(gamma * pL / rL), cR = sqrt(gamma * pR / rR);

    double drho = rR - rL, dp = pR - pL, dv[3];
    for (int d = 0; d < 3; ++d) dv[d] = vR[d] - vL[d];
    double dvn = dv[0] * nrm[0] + dv[1] * nrm[1] + dv[2] * nrm[2];

    /* wave strengths: two acoustic waves, entropy wave, shear (tangential velocity jump) */
    double a1 = (dp - rho * c * dvn) / (2.0 * c * c);
    double a5 = (dp + rho * c * dvn) / (2.0 * c * c);
    double a2 = drho - dp / (c * c);

    double l1 = entropy_fix ? hh_abs(un - c, vnL - cL, vnR - cR) : fabs(un - c);
    double l2 = fabs(un);
    double l5 = entropy_fix ? hh_abs(un + c, vnL + cL, vnR + cR) : fabs(un + c);

    double D[5];
    /* acoustic wave u - c */
    D[0] = l1 * a1;
    for (int d = 0; d < 3; ++d) D[1 + d] = l1 * a1 * (u[d] - c * nrm[d]);
    D[4] = l1 * a1 * (H - un * c);
    /* acoustic wave u + c */
    D[0] += l5 * a5;
    for (int d = 0; d < 3; ++d) D[1 + d] += l5 * a5 * (u[d] + c * nrm[d]);
    D[4] += l5 * a5 * (H + un * c);
    /* entropy wave */
    D[0] += l2 * a2;
    for (int d = 0; d < 3; ++d) D[1 + d] += l2 * a2 * u[d];
    D[4] += l2 * a2 * 0.5 * q2;
    /* shear waves: rho * (tangential velocity jump) */
    double dvt[3];
    for (int d = 0; d < 3; ++d) dvt[d] = dv[d] - dvn * nrm[d];
    for (int d = 0; d < 3; ++d) D[1 + d] += l2 * rho * dvt[d];
    D[4] += l2 * rho * (u[0] * dvt[0] + u[1] * dvt[1] + u[2] * dvt[2]);

    for (int v = 0; v < 5; ++v) F[v] = 0.5 * (FL[v] + FR[v]) - 0.5 * D[v];
}

void orc_viscous_normal_flux(const double *U, const double *g, const double *nrm,
                             double gamma, double mu, double Pr, double *F)
{
    /* g[d*5 + v] = d U_v / d x_d (conservative variables). */
    double rho, v[3], p;
    primitive(U, gamma, &rho, v, &p);
    double gv[3][3]; /* gv[i][d] = d v_i / d x_d */
    double gp[3];
    double vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    for (int d = 0; d < 3; ++d) {
        const double *gd = g + d * 5;
        for (int i = 0; i < 3; ++i) gv[i][d] = (gd[1 + i] - v[i] * gd[0]) / rho;
        gp[d] = (gamma - 1.0) * (gd[4] - (v[0] * gd[1] + v[1] * gd[2] + v[2] * gd[3]) + 0.5 * vv * gd[0]);
    }
    double div = gv[0][0] + gv[1][1] + gv[2][2];
    double tau[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            tau[i][j] = mu * (gv[i][j] + gv[j][i]) + ((i == j) ? (-2.0 / 3.0) * mu * div : 0.0);
    /* heat flux q = -k grad T, k = mu cp / Pr, T = p / (rho R): the gas constant cancels. */
    double kfac = mu * gamma / ((gamma - 1.0) * Pr);
    double q[3];
    for (int d = 0; d < 3; ++d) q[d] = -kfac * (gp[d] - (p / rho) * g[d * 5 + 0]) / rho;
    F[0] = 0.0;
    for (int i = 0; i < 3; ++i)
        F[1 + i] = tau[i][0] * nrm[0] + tau[i][1] * nrm[1] + tau[i][2] * nrm[2];
    double e = 0.0;
    for (int i = 0; i < 3; ++i) {
        double ti = tau[i][0] * v[0] + tau[i][1] * v[1] + tau[i][2] * v[2] - q[i];
        e += ti * nrm[i];
    }
    F[4] = e;
}

void orc_point_flux(const double *UL, const double *UR, const double *gL, const double *gR,
                    const double *nrm, double dS, int physics, int riemann,
                    double gamma, double mu, double Pr, double *F)
{
    double Fc[5];
    if (riemann == ORC_AVG) {
        for (int v = 0; v < 5; ++v) F[v] = 0.5 * (UL[v] + UR[v]) * dS;
        return;
    }
    if (riemann >= ORC_LIFT && riemann < ORC_LIFT + 3) {
        /* BR1 lifting (Sec. 2): U* = (U_L + U_R)/2, component d of U* n dS */
        const double nd = nrm[riemann - ORC_LIFT];
        for (int v = 0; v < 5; ++v) F[v] = 0.5 * (UL[v] + UR[v]) * nd * dS;
        return;
    }
    if (riemann == ORC_LF) flux_lf(UL, UR, nrm, gamma, Fc);
    else flux_roe(UL, UR, nrm, gamma, riemann != ORC_ROE_NOFIX, Fc);
    if (physics == ORC_NS) {
        double FvL[5], FvR[5];
        orc_viscous_normal_flux(UL, gL, nrm, gamma, mu, Pr, FvL);
        orc_viscous_normal_flux(UR, gR, nrm, gamma, mu, Pr, FvR);
        for (int v = 0; v < 5; ++v) Fc[v] -= 0.5 * (FvL[v] + FvR[v]);
    }
    for (int v = 0; v < 5; ++v) F[v] = Fc[v] * dS;
}

/* ------------------------------------------------------------------------- */
/* The operator (Sec. 3.3, five steps).                                      */
/* ------------------------------------------------------------------------- */

typedef struct {
    int jt;        /* paired moving face */
    int64_t rel;   /* i - base of the moving face image */
    double oa, ob; /* mortar span relative to its static face start */
} mortar_info;

typedef struct {
    int i, k;      /* static face and sub index of the overlapping mortar */
    double c, d;   /* overlap, relative to the moving face image base */
    double ma, mb; /* mortar span, relative to the same base */
    int64_t rel;   /* i - base */
} overlap_info;

int orc_mortar_flux(const orc_iface *dsc, int64_t n, double s,
                    const double *Us, const double *Um, const double *Gs, const double *Gm,
                    double *Fs, double *Fm, int row0, int row1)
{
    const int N = dsc->N, NP = N + 1, P = NP * NP, Q = 2 * N + 2;
    const int np = dsc->n_par;
    const int ns_ = dsc->n_face_static, nm_ = dsc->n_face_moving;
    const int ns_visc = (dsc->physics == ORC_NS);
    double x[ORC_MAXN], w[ORC_MAXN], t[ORC_MAXQ], wt[ORC_MAXQ];
    double M[ORC_MAXN * ORC_MAXN], L[ORC_MAXN * ORC_MAXN];
    if (N < 1 || N >= ORC_MAXN || np < 1) return -1;
    if (s < 0.0 || s >= 1.0) return -1;
    if (orc_nodes(N, dsc->node_set, x, w)) return -1;
    if (orc_gauss_rule(Q, t, wt)) return -1;
    if (mass_matrix(N, x, M) || cholesky(NP, M, L)) return -1;
    if (ns_visc && (!Gs || !Gm)) return -1;

    mortar_info *mi = (mortar_info *)malloc(sizeof(mortar_info) * 2 * np);
    overlap_info *ov = (overlap_info *)malloc(sizeof(overlap_info) * 8 * np);
    int *ov_start = (int *)malloc(sizeof(int) * (np + 1));
    double *Fmort = (double *)malloc(sizeof(double) * 2 * np * NP * 5);
    int rc = 0;
    if (!mi || !ov || !ov_start || !Fmort) { rc = -3; goto done; }

    /* Step 1: dynamic definition of the interface (the same for every row). */
    for (int i = 0; i < np; ++i)
        for (int k = 0; k < 2; ++k) {
            mortar_info *m = &mi[2 * i + k];
            mortar_offsets(k, s, &m->oa, &m->ob);
            m->jt = pair_full(np, n, s, i, k, &m->rel);
            if (m->jt < 0 || m->jt != orc_pair_relation(np, n, i, k)) { rc = -2; goto done; }
        }
    /* Overlaps of every moving face with the mortars (brute force over all mortars
     * and the periodic images); zero-length overlaps contribute nothing. */
    {
        int64_t nm = mod_pos(n, np);
        int cnt = 0;
        for (int jt = 0; jt < np; ++jt) {
            ov_start[jt] = cnt;
            for (int img = -1; img <= 1; ++img) {
                int64_t base = jt + nm + (int64_t)img * np;
                for (int i = 0; i < np; ++i) {
                    int64_t rel = (int64_t)i - base;
                    if (rel < -2 || rel > 2) continue;
                    for (int k = 0; k < 2; ++k) {
                        double a = (double)rel + mi[2 * i + k].oa;
                        double b = (double)rel + mi[2 * i + k].ob;
                        double c = a > s ? a : s;
                        double d = b < 1.0 + s ? b : 1.0 + s;
                        if (d > c && b > a) {
                            if (cnt >= 8 * np) { rc = -2; goto done; }
                            overlap_info *o = &ov[cnt++];
                            o->i = i; o->k = k; o->c = c; o->d = d;
                            o->ma = a; o->mb = b; o->rel = rel;
                        }
                    }
                }
            }
        }
        ov_start[np] = cnt;
    }

    for (int row = row0; row < row1; ++row) {
        const int32_t *fid_s = dsc->face_id_static + (int64_t)row * np;
        const int32_t *fid_m = dsc->face_id_moving + (int64_t)row * np;
        for (int pp = 0; pp < NP; ++pp) {
            /* Steps 2-4: mortar states by evaluation of both face polynomials at the
             * mortar nodes, then the Riemann + viscous flux at every mortar node. */
            for (int i = 0; i < np; ++i)
                for (int k = 0; k < 2; ++k) {
                    const mortar_info *m = &mi[2 * i + k];
                    int cs = fid_s[i], cm = fid_m[m->jt];
                    for (int q = 0; q < NP; ++q) {
                        double xrel = m->oa + 0.5 * (x[q] + 1.0) * (m->ob - m->oa); /* X - i */
                        double xi_s = -1.0 + 2.0 * xrel;
                        /* moving image base = i - rel; its face spans [s, 1 + s] from there */
                        double xi_m = -1.0 + 2.0 * ((xrel + (double)m->rel) - s);
                        double ls[ORC_MAXN], lm[ORC_MAXN];
                        for (int j = 0; j < NP; ++j) {
                            ls[j] = orc_lagrange(N, x, j, xi_s);
                            lm[j] = orc_lagrange(N, x, j, xi_m);
                        }
                        double UL[5], UR[5], gL[15], gR[15], nrm[3], dS;
                        for (int v = 0; v < 5; ++v) {
                            double a = 0.0, b = 0.0;
                            for (int j = 0; j < NP; ++j) {
                                int p = j + NP * pp;
                                a += Us[((int64_t)v * P + p) * ns_ + cs] * ls[j];
                                b += Um[((int64_t)v * P + p) * nm_ + cm] * lm[j];
                            }
                            UL[v] = a; UR[v] = b;
                        }
                        if (ns_visc)
                            for (int g = 0; g < 15; ++g) {
                                double a = 0.0, b = 0.0;
                                for (int j = 0; j < NP; ++j) {
                                    int p = j + NP * pp;
                                    a += Gs[((int64_t)g * P + p) * ns_ + cs] * ls[j];
                                    b += Gm[((int64_t)g * P + p) * nm_ + cm] * lm[j];
                                }
                                gL[g] = a; gR[g] = b;
                            }
                        if (dsc->metrics) {
                            double mv[4];
                            for (int c = 0; c < 4; ++c) {
                                double a = 0.0;
                                for (int j = 0; j < NP; ++j)
                                    a += dsc->metrics[((int64_t)c * P + j + NP * pp) * ns_ + cs] * ls[j];
                                mv[c] = a;
                            }
                            /* On a curved face the interpolant of unit nodal normals is
                             * shorter than one between the nodes: the flux takes the
                             * interpolated direction, scaled to unit length, and the
                             * interpolated surface element. */
                            double len = sqrt(mv[0] * mv[0] + mv[1] * mv[1] + mv[2] * mv[2]);
                            nrm[0] = mv[0] / len; nrm[1] = mv[1] / len; nrm[2] = mv[2] / len;
                            dS = mv[3];
                        } else {
                            nrm[0] = dsc->normal[0]; nrm[1] = dsc->normal[1]; nrm[2] = dsc->normal[2];
                            dS = dsc->dS;
                        }
                        orc_point_flux(UL, UR, gL, gR, nrm, dS, dsc->physics, dsc->riemann,
                                       dsc->gamma, dsc->mu, dsc->Pr,
                                       Fmort + ((int64_t)(2 * i + k) * NP + q) * 5);
                    }
                }
            /* Step 5, static side: L2 projection of the two mortar fluxes onto face i. */
            for (int i = 0; i < np; ++i) {
                double b[5][ORC_MAXN];
                memset(b, 0, sizeof(b));
                for (int k = 0; k < 2; ++k) {
                    const mortar_info *m = &mi[2 * i + k];
                    double len = m->ob - m->oa;
                    if (!(len > 0.0)) continue;
                    const double *Fk = Fmort + (int64_t)(2 * i + k) * NP * 5;
                    for (int r = 0; r < Q; ++r) {
                        double xrel = m->oa + 0.5 * (t[r] + 1.0) * len;
                        double z = -1.0 + 2.0 * (xrel - m->oa) / len;
                        double xi = -1.0 + 2.0 * xrel;
                        double wgt = wt[r] * len; /* d xi = 2 d X, d X = len/2 d t */
                        double fz[5] = {0, 0, 0, 0, 0};
                        for (int q = 0; q < NP; ++q) {
                            double lq = orc_lagrange(N, x, q, z);
                            for (int v = 0; v < 5; ++v) fz[v] += Fk[q * 5 + v] * lq;
                        }
                        for (int j = 0; j < NP; ++j) {
                            double lj = orc_lagrange(N, x, j, xi);
                            for (int v = 0; v < 5; ++v) b[v][j] += wgt * fz[v] * lj;
                        }
                    }
                }
                for (int v = 0; v < 5; ++v) {
                    double f[ORC_MAXN];
                    cholesky_solve(NP, L, b[v], f);
                    for (int j = 0; j < NP; ++j)
                        Fs[((int64_t)v * P + j + NP * pp) * ns_ + fid_s[i]] = f[j];
                }
            }
            /* Step 5, moving side: L2 projection of every overlapping mortar flux. */
            for (int jt = 0; jt < np; ++jt) {
                double b[5][ORC_MAXN];
                memset(b, 0, sizeof(b));
                for (int e = ov_start[jt]; e < ov_start[jt + 1]; ++e) {
                    const overlap_info *o = &ov[e];
                    const double *Fk = Fmort + (int64_t)(2 * o->i + o->k) * NP * 5;
                    double len = o->d - o->c, mlen = o->mb - o->ma;
                    for (int r = 0; r < Q; ++r) {
                        double X = o->c + 0.5 * (t[r] + 1.0) * len; /* relative to base */
                        double z = -1.0 + 2.0 * (X - o->ma) / mlen;
                        double xi = -1.0 + 2.0 * (X - s);
                        double wgt = wt[r] * len;
                        double fz[5] = {0, 0, 0, 0, 0};
                        for (int q = 0; q < NP; ++q) {
                            double lq = orc_lagrange(N, x, q, z);
                            for (int v = 0; v < 5; ++v) fz[v] += Fk[q * 5 + v] * lq;
                        }
                        for (int j = 0; j < NP; ++j) {
                            double lj = orc_lagrange(N, x, j, xi);
                            for (int v = 0; v < 5; ++v) b[v][j] += wgt * fz[v] * lj;
                        }
                    }
                }
                for (int v = 0; v < 5; ++v) {
                    double f[ORC_MAXN];
                    cholesky_solve(NP, L, b[v], f);
                    for (int j = 0; j < NP; ++j)
                        Fm[((int64_t)v * P + j + NP * pp) * nm_ + fid_m[jt]] = f[j];
                }
            }
        }
    }
done:
    free(mi); free(ov); free(ov_start); free(Fmort);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* Mortar sorting and index mapping (Sec. 4.4, Appendix A).                  */
/* ------------------------------------------------------------------------- */

static int cmp_tuple(const void *pa, const void *pb)
{
    const int32_t *a = (const int32_t *)pa, *b = (const int32_t *)pb;
    for (int r = 0; r < 4; ++r) {
        if (a[r] < b[r]) return -1;
        if (a[r] > b[r]) return 1;
    }
    return 0;
}

int orc_sort_mortars(int count, const int32_t *tuples, int32_t *A, int32_t *m,
                     int m_col0, int m_cols)
{
    int32_t *tmp = (int32_t *)malloc(sizeof(int32_t) * 5 * (count > 0 ? count : 1));
    if (!tmp) return -3;
    memcpy(tmp, tuples, sizeof(int32_t) * 5 * count);
    qsort(tmp, count, sizeof(int32_t) * 5, cmp_tuple);
    for (int c = 1; c < count; ++c)
        if (cmp_tuple(tmp + 5 * (c - 1), tmp + 5 * c) == 0) { free(tmp); return -2; }
    for (int c = 0; c < count; ++c)
        for (int r = 0; r < 5; ++r) A[r * count + c] = tmp[5 * c + r];
    for (int i = 0; i < 2 * m_cols; ++i) m[i] = -1;
    for (int c = 0; c < count; ++c) {
        int isub = tmp[5 * c + 3], f = tmp[5 * c + 4] - m_col0;
        if (isub < 0 || isub > 1 || f < 0 || f >= m_cols) { free(tmp); return -1; }
        m[isub * m_cols + f] = c;
    }
    free(tmp);
    return 0;
}

int orc_index_map(int side, int n_par, int n_perp, int64_t n, const int32_t *face_id,
                  int n_face, const int32_t *owner_opp, int32_t *A, int32_t *m)
{
    int count = 2 * n_par * n_perp;
    int32_t *tup = (int32_t *)malloc(sizeof(int32_t) * 5 * count);
    if (!tup) return -3;
    int c = 0;
    for (int ip = 0; ip < n_perp; ++ip)
        for (int ia = 0; ia < n_par; ++ia)
            for (int k = 0; k < 2; ++k) {
                int i_static, opp_col;
                if (side == 0) {
                    /* static face ia: its mortar k pairs with the moving face of the relation */
                    i_static = ia;
                    opp_col = orc_pair_relation(n_par, n, ia, k);
                } else {
                    /* moving face ia: mortar k belongs to static face ia + n - k + 1 */
                    i_static = (int)mod_pos((int64_t)ia + mod_pos(n, n_par) - k + 1, n_par);
                    opp_col = i_static;
                }
                int32_t *t = tup + 5 * c++;
                t[0] = owner_opp ? owner_opp[(int64_t)ip * n_par + opp_col] : 0;
                t[1] = i_static;
                t[2] = ip;
                t[3] = k;
                t[4] = face_id[(int64_t)ip * n_par + ia];
            }
    int rc = orc_sort_mortars(count, tup, A, m, 0, n_face);
    free(tup);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* Conservation sums.                                                        */
/* ------------------------------------------------------------------------- */

typedef struct { double s, c; } neumaier;
static void nm_add(neumaier *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}

void orc_conservation(const orc_iface *d, const double *Fs, const double *Fm, double *out)
{
    const int N = d->N, NP = N + 1, P = NP * NP;
    double x[ORC_MAXN], w[ORC_MAXN];
    orc_nodes(N, d->node_set, x, w);
    for (int v = 0; v < 5; ++v) {
        neumaier S = {0, 0}, Mv = {0, 0}, A = {0, 0};
        for (int f = 0; f < d->n_par * d->n_perp; ++f)
            for (int p = 0; p < P; ++p) {
                double wp = w[p % NP] * w[p / NP];
                double a = wp * Fs[((int64_t)v * P + p) * d->n_face_static + d->face_id_static[f]];
                double b = wp * Fm[((int64_t)v * P + p) * d->n_face_moving + d->face_id_moving[f]];
                nm_add(&S, a);
                nm_add(&Mv, b);
                nm_add(&A, fabs(a));
                nm_add(&A, fabs(b));
            }
        out[v * 3 + 0] = S.s + S.c;
        out[v * 3 + 1] = Mv.s + Mv.c;
        out[v * 3 + 2] = A.s + A.c;
    }
}
