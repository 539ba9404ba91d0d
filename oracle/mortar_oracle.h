/*
 * Plain FP64 CPU oracle for the sliding-mesh mortar interface operator of
 * Duerrwaechter, Kurz, Kopper, Kempf, Munz, Beck, "An Efficient Sliding Mesh
 * Interface Method for High-Order Discontinuous Galerkin Schemes" (arXiv 2008.04356).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes or
 * calls this code; only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark use it.  It shares no code with the GPU path.
 *
 * Conventions (shared with the public C API only as a data layout, not as code):
 *   NP = N+1 nodes per direction, P = NP*NP points per face, point p = p_par + NP*p_perp.
 *   Face arrays are structure-of-arrays  U[var][P][n_face]  (5 conservative vars),
 *   gradients G[dir][var][P][n_face]  (3 x 5), metrics M[4][P][n_face] = (nx, ny, nz, dS).
 *   face_id[i_perp*n_par + i_par] gives the column of face (i_par, i_perp).
 *   Positions along the sliding direction are measured in face lengths l_par.
 */
#ifndef MORTAR_ORACLE_H
#define MORTAR_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_GAUSS = 0, ORC_LGL = 1 };
enum { ORC_EULER = 0, ORC_NS = 1 };
/* ORC_AVG is a test-only "flux": the arithmetic mean of both mortar states
 * (linear, so projection exactness can be checked through the whole operator).
 * ORC_ROE_NOFIX is Roe's flux without the entropy fix (test reference only).
 * ORC_LIFT + d (d = 0, 1, 2) is the BR1 lifting surface flux of the first Bassi-Rebay
 * method (Sec. 2): the mean of both states times normal component d and dS. */
enum { ORC_LF = 0, ORC_ROE = 1, ORC_ROE_NOFIX = 2, ORC_AVG = 99, ORC_LIFT = 100 };

typedef struct {
    int N;                 /* polynomial degree */
    int node_set;          /* ORC_GAUSS or ORC_LGL */
    int n_par, n_perp;     /* faces per side along / across the sliding direction */
    const int32_t *face_id_static;  /* [n_perp*n_par] column in the static arrays */
    const int32_t *face_id_moving;  /* [n_perp*n_par] column in the moving arrays */
    int n_face_static, n_face_moving;  /* column counts of the caller's arrays */
    int physics, riemann;
    double gamma, mu, Pr;
    double normal[3];      /* constant unit normal (static side), used if metrics == NULL */
    double dS;             /* constant surface element per reference area, if metrics == NULL */
    const double *metrics; /* optional [4][P][n_face_static] static-side (nx, ny, nz, dS) */
} orc_iface;

/* 1D node sets (ascending) and quadrature weights. 0 on success. */
int orc_nodes(int N, int node_set, double *x, double *w);
/* Gauss-Legendre rule with q points (used for exact integrals). */
int orc_gauss_rule(int q, double *x, double *w);
/* Lagrange basis polynomial l_j of the node set x[0..N] evaluated at xi. */
double orc_lagrange(int N, const double *x, int j, double xi);

/* Displacement Delta -> (n, s), Delta = (n + s) l_par. */
void orc_decompose(double delta, double l_par, int64_t *n, double *s);

/* Pairing: moving face index of mortar (i_par, i_sub), by brute-force interval containment. */
int orc_pair_bruteforce(int n_par, int64_t n, double s, int i_par, int i_sub);
/* Pairing by the index relation of the paper (with periodic wrap). */
int orc_pair_relation(int n_par, int64_t n, int i_par, int i_sub);

/* Matrix form of the projections, by quadrature of the defining integrals.
 * Matrices are row-major [NP][NP].  Order k: 0 = static i_sub 0, 1 = static i_sub 1,
 * 2 = moving i_sub 0 (upper part of the moving face), 3 = moving i_sub 1 (lower part).
 * M: mass matrix, S[k]: S_ij = int l_i(xi_k(z)) l_j(z) dz, Pf[k] = M^-1 S^T (face->mortar),
 * Pb[k] = J_k M^-1 S (mortar->face), J[k] = sub-interval fraction. */
int orc_projection_matrices(int N, int node_set, double s, double *M, double *S,
                            double *Pf, double *Pb, double *J);

/* Point flux: F = [Fc*(UL,UR;n) - 1/2 (Fv(UL,gL) + Fv(UR,gR)).n] * dS.
 * gL/gR are [3][5] (dir-major) conservative gradients, ignored for Euler. */
void orc_point_flux(const double *UL, const double *UR, const double *gL, const double *gR,
                    const double *nrm, double dS, int physics, int riemann,
                    double gamma, double mu, double Pr, double *F);
/* Physical normal fluxes (for tests). */
void orc_euler_normal_flux(const double *U, const double *nrm, double gamma, double *F);
void orc_viscous_normal_flux(const double *U, const double *g, const double *nrm,
                             double gamma, double mu, double Pr, double *F);

/* Full operator for one interface over rows [row0, row1).  Writes the rows'
 * faces of Fs (static columns) and Fm (moving columns); other columns untouched.
 * Gs/Gm may be NULL for Euler.  Returns 0, or a negative code on a pairing
 * inconsistency / bad input. */
int orc_mortar_flux(const orc_iface *d, int64_t n, double s,
                    const double *Us, const double *Um, const double *Gs, const double *Gm,
                    double *Fs, double *Fm, int row0, int row1);

/* Mortar sort: tuples[count][5] = (owner, i_par, i_perp, i_sub, i_face); sorted
 * nestedly by the first four entries (i_face carried passively).  A is [5][count]
 * (row-major), m is [2][m_cols] with m[i_sub][i_face - m_col0] = 0-based column of A
 * (entries not hit are set to -1). */
int orc_sort_mortars(int count, const int32_t *tuples, int32_t *A, int32_t *m,
                     int m_col0, int m_cols);
/* Index map of a whole interface side: side 0 = static (owner = owner of the paired
 * moving face), side 1 = moving (owner = owner of the static face of the mortar).
 * owner_opp is [n_perp*n_par] of the opposite side, or NULL (all 0). */
int orc_index_map(int side, int n_par, int n_perp, int64_t n, const int32_t *face_id,
                  int n_face, const int32_t *owner_opp, int32_t *A, int32_t *m);

/* Conservation sums: for each var, out[v*3+0] = sum over static faces and points of
 * w_par w_perp Fs, out[v*3+1] = the same over moving faces, out[v*3+2] = sum of |terms|
 * of both sides.  Compensated (Neumaier) summation. */
void orc_conservation(const orc_iface *d, const double *Fs, const double *Fm, double *out);

#ifdef __cplusplus
}
#endif
#endif
